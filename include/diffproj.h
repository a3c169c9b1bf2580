/*
 * diffproj.h -- C ABI of the MI355X (gfx950) differentiable cone-beam
 * projector library `libdiffproj.so`.
 *
 * Method: arXiv 2508.13304, "Differentiable Forward and Back-Projector for
 * Rigid Motion Estimation in X-ray Imaging".  The library computes
 *   - the ray-driven forward projection l(d, theta) of a rigidly moved
 *     volume (Eq. forward, Sec. II-A), discretised as a trilinear march;
 *   - its pose gradient dL/dtheta given dL/dl, obtained by projecting the
 *     per-voxel matrix G_f = grad'mu^T grad_M r' with the same weights
 *     (Eqs. final_forward, for_int, dis_forward, Sec. II-B/C);
 *   - the voxel-driven back-projection mu(r', theta) (Eq. back);
 *   - its pose gradient dL/dtheta given dL/dmu, obtained by back-projecting
 *     G_b = grad_d l^T grad_r p grad_M r with the same weights
 *     (Eqs. final_back, back_int, dis_back);
 *   - the chain rule dL/dtheta = grad_theta M . dL/dM (Sec. II-B).
 *
 * Geometry (all lengths mm, angles rad):
 *   - volume voxel (i,j,k) has object-frame centre
 *       p = ((i-(nx-1)/2) vx, (j-(ny-1)/2) vy, (k-(nz-1)/2) vz);
 *     memory order [nz][ny][nx], x fastest, float32;
 *   - rigid motion theta = (tx,ty,tz,gx,gy,gz): r = R p + t with
 *     R = Rz(gz) Ry(gy) Rx(gx) (right-handed elemental rotations);
 *   - view v has gantry angle beta: source s = SAD (cos b, sin b, 0),
 *     e_w = (-cos b, -sin b, 0) (source -> isocentre), detector axes
 *     e_u = (-sin b, cos b, 0) (columns) and e_v = (0,0,1) (rows); pixel
 *     (a, b) centre = s + SDD e_w + (a-cu) du e_u + (b-cv) dv e_v with
 *     cu = (nu-1)/2 + off_u, cv = (nv-1)/2 + off_v; images [V][nv][nu];
 *   - forward: l[v][b][a] = step * sum_{k>=0} mu~(R^T(s + k step u_ab - t)),
 *     mu~ the zero-extended trilinear interpolant, u_ab the unit direction
 *     from the source to the pixel centre;
 *   - back: mu[j] = sum_v W_v(j) l~_v(p_v(R_v p_j + t_v)), l~ the
 *     zero-extended bilinear interpolant on pixel centres, W = 1
 *     (DP_W_NONE) or (SAD / depth)^2 (DP_W_FDK, depth = e_w.r + SAD);
 *   - spatial gradients of mu and l are central differences on grid points,
 *     zero outside the grid.
 *
 * Conventions for every entry point:
 *   - all array pointers are DEVICE pointers owned by the caller; `g` is a
 *     host pointer; `stream` is a hipStream_t (NULL = default stream);
 *   - calls are asynchronous on `stream`, never synchronise and never
 *     allocate device memory: scratch space comes from the caller's
 *     workspace `ws` of `ws_bytes` bytes (query dp_workspace_bytes);
 *   - outputs are overwritten, not accumulated;
 *   - arguments are validated before any launch; on error nothing is
 *     launched, outputs are untouched and the return value is negative;
 *     dp_last_error() then describes the failure (thread-local).
 *   - results are deterministic: reductions use fixed-order per-block
 *     partials; FP64 is used only for per-view setup and the final
 *     cross-block sum of the pose gradient.
 */
#ifndef DIFFPROJ_H
#define DIFFPROJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Acquisition geometry and voxel grid (host struct, passed by pointer). */
typedef struct dp_geom {
    int32_t nx, ny, nz;   /* volume size in voxels                                */
    double  vx, vy, vz;   /* voxel size (mm)                                      */
    int32_t nu, nv;       /* detector columns (u, fastest) and rows (v)           */
    double  du, dv;       /* pixel pitch (mm)                                     */
    double  off_u, off_v; /* detector-centre offset (pixels)                      */
    double  sad, sdd;     /* source-to-axis and source-to-detector distance (mm)  */
    double  step;         /* ray-march step (mm)                                  */
} dp_geom;

enum {
    DP_OK = 0,
    DP_ERR_ARG = -1,         /* null pointer, non-positive size, sdd <= sad, ...    */
    DP_ERR_WORKSPACE = -2,   /* ws_bytes smaller than dp_workspace_bytes()          */
    DP_ERR_HIP = -3,         /* a HIP launch reported an error                      */
    DP_ERR_UNSUPPORTED = -4  /* sizes beyond the kernels' index ranges              */
};

enum { DP_W_NONE = 0, DP_W_FDK = 1 };

enum {
    DP_OP_FWD = 0, DP_OP_FWD_GRAD = 1, DP_OP_BP = 2, DP_OP_BP_GRAD = 3, DP_OP_FWD_SSD = 4,
    DP_OP_FP_FWD = 5, DP_OP_FP_FWD_GRAD = 6, DP_OP_FP_BP = 7, DP_OP_FP_BP_GRAD = 8
};

/* Workspace size (bytes) needed by operation `op` (DP_OP_*) for this
 * geometry and view count; 0 for invalid arguments. */
size_t dp_workspace_bytes(const dp_geom* g, int32_t n_views, int32_t op);

/* Forward projection (Eq. forward).
 *   angles [V] f64 gantry angles, poses [V][6] f64 (tx,ty,tz mm; gx,gy,gz rad),
 *   vol [nz][ny][nx] f32, proj [V][nv][nu] f32 (overwritten). */
int dp_project_fwd(const dp_geom* g, int32_t n_views, const double* angles,
                   const double* poses, const float* vol, float* proj,
                   void* ws, size_t ws_bytes, void* stream);

/* Forward-projection pose gradient (Eqs. final_forward, dis_forward).
 *   grad_proj [V][nv][nu] f32 = dL/dl; grad_pose [V][6] f64 = dL/dtheta
 *   (overwritten; per mm and per rad).  Ray samples are recomputed, never
 *   stored. */
int dp_project_fwd_grad_pose(const dp_geom* g, int32_t n_views, const double* angles,
                             const double* poses, const float* vol,
                             const float* grad_proj, double* grad_pose,
                             void* ws, size_t ws_bytes, void* stream);

/* Forward projection, SSD loss and its pose gradient in one pass over the
 * samples (Eq. forward with Eqs. final_forward, dis_forward for the loss
 * L_v = sum over the view's pixels of (l - y)^2, whose dL/dl = 2 (l - y) is
 * known at the end of each ray, so the per-ray gradient sums are weighted
 * after the march and no separate forward launch is needed).
 *   target [V][nv][nu] f32 = y; proj [V][nv][nu] f32 = l (overwritten);
 *   loss [V] f64 = L_v (overwritten; may be NULL); grad_pose [V][6] f64 =
 *   dL_v/dtheta_v (overwritten).  Workspace: dp_workspace_bytes(g, V,
 *   DP_OP_FWD_SSD).  Same samples, tolerances and errors as the two calls it
 *   replaces. */
int dp_project_fwd_ssd_grad_pose(const dp_geom* g, int32_t n_views, const double* angles,
                                 const double* poses, const float* vol, const float* target,
                                 float* proj, double* loss, double* grad_pose,
                                 void* ws, size_t ws_bytes, void* stream);

/* As dp_project_fwd_ssd_grad_pose, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): no workspace argument and no allocation of any kind.
 * The workspace is a 16 MiB array in the library's device memory, one per
 * GPU, held until the process ends and shared by every call on that GPU; it
 * holds the per-view setup and the per-tile partial sums, so calls with
 * dp_workspace_bytes(g, n_views, DP_OP_FWD_SSD) > 16 MiB return
 * DP_ERR_UNSUPPORTED (at 512 x 512 pixels this allows about 390 views per
 * call).  Calls that overlap on one GPU (concurrent streams or threads) race
 * on that array; the kernels overwrite everything they read from it, so
 * nothing needs clearing between calls.  Arguments, outputs and errors as
 * dp_project_fwd_ssd_grad_pose. */
int dp_project_fwd_ssd_grad_pose_noalloc(const dp_geom* g, int32_t n_views, const double* angles,
                                         const double* poses, const float* vol,
                                         const float* target, float* proj, double* loss,
                                         double* grad_pose, void* stream);

/* As dp_project_fwd_ssd_grad_pose, plus the Gauss-Newton matrix of each
 * view's SSD: with J_p = dl_p/dtheta the per-ray pose Jacobian (the sums of
 * Eqs. final_forward / dis_forward for a unit weight on one ray),
 *   H_v = 2 sum over the view's rays of J_p J_p^T,
 * returned as hess [V][21] f64, the upper triangle row by row
 * ((0,0), (0,1), ..., (0,5), (1,1), ..., (5,5)), parameter order and units
 * as grad_pose.  Same workspace (DP_OP_FWD_SSD) and samples; the extra cost
 * is per ray, not per sample. */
int dp_project_fwd_ssd_gauss_newton(const dp_geom* g, int32_t n_views, const double* angles,
                                    const double* poses, const float* vol, const float* target,
                                    float* proj, double* loss, double* grad_pose, double* hess,
                                    void* ws, size_t ws_bytes, void* stream);

/* Voxel-driven back-projection (Eq. back), weight_mode DP_W_NONE | DP_W_FDK.
 *   proj [V][nv][nu] f32 (already filtered by the caller if FDK is meant),
 *   vol [nz][ny][nx] f32 (overwritten; between chunks of views it holds the
 *   unscaled partial sums, so it must not alias proj).  No angular scale is
 *   applied.  Views are processed in chunks whose detector-image copies fit
 *   a fixed budget of the workspace; the result does not depend on the
 *   chunking (the per-voxel sums run in view order either way). */
int dp_backproject(const dp_geom* g, int32_t n_views, const double* angles,
                   const double* poses, const float* proj, float* vol,
                   int32_t weight_mode, void* ws, size_t ws_bytes, void* stream);

/* Back-projection pose gradient (Eqs. final_back, back_int, dis_back).
 *   grad_vol [nz][ny][nx] f32 = dL/dmu; grad_pose [V][6] f64 (overwritten).
 *   With DP_W_FDK the product-rule term l~ grad_r W is included. */
int dp_backproject_grad_pose(const dp_geom* g, int32_t n_views, const double* angles,
                             const double* poses, const float* proj,
                             const float* grad_vol, double* grad_pose,
                             int32_t weight_mode, void* ws, size_t ws_bytes, void* stream);

/* Diagnostics of dp_backproject_grad_pose: byte offset, within its
 * workspace (DP_OP_BP_GRAD, same geometry and view count), of int32
 * flags[V].  After a call, flags[v] != 0 iff some voxel column of view v had
 * no usable FP32 anchor (it lies within 1 mm of the source plane, or its
 * middle voxel projects more than 2 max(nu, nv) + 64 pixels from the
 * detector centre) and was projected voxel by voxel in FP64.  Returns
 * (size_t)-1 for invalid arguments. */
size_t dp_bp_grad_flags_offset(const dp_geom* g, int32_t n_views);

/* ---------------------------------------------------------------------------
 * Uneven batches: many independent ray-driven problems (own volume,
 * detector, views and poses) in ONE forward launch and ONE gradient launch
 * (plus small per-problem setup / prep / finalize launches), e.g. many
 * registrations or calibrations of different sizes at once (the paper's
 * registration and calibration tasks, Sec. II-D, run many such problems).
 * Problem descriptors travel as kernel arguments, so a batch can be
 * captured in a graph.  At most 16 problems per call; workspace from
 * dp_batch_workspace_bytes.  variant = -1 uses the autotuned (or default)
 * variant of the largest problem.
 * ------------------------------------------------------------------------- */
typedef struct dp_problem {
    dp_geom       geom;
    int32_t       n_views;
    const double* angles;     /* device [V]                                     */
    const double* poses;      /* device [V][6]                                  */
    const float*  vol;        /* device [nz][ny][nx]                            */
    float*        proj;       /* device [V][nv][nu]  forward output             */
    const float*  grad_proj;  /* device [V][nv][nu]  gradient input dL/dl; the  */
                              /* target image y for the single-pass SSD batch    */
    double*       grad_pose;  /* device [V][6]       gradient output            */
    double*       loss;       /* device [V]  SSD batch: per-view SSD (or NULL)   */
    double*       hess;       /* device [V][21] SSD batch: Gauss-Newton matrix   */
} dp_problem;

size_t dp_batch_workspace_bytes(const dp_problem* problems, int32_t n, int32_t op);
int dp_project_fwd_batch(const dp_problem* problems, int32_t n, void* ws, size_t ws_bytes,
                         int32_t variant, void* stream);
int dp_project_fwd_grad_pose_batch(const dp_problem* problems, int32_t n, void* ws,
                                   size_t ws_bytes, int32_t variant, void* stream);
/* Single-pass SSD batch (dp_project_fwd_ssd_gauss_newton for every problem
 * in one ray launch): per problem proj (out), grad_proj = target y, loss
 * (optional), grad_pose and hess (both required).  Workspace:
 * dp_batch_workspace_bytes(problems, n, DP_OP_FWD_SSD). */
int dp_project_fwd_ssd_gauss_newton_batch(const dp_problem* problems, int32_t n, void* ws,
                                          size_t ws_bytes, int32_t variant, void* stream);

/* One Levenberg-Marquardt update per view, on the device, for n views laid
 * out back to back (e.g. every view of a batch).  In the scaled parameters
 * z = (t / 1 mm, gamma / 1 deg), with (f, g, H) the SSD, gradient and
 * Gauss-Newton matrix just evaluated at the trial poses `trial` [n][6]
 * (loss [n], grad [n][6], hess [n][21] as written by the SSD entries) and
 * the state of the last accepted point (state_pose [n][6], state_f [n],
 * state_g [n][6], state_h [n][21], lam [n]):
 *   accept if f < state_f (state <- trial values, lam /= 3; a NaN f is
 *   rejected), else lam *= 4; then solve (H + lam (diag H + 1e-12)) d = -g
 *   by FP64 Cholesky and write the next trial pose state_pose + d into
 *   `trial`.
 * A view whose accepted step is below tol in every scaled parameter, whose
 * lam exceeds 1e10, or whose damped matrix is not positive definite is
 * marked done[n] = 1 and its trial pose stays at the accepted pose; done
 * views are left untouched by later calls.  Initialise state_f to +inf (the
 * first evaluation is then accepted without changing lam), state_g and
 * state_h to anything finite, lam to the initial damping and done to 0.
 * All arrays are caller-owned device memory, FP64 (done: int32), disjoint;
 * no allocation, no host synchronisation, so an iteration (SSD batch + this
 * update) can be captured in a graph and replayed.  Returns DP_ERR_ARG for
 * n <= 0, a NULL array or a negative tol. */
int dp_lm_update(int32_t n, double* trial, const double* loss, const double* grad,
                 const double* hess, double* state_pose, double* state_f, double* state_g,
                 double* state_h, double* lam, int32_t* done, double tol, void* stream);

/* ---------------------------------------------------------------------------
 * Kernel variants of the ray-driven kernels: DP_RD_VARIANTS = 9, variant =
 * 3 * tile shape + chunk class.  Tile shapes (detector pixels per block,
 * u x v): 0 = 16 x 16, 1 = 32 x 8, 2 = 8 x 32; chunk classes (chunk length
 * before adaptation and LDS budget): 0, 1, 2.  Variant 1 (16 x 16, class 1)
 * is the default.  Every variant computes the same result up to FP32
 * summation order.  dp_autotune times every variant of `op` (DP_OP_FWD,
 * DP_OP_FWD_GRAD or DP_OP_FWD_SSD) on the given inputs (reps timed calls
 * each, after one warm-up; `out` is proj for FWD and FWD_SSD, grad_pose for
 * FWD_GRAD; grad_proj is dL/dl for FWD_GRAD and the target image for
 * FWD_SSD, whose pose gradient lands in the workspace), records the fastest for this shape
 * class (grid and detector sizes, view-count octave, pixel-to-voxel ratio)
 * in a process-wide cache used by later calls, and synchronises `stream`.
 * dp_set_variant forces a variant for `op` (-1 = cached / default);
 * dp_get_variant returns the variant a call of `op` on this shape would use
 * (-1 for another op or a NULL geometry).
 * ------------------------------------------------------------------------- */
#define DP_RD_VARIANTS 9
int dp_autotune(int32_t op, const dp_geom* g, int32_t n_views, const double* angles,
                const double* poses, const float* vol, const float* grad_proj, void* out,
                void* ws, size_t ws_bytes, void* stream, int32_t reps, int32_t* best,
                float* ms_per_variant /* [DP_RD_VARIANTS] or NULL */);
int dp_set_variant(int32_t op, int32_t variant);
int32_t dp_get_variant(const dp_geom* g, int32_t n_views, int32_t op);

/* ---------------------------------------------------------------------------
 * Learned pose proposal (not in the paper; its discussion, Sec. IV, points
 * to learning-based initialisation): primitives of a strided CNN on BF16
 * matrix cores with FP32 accumulation.  Activations are NHWC BF16; a 3x3
 * convolution with padding 1 and stride s maps H x W to
 * Ho = (H - 1) / s + 1, Wo = (W - 1) / s + 1.  All pointers are device
 * pointers; calls are asynchronous on `stream`.
 * ------------------------------------------------------------------------- */
/* C[M][N] (FP32, row stride ldc) = op(A) op(B) (+ C if accumulate); A is
 * BF16 [M][K] (trans_a = 0) or [K][M]; B is BF16 [K][N] (trans_b = 0) or [N][K]. */
int dp_gemm_bf16(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                 const void* A, int32_t lda, const void* B, int32_t ldb, float* C,
                 int32_t ldc, int32_t accumulate, void* stream);
/* The same product with split-K partial sums in a caller workspace of
 * dp_gemm_bf16_ws_bytes(M, N, K) bytes (0: none needed) for few output
 * tiles and a long reduction (weight gradients), reduced in split order, so
 * the result does not depend on block timing; dp_gemm_bf16 runs such
 * products in one pass.  Error DP_ERR_ARG if the workspace is too small. */
size_t dp_gemm_bf16_ws_bytes(int32_t M, int32_t N, int32_t K);
int dp_gemm_bf16_ws(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                    const void* A, int32_t lda, const void* B, int32_t ldb, float* C, int32_t ldc,
                    int32_t accumulate, void* ws, size_t ws_bytes, void* stream);
/* Forward convolution product with its epilogue: Y [M][N] BF16 (row stride
 * ldy) = act(A B^T + bias), A [M][K] and B [N][K] BF16, FP32 accumulation,
 * bias of output column n at bias[n * bias_stride] (FP32), act = ReLU if
 * relu else identity, rounded to BF16 once. */
int dp_gemm_bias_act_bf16(int32_t M, int32_t N, int32_t K, const void* A, int32_t lda,
                          const void* B, int32_t ldb, const float* bias, int32_t bias_stride,
                          int32_t relu, void* Y, int32_t ldy, void* stream);
/* col [N Ho Wo][9 C] BF16 from x [N][H][W][C] BF16; K index (ky, kx, c).
 * N Ho Wo 9 C and N H W C must stay below 2^31 (DP_ERR_UNSUPPORTED otherwise;
 * split the batch).  The same limit holds for dp_col2im3x3. */
int dp_im2col3x3_bf16(int32_t N, int32_t H, int32_t W, int32_t C, int32_t stride,
                      const void* x, void* col, void* stream);
/* As dp_im2col3x3_bf16 with rows of ld >= 9 C (+ 1) entries: the 9 C window
 * values, then 1 in column 9 C if ones (the product dz^T col then carries
 * the column sums of dz, the bias gradient, in that column), zeros after. */
int dp_im2col3x3_ld_bf16(int32_t N, int32_t H, int32_t W, int32_t C, int32_t stride,
                         const void* x, void* col, int32_t ld, int32_t ones, void* stream);
/* dx [N][H][W][C] FP32 = adjoint of im2col applied to dcol [N Ho Wo][9 C] FP32. */
int dp_col2im3x3(int32_t N, int32_t H, int32_t W, int32_t C, int32_t stride,
                 const float* dcol, float* dx, void* stream);
/* The same adjoint followed by the activation backward of the layer below:
 * dz [N][H][W][C] BF16 = dx * (y > 0) if relu else dx, y [N][H][W][C] BF16
 * that layer's output (one rounding to BF16). */
int dp_col2im3x3_act_bf16(int32_t N, int32_t H, int32_t W, int32_t C, int32_t stride,
                          const float* dcol, const void* y, int32_t relu, void* dz, void* stream);
/* Implicit-GEMM 3x3 convolutions (padding 1, stride >= 1) on NHWC BF16
 * tensors: no im2col matrix is formed, each product gathers its operand
 * tiles from the tensors.  Ci and Co multiples of 8, ldw a multiple of 8 and
 * >= 9 Ci (+ 1 with ones), every pointer 16-byte aligned; N H W Ci and
 * N Ho Wo 9 Ci below 2^31 (DP_ERR_UNSUPPORTED otherwise; split the batch).
 * Weights w [Co][ldw] BF16, row co = the 9 Ci kernel values in (ky, kx, ci)
 * order, further entries ignored.
 * dp_conv3x3_fwd_bf16: y [N][Ho][Wo][Co] BF16 = act(conv(x) + bias), bias of
 *   output channel o at bias[o * bias_stride], act = ReLU if relu.  The same
 *   values as dp_im2col3x3_bf16 + dp_gemm_bias_act_bf16. */
int dp_conv3x3_fwd_bf16(int32_t N, int32_t H, int32_t W, int32_t Ci, int32_t Co, int32_t stride,
                        const void* x, const void* w, int32_t ldw, const float* bias,
                        int32_t bias_stride, int32_t relu, void* y, void* stream);
/* dp_conv3x3_wgrad_bf16: dw [Co][ldw] FP32 = dz^T . im2col(x) over the N Ho Wo
 *   output pixels, dz [N][Ho][Wo][Co] BF16: columns < 9 Ci the weight
 *   gradient, column 9 Ci the bias gradient (column sums of dz) if ones,
 *   further columns zero.  Long reductions are split over a workspace of
 *   dp_conv3x3_wgrad_ws_bytes bytes (may be 0; NULL then allowed) and
 *   reduced in a fixed order. */
size_t dp_conv3x3_wgrad_ws_bytes(int32_t N, int32_t H, int32_t W, int32_t Ci, int32_t Co,
                                 int32_t stride, int32_t ldw);
int dp_conv3x3_wgrad_bf16(int32_t N, int32_t H, int32_t W, int32_t Ci, int32_t Co,
                          int32_t stride, const void* x, const void* dz, int32_t ldw,
                          int32_t ones, float* dw, void* ws, size_t ws_bytes, void* stream);
/* dp_conv3x3_dgrad_act_bf16: the input gradient dx [N][H][W][Ci] of
 *   sum(dz . conv(x)), followed by the activation backward of the layer
 *   below: out BF16 = dx * (y > 0) if relu (y [N][H][W][Ci] BF16, that
 *   layer's output) else dx (y may be NULL).  Computed per parity class of
 *   input pixels (stride^2 products, one per class, each summing exactly the
 *   taps that reach the class), one rounding to BF16. */
int dp_conv3x3_dgrad_act_bf16(int32_t N, int32_t H, int32_t W, int32_t Ci, int32_t Co,
                              int32_t stride, const void* dz, const void* w, int32_t ldw,
                              const void* y, int32_t relu, void* out, void* stream);
/* One Adam step over n parameters in flat FP32 buffers: m = b1 m + (1 - b1) g,
 * v = b2 v + (1 - b2) g^2, p -= lr (m / c1) / (sqrt(v / c2) + eps), and p
 * rounded to BF16 into p_bf16 [n].  c1, c2 > 0: the bias corrections. */
int dp_adam_f32(int64_t n, float* p, const float* g, float* m, float* v, void* p_bf16, float lr,
                float beta1, float beta2, float eps, float c1, float c2, void* stream);
/* y [rows][C] BF16 = act(z + bias), act = ReLU if relu else identity. */
int dp_bias_act_bf16(int64_t rows, int32_t C, const float* z, const float* bias,
                     int32_t relu, void* y, void* stream);
/* dz BF16 = dy * (y > 0) if relu else dy, elementwise (y BF16, dy FP32). */
int dp_act_bwd_bf16(int64_t total, const float* dy, const void* y, int32_t relu, void* dz,
                    void* stream);
/* db[c] = sum over the M rows of dz [M][C] (BF16), FP32 out (db is
 * overwritten; block sums are combined with FP32 atomics, so the last bits
 * can differ between runs). */
int dp_colsum_bf16(int32_t M, int32_t C, const void* dz, float* db, void* stream);

/* ---------------------------------------------------------------------------
 * Footprint projector pairs and their pose gradients (the discrete
 * projectors of Sec. II-C, l = A mu and mu = A^T l with footprint weights
 * a_ij; gradients by Eqs. dis_forward / dis_back).  The footprint of a
 * voxel moved by the view's pose is a unit-height shape in the detector
 * column times a unit-height rectangle in the row (the projected top and
 * bottom centres), scaled by an amplitude:
 *   DP_FP_SF (separable footprint): trapezoid with breakpoints at the
 *     projected corners of the voxel's mid-height cross-section; amplitude
 *     the voxel's chord along the line from the source through its centre;
 *   DP_FP_DD (distance-driven): rectangle between the projected boundaries
 *     across the view's dominant transaxial axis (x if the source's
 *     object-frame offset from the volume centre has |x| >= |y|, else y);
 *     amplitude the path through the slab along that axis.
 * a_ij = amplitude x (column shape integrated over pixel i's column cell)
 * x (row rectangle's overlap with its row cell).  Arguments, layouts and
 * errors as for the ray-driven / voxel-driven entries; kind must be
 * DP_FP_SF or DP_FP_DD; workspace: dp_workspace_bytes(g, V, DP_OP_FP_*).
 *   dp_fp_project: proj [V][nv][nu] (overwritten) = A vol (FP32 atomic
 *     accumulation: not bitwise reproducible).
 *   dp_fp_backproject: vol (overwritten) = A^T proj (no angular weight).
 *   dp_fp_project_grad_pose: dL/dtheta [V][6] from dL/dl = grad_proj.
 *   dp_fp_backproject_grad_pose: dL/dtheta [V][6] from dL/dmu = grad_vol.
 * ------------------------------------------------------------------------- */
enum { DP_FP_SF = 0, DP_FP_DD = 1 };
int dp_fp_project(const dp_geom* g, int32_t n_views, const double* angles, const double* poses,
                  const float* vol, float* proj, int32_t kind, void* ws, size_t ws_bytes,
                  void* stream);
int dp_fp_backproject(const dp_geom* g, int32_t n_views, const double* angles, const double* poses,
                      const float* proj, float* vol, int32_t kind, void* ws, size_t ws_bytes,
                      void* stream);
int dp_fp_project_grad_pose(const dp_geom* g, int32_t n_views, const double* angles,
                            const double* poses, const float* vol, const float* grad_proj,
                            double* grad_pose, int32_t kind, void* ws, size_t ws_bytes,
                            void* stream);
int dp_fp_backproject_grad_pose(const dp_geom* g, int32_t n_views, const double* angles,
                                const double* poses, const float* proj, const float* grad_vol,
                                double* grad_pose, int32_t kind, void* ws, size_t ws_bytes,
                                void* stream);

/* ---------------------------------------------------------------------------
 * Motion-compensated FDK reconstruction (Sec. III-B, motion-compensated
 * analytical reconstruction: FDK-style back-projection of ramp-filtered
 * projections, motion estimated by maximising image sharpness).
 *
 * dp_fdk_filter: out[V][nv][nu] = FDK pre-filtered proj[V][nv][nu] (both
 * FP32 device arrays; out == proj is allowed).  Detector coordinates are
 * referred to the isocentre (pitch tau = du * sad / sdd, centre as in the
 * projector), multiplied by the cosine weight sad / sqrt(sad^2 + u'^2 + v'^2)
 * and convolved along u with the band-limited ramp kernel (h[0] = 1/(4 tau^2),
 * h[k] = -1/(pi^2 k^2 tau^2) for odd k, 0 otherwise; rows zero outside the
 * detector), times scale * tau.  With scale = pi / V for V views over a full
 * circle, dp_backproject(..., DP_W_FDK) of the result is the FDK
 * reconstruction.  Only the detector fields of `g` are used (the volume
 * fields must still be valid).  Errors: DP_ERR_ARG for bad arguments,
 * DP_ERR_UNSUPPORTED for rows longer than 4000 pixels.
 *
 * dp_sharpness: *loss (one FP64 on the device) = S(vol) = -(sum of the
 * squared forward differences of vol [nz][ny][nx] along x, y and z, over
 * pairs inside the grid); if grad is not NULL, grad [nz][ny][nx] FP32 =
 * dS/dvol.  ws: device workspace of dp_sharpness_workspace_bytes(nx, ny,
 * nz) bytes, 256-byte aligned.  The result is bitwise reproducible.
 * ------------------------------------------------------------------------- */
int dp_fdk_filter(const dp_geom* g, int32_t n_views, const float* proj, float* out, double scale,
                  void* stream);
size_t dp_sharpness_workspace_bytes(int32_t nx, int32_t ny, int32_t nz);
int dp_sharpness(int32_t nx, int32_t ny, int32_t nz, const float* vol, double* loss, float* grad,
                 void* ws, size_t ws_bytes, void* stream);
/* dp_gradient_entropy: the sharpness criterion of the paper's
 * motion-compensated FBP experiment (Sec. III-B).  With the forward
 * differences above (zero where the +axis neighbour is outside the grid),
 * g_j = sqrt(dx_j^2 + dy_j^2 + dz_j^2 + eps), p_j = g_j / sum g and
 * *loss (device FP64) = GE = -sum p_j log p_j (lower is sharper); grad
 * (optional, FP32 like vol) = dGE/dvol.  eps > 0 keeps g differentiable at
 * zero (1e-12 for attenuation volumes in mm^-1).  ws: device workspace of
 * dp_gradient_entropy_workspace_bytes(nx, ny, nz) bytes, 256-byte aligned.
 * Bitwise reproducible. */
size_t dp_gradient_entropy_workspace_bytes(int32_t nx, int32_t ny, int32_t nz);
int dp_gradient_entropy(int32_t nx, int32_t ny, int32_t nz, const float* vol, float eps,
                        double* loss, float* grad, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Streaming-read probe (measurement only; not part of the paper's method).
 * The ray kernels gather trilinear taps through the cache hierarchy, so their
 * ceiling is a read bandwidth: this kernel measures it on the running GPU.
 *
 * dp_read_probe: n_blocks blocks of 256 threads read the FP32 device buffer
 * buf (16-byte aligned, n_vec float4) and write one FP32 sum per thread to
 * out (n_blocks * 256 floats, device).
 *   shared != 0: every block reads all n_vec float4 `reps` times (from its
 *     own starting offset, wrapping around); n_vec must be a power of two in
 *     [2048, 2^30].  A footprint of a few MiB stays resident in every XCD's
 *     L2 and far exceeds a CU's L1, so bytes read = n_blocks * reps * n_vec * 16
 *     measures the L2 read bandwidth.
 *   shared == 0: with per = 2048 * floor(n_vec / (2048 * n_blocks)), block b
 *     reads float4 [b * per, (b + 1) * per) with nontemporal loads (thread j
 *     the ones whose offset in the slab is j mod 256), then the blocks share
 *     the tail [n_blocks * per, n_vec) grid-stride (thread j of block b from
 *     n_blocks * per + 256 b + j, stepping 256 n_blocks); every float4 is read
 *     once per pass.  n_vec + 256 * n_blocks must stay below 2^32.  A buffer
 *     far above L2 and the last-level cache measures HBM read bandwidth.
 * Thread j of block b writes the sum of the components of the float4 it read
 * to out[256 b + j]; with buf all ones and shared != 0 every sum is
 * reps * n_vec * 4 / 256.  Errors: DP_ERR_ARG for
 * NULL or misaligned pointers, non-positive sizes or a bad shared footprint,
 * DP_ERR_UNSUPPORTED beyond the index range or 2^20 blocks.
 * ------------------------------------------------------------------------- */
int dp_read_probe(const void* buf, int64_t n_vec, int32_t reps, int32_t shared, int32_t n_blocks,
                  float* out, void* stream);

/* dp_lds_probe (measurement only): n_blocks blocks of 256 threads each fill
 * 32 KiB of LDS with 2048 float4 (vector i = (i, 1, 2, 3)), then every
 * thread reads `reps` * 8 float4 from it with 16-byte LDS loads (in step r,
 * lane j reads vectors (64 r + 256 u + j) mod 2048, u = 0..7: conflict-free), and
 * writes the sum of their components to out[256 b + j] (n_blocks * 256
 * floats, device).  LDS bytes read = n_blocks * 256 * reps * 128, the ceiling
 * of LDS-staged gathers.  Errors: DP_ERR_ARG for NULL out or non-positive
 * sizes, DP_ERR_UNSUPPORTED beyond 2^20 blocks. */
int dp_lds_probe(int32_t reps, int32_t n_blocks, float* out, void* stream);

/* Thread-local description of the last non-zero return. */
const char* dp_last_error(void);

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t dp_version(void);

/* Optional per-kernel timing with HIP events recorded on the caller's
 * stream around every launch (for benchmarks; adds two event records per
 * launch).  Not thread-safe: enable, run, collect from one thread.
 *   dp_profile_enable(1) starts recording (creates the event pool),
 *   dp_profile_enable(0) stops;
 *   dp_profile_collect() waits for the recorded events and accumulates
 *   their durations per kernel;
 *   dp_profile_read(k, &ms, &n) returns the accumulated time and launch
 *   count of kernel k (DP_K_*) and resets them.  DP_K_VOL_PREP times the
 *   (mu, gradient) copy that the gradient calls make only for geometries
 *   whose rays are sparse relative to the voxels (pixel footprint at the
 *   isocentre above 0.85 voxel); otherwise the ray-driven kernels read the
 *   caller's volume and form its gradient while staging it. */
enum {
    DP_K_SETUP = 0, DP_K_VOL_PREP = 1, DP_K_RD_FWD = 2, DP_K_RD_GRAD = 3,
    DP_K_DET_PREP = 4, DP_K_VD_BP = 5, DP_K_VD_GRAD = 6, DP_K_FINALIZE = 7,
    DP_K_FDK_FILTER = 8, DP_K_SHARPNESS = 9, DP_K_RD_FUSED = 10, DP_K_SF = 11,
    DP_K_COUNT = 12
};
int dp_profile_enable(int32_t on);
int dp_profile_collect(void);
int dp_profile_read(int32_t kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* DIFFPROJ_H */
