// Internal definitions shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "diffproj.h"

namespace dp {

// Zero border added around internal copies of the volume and of detector
// images: every trilinear / bilinear tap of an in-support sample lands
// inside the padded buffer, so the hot loops carry no per-tap bounds test.
constexpr int kPadV = 2;
constexpr int kPadD = 2;

// Ray-driven launch shape: one block = 256 detector pixels = 4 wavefronts,
// each wavefront an 8x8 pixel tile (compact footprint in the volume).  The
// block's tile is 16x16 (shape 0), 32x8 (shape 1) or 8x32 (shape 2) pixels
// (u x v), its wavefront sub-tiles laid out along u first.
constexpr int kRdThreads = 256;
constexpr int kRdShapes = 3;
__host__ __device__ constexpr int rd_tile_w(int shape)
{
    return shape == 1 ? 32 : shape == 2 ? 8 : 16;
}
__host__ __device__ constexpr int rd_tile_h(int shape) { return kRdThreads / rd_tile_w(shape); }
constexpr int kRdChannels = 9;   // B (3) and T (6) accumulators of the pose gradient

// Voxel-driven launch shape: 64 (x) x 4 (y) threads, each thread owns a
// column of voxels along z (kVdBpCol for the back-projection, kVdGradCol for
// its gradient); the FP64 column anchor is computed once per view per column.
constexpr int kVdBx = 64;
constexpr int kVdBy = 4;
constexpr int kVdBpCol = 32;
constexpr int kVdGradCol = 32;
constexpr int kVdChannels = 12;  // A (3), QX (3), QY (3), QZ (3)
// Back-projection gradient blocks: kVgBx x kVgBy voxel columns (4
// wavefronts), and the detector pixels per view they stage in LDS.
constexpr int kVgBx = 16;
constexpr int kVgBy = 16;
constexpr int kVgStage = 640;
// Views per back-projection gradient launch (per-view block sums held in LDS)
// and the block count below which blocks stop taking several column groups.
constexpr int kVdMaxChunk = 64;
#ifndef DP_VD_GRAD_MIN_BLOCKS
#define DP_VD_GRAD_MIN_BLOCKS 8192
#endif
constexpr int kVdGradMinBlocks = DP_VD_GRAD_MIN_BLOCKS;
// Detector images are staged per chunk of views, within this many bytes
// (a build-time choice; results do not depend on it).
#ifndef DP_DET_CHUNK_MIB
#define DP_DET_CHUNK_MIB 512
#endif
constexpr size_t kDetChunkBytes = (size_t)DP_DET_CHUNK_MIB << 20;

// Per padded detector pixel (A, B): the bilinear coefficients of l, dl/da
// and dl/db on the cell [A, A+1] x [B, B+1] (value, a-difference,
// b-difference, mixed second difference).
struct alignas(16) DetTap3 {
    float4 l, a, b;
};

struct VdGradGrid {
    int zpb;     // column groups of kVdGradCol voxels per block
    int gz;      // blocks along z
    int blocks;  // blocks per launch = partial sets per view
};

// Per-view parameters, produced on the device by the setup kernel from the
// gantry angles and the (device-resident) poses.
struct alignas(16) ViewGeo {
    // Ray-driven: object-frame basis in padded voxel-index units.
    double EU[3], EV[3], EW[3];  // R^T e_{u,v,w} / h  (index units per mm)
    double OT[3];                // padded index of the world isocentre: R^T(-t)/h + c + pad
    // Voxel-driven: (U, V, W) = rows . (i, j, k, 1) with original voxel
    // indices; a = U / W + cu, b = V / W + cv, W = depth (mm).  FP64 rows
    // anchor each voxel column; the FP32 copies of the z coefficients
    // evaluate the small in-column offsets.
    double PUd[4], PVd[4], PWd[4];
    float PU[4], PV[4], PW[4];
    // Pose quantities for the final contraction (FP64).
    double E[9];                 // world frame: (S/du) e_u, (S/dv) e_v, e_w
    double R[9];                 // rotation, row-major
    double omega[9];             // generators omega_x, omega_y, omega_z (world)
};

struct GeoScalars {
    int nx, ny, nz, nu, nv;
    double vx, vy, vz, du, dv, cu, cv, sad, sdd, step;
};

inline GeoScalars make_scalars(const dp_geom& g)
{
    GeoScalars s;
    s.nx = g.nx; s.ny = g.ny; s.nz = g.nz; s.nu = g.nu; s.nv = g.nv;
    s.vx = g.vx; s.vy = g.vy; s.vz = g.vz; s.du = g.du; s.dv = g.dv;
    s.cu = 0.5 * (g.nu - 1) + g.off_u;
    s.cv = 0.5 * (g.nv - 1) + g.off_v;
    s.sad = g.sad; s.sdd = g.sdd; s.step = g.step;
    return s;
}

// Kernel launchers (defined next to their kernels).
void launch_view_setup(const GeoScalars& s, int V, const double* angles, const double* poses,
                       ViewGeo* views, hipStream_t st);
// per padded pixel, the bilinear cell coefficients of l as one float4
void launch_det_pad(const GeoScalars& s, int V, const float* proj, float4* projq, hipStream_t st);
void launch_det_grad(const GeoScalars& s, int V, const float* proj, float4* proj4, hipStream_t st);
void launch_det_tap3(const GeoScalars& s, int V, const float* proj, DetTap3* det, hipStream_t st);
// The ray-driven kernels read the caller's volume [nz][ny][nx] directly.
void launch_rd_fwd(const GeoScalars& s, int V, const ViewGeo* views, const float* mu,
                   float* proj, int variant, hipStream_t st);
// inter: padded (mu, Gx, Gy, Gz) copy for tiles that cannot stage a box, or NULL
void launch_rd_grad(const GeoScalars& s, int V, const ViewGeo* views, const float* mu,
                    const float4* inter, const float* grad_proj, float* partials, int variant,
                    hipStream_t st);
// The padded (mu, Gx, Gy, Gz) copy (G: central differences, not halved), and
// whether a geometry's rays are sparse enough relative to its voxels that the
// gradient kernels want it.
void launch_vol_inter(const GeoScalars& s, const float* vol, float4* inter, hipStream_t st);
bool sparse_rays(const GeoScalars& s);

// Uneven batches of ray-driven problems in one launch (descriptors by value).
constexpr int kRdMaxBatch = 16;
// Compiled variants: tile shape (above) x chunk class (chunk length before
// adaptation and LDS budget, three per kernel); variant = shape * 3 + class.
constexpr int kRdChunkClasses = 3;
constexpr int kRdVariants = kRdShapes * kRdChunkClasses;
static_assert(kRdVariants == DP_RD_VARIANTS, "variant count of the public header");
inline int rd_variant_shape(int variant) { return variant / kRdChunkClasses; }
// fused SSD kernel with the Gauss-Newton matrix: 9 gradient sums, the SSD,
// and the 21 upper-triangle entries of 2 J J^T
constexpr int kRdChannelsGN = kRdChannels + 1 + 21;
struct RdBatchItem {
    GeoScalars s;
    const ViewGeo* views;
    const float* vol;   // the problem's volume [nz][ny][nx]
    const float4* inter;  // padded (mu, Gx, Gy, Gz) for sparse-ray geometries, or NULL
    const float* gin;   // dL/dl (gradient) or the target y (single-pass SSD)
    float* out;         // DRRs (forward) or per-block partials (gradient, SSD)
    float* proj;        // DRRs of the single-pass SSD batch
    int tiles;          // detector tiles per view
    int first;          // first block of this problem
};
struct RdBatch {
    int n;
    RdBatchItem it[kRdMaxBatch];
};
void launch_rd_fwd_batch(const RdBatch& bt, int blocks, int variant, hipStream_t st);
void launch_rd_fused(const GeoScalars& s, int V, const ViewGeo* views, const float* mu,
                     const float4* inter, const float* target, float* proj, float* partials,
                     bool hess, int variant, hipStream_t st);
void launch_finalize_fwd_ssd(const GeoScalars& s, int V, const ViewGeo* views,
                             const float* partials, int n_part, double* grad_pose, double* loss,
                             double* hess, hipStream_t st);
void launch_rd_grad_batch(const RdBatch& bt, int blocks, int variant, hipStream_t st);
void launch_rd_fused_batch(const RdBatch& bt, int blocks, int variant, hipStream_t st);
void launch_lm_update(int n, double* trial, const double* loss, const double* grad,
                      const double* hess, double* state_pose, double* state_f, double* state_g,
                      double* state_h, double* lam, int* done, double tol, hipStream_t st);
// Back-projection of the views [v0, v0 + Vc), whose footprint images are
// projq[0 .. Vc); sums carried in vol between chunks (first / last chunk).
void launch_vd_bp(const GeoScalars& s, int v0, int Vc, const ViewGeo* views, const float4* projq,
                  float* vol, int weight_mode, bool first, bool last, hipStream_t st);
// Pose-gradient partials of the views [v0, v0 + Vc) (images det[0 .. Vc)),
// partials[v][blocks][kVdChannels]; flags[V] must be cleared before the first chunk.
VdGradGrid vd_grad_grid(const GeoScalars& s);
void launch_vd_flags_clear(int V, int* flags, hipStream_t st);
void launch_vd_grad(const GeoScalars& s, int v0, int Vc, const ViewGeo* views, const DetTap3* det,
                    const float* grad_vol, float* partials, int* flags, int weight_mode,
                    hipStream_t st);
void launch_finalize_fwd(const GeoScalars& s, int V, const ViewGeo* views, const float* partials,
                         int n_part, double* grad_pose, hipStream_t st);
void launch_finalize_bp(const GeoScalars& s, int V, const ViewGeo* views, const float* partials,
                        int n_part, double* grad_pose, hipStream_t st);

// Learned-proposal CNN primitives (cnn.hip).
// ws (may be NULL): split-K partials for few output tiles and a long
// reduction, gemm_ws_bytes(M, N, K) bytes; without it the product runs in one
// pass.  Either way the result does not depend on block timing.
size_t gemm_ws_bytes(int M, int N, int K);
void launch_gemm_bf16(bool ta, bool tb, int M, int N, int K, const void* A, int lda, const void* B,
                      int ldb, float* C, int ldc, bool accumulate, float* ws, size_t ws_bytes,
                      hipStream_t st);
// Y [M][N] BF16 (row stride ldy) = act(A B^T + bias), A [M][K], B [N][K] BF16.
void launch_gemm_bias_act(int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                          const float* bias, int bias_stride, bool relu, void* Y, int ldy,
                          hipStream_t st);
// Implicit-GEMM 3x3 convolutions (padding 1, stride s) on NHWC BF16 tensors
// with Ci and Co multiples of 8, weights w [Co][ldw] BF16 (9 Ci per row,
// (ky, kx, ci) order; ldw a multiple of 8), 16-byte aligned pointers.
// Forward: y [N][Ho][Wo][Co] = act(conv(x) + bias).
void launch_conv_fwd(int N, int H, int W, int Ci, int Co, int s, const void* x, const void* w,
                     int ldw, const float* bias, int bias_stride, bool relu, void* y, hipStream_t st);
// Weight gradient dw [Co][ldw] FP32 = dz^T . im2col(x) (column 9 Ci: the
// bias gradient if `ones`; further columns zero); split-K workspace as for
// the GEMM.
size_t conv_wgrad_ws_bytes(int N, int H, int W, int Ci, int Co, int s, int ldw);
void launch_conv_wgrad(int N, int H, int W, int Ci, int Co, int s, const void* x, const void* dz,
                       int ldw, bool ones, float* dw, float* ws, size_t ws_bytes, hipStream_t st);
// Input gradient, per parity class of input pixels, with the ReLU backward
// of the layer below: out [N][H][W][Ci] BF16 = dx (y == NULL or !relu) or
// dx * (y > 0).
void launch_conv_dgrad_act(int N, int H, int W, int Ci, int Co, int s, const void* dz,
                           const void* w, int ldw, const void* y, bool relu, void* out,
                           hipStream_t st);
// col rows of ld >= 9 C entries: the 9 C window values, then 1 (ones) and zeros.
void launch_im2col(int N, int H, int W, int C, int s, int Ho, int Wo, const void* x, void* col,
                   int ld, bool ones, hipStream_t st);
// y == NULL: FP32 dx; else the BF16 dz = dx * (y > 0) (relu) or dx of the layer below.
void launch_col2im(int N, int H, int W, int C, int s, int Ho, int Wo, const float* dcol, float* dx,
                   const void* y, bool relu, void* dz, hipStream_t st);
void launch_adam(size_t n, float* p, const float* g, float* m, float* v, void* pb, float lr,
                 float b1, float b2, float eps, float c1, float c2, hipStream_t st);
void launch_bias_relu(size_t total, int C, const float* z, const float* b, bool relu, void* y,
                      hipStream_t st);
void launch_relu_bwd(size_t total, const float* dy, const void* y, bool relu, void* dz,
                     hipStream_t st);
void launch_colsum(int M, int C, const void* dz, float* db, hipStream_t st);

// Separable-footprint projector pair and gradients (sf.hip).
int sf_blocks(const GeoScalars& s);
// kind: DP_FP_SF or DP_FP_DD
void launch_sf_fwd(const GeoScalars& s, int V, const ViewGeo* views, const float* vol, float* proj,
                   int kind, hipStream_t st);
void launch_sf_bp(const GeoScalars& s, int V, const ViewGeo* views, const float* proj, float* vol,
                  int kind, hipStream_t st);
void launch_sf_fwd_grad(const GeoScalars& s, int V, const ViewGeo* views, const float* vol,
                        const float* grad_proj, float* partials, int kind, hipStream_t st);
// views [v0, v0 + Vc), proj4 = this chunk's detector gradient images
void launch_sf_bp_grad(const GeoScalars& s, int v0, int Vc, const ViewGeo* views,
                       const float4* proj4, const float* grad_vol, float* partials, int kind,
                       hipStream_t st);

// FDK pre-filter and sharpness loss (fdk.hip).
void launch_fdk_filter(const GeoScalars& s, int V, const float* proj, float* out, double scale,
                       hipStream_t st);
int fdk_max_nu();
size_t sharpness_partials(int nx, int ny, int nz);
void launch_sharpness(int nx, int ny, int nz, const float* vol, float* grad, double* loss,
                      double* partial, hipStream_t st);
size_t gradient_entropy_ws_doubles(int nx, int ny, int nz);
void launch_gradient_entropy(int nx, int ny, int nz, float eps, const float* vol, float* grad,
                             double* loss, double* ws, hipStream_t st);

inline int rd_tiles(const GeoScalars& s, int shape)
{
    const int tw = rd_tile_w(shape), th = rd_tile_h(shape);
    return ((s.nu + tw - 1) / tw) * ((s.nv + th - 1) / th);
}

// Tiles of the shape with the most (per-block partial buffers are sized for it).
inline int rd_tiles_max(const GeoScalars& s)
{
    int m = 0;
    for (int sh = 0; sh < kRdShapes; ++sh) m = m > rd_tiles(s, sh) ? m : rd_tiles(s, sh);
    return m;
}


// Profiling hooks (abi.hip): bracket a launch with events when enabled.
void prof_begin(int kernel, hipStream_t st);
void prof_end(int kernel, hipStream_t st);

}  // namespace dp
