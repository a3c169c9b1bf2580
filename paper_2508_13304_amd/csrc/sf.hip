// Footprint projector pairs -- separable footprint (SF) and distance-driven
// (DD) -- and their rigid-motion gradients (the discrete projectors
// l = A mu, mu = A^T l of Sec. II-C with footprint weights a_ij; gradients by
// Eqs. dis_forward / dis_back: the same weights applied to G_f per voxel and
// to G_b per pixel).
//
// DD replaces the transaxial trapezoid by a unit-height rectangle between
// the projections of the voxel's two boundaries across the view's dominant
// transaxial axis (x if the source's object-frame offset from the volume
// centre has |x| >= |y|, else y), taken at the voxel centre, and the chord
// by the path length h_dom |d| / |d_dom| through the slab along that axis.
// Everything else below is shared.
//
// Footprint of voxel j in one view, with the voxel moved by the pose (the
// view's projective map on voxel indices, FP64):
//   transaxial: the corners (i +- 1/2, j +- 1/2) of the mid-height
//     cross-section project to columns tau0 <= tau1 <= tau2 <= tau3, the
//     breakpoints of a unit-height trapezoid T(a);
//   axial: the top and bottom centres (k +- 1/2) project to rows
//     [b_lo, b_hi], a unit-height rectangle;
//   amplitude: the chord L_j of the voxel along the line from the source
//     through its centre;
//   a_ij = L_j * int_{a_i - 1/2}^{a_i + 1/2} T * |[b_lo, b_hi] cap [b_i - 1/2, b_i + 1/2]|.
// Every thread owns a column of K voxels along z and walks the views (the
// forward scatter picks the column per view, see sf_fwd_kernel); per
// voxel-view it visits the footprint's pixel window (clipped to the
// detector).  The forward projection scatters a_ij mu_j with FP32 atomics;
// the back-projection and both gradients gather, so they are deterministic.
//
// Forward gradient: s_j = sum_i a_ij dL/dl_i, then the ray kernel's nine
// sums B_c = sum s_j G_c(j), T_ac = sum s_j (I_a - centre_a) G_c(j) with the
// central-difference gradient in index units; the ray kernel's FP64
// finalize turns them into dL/dtheta.
// Back-projection gradient: d_j = sum_i a_ij (l_a, l_b)_i (central
// differences at the pixel centres), then the voxel kernel's twelve sums
// with c = (d_a, d_b, -(d_a a' + d_b b')) e_j / w' (a', b', w' of the voxel
// centre), finalized by the voxel kernel's FP64 finalize.
#include <cmath>

#include "dp_internal.h"

namespace dp {

constexpr int kSfBx = 64, kSfBy = 4, kSfCol = 8;
constexpr int kFpSF = DP_FP_SF, kFpDD = DP_FP_DD;

struct SfFootprint {
    double tau[4];
    double blo, bhi;
    double L;
    int a0, a1, b0, b1;  // pixel window (inclusive), clipped; empty if a0 > a1 or b0 > b1
};

__device__ inline double trap_cdf(double x, const double* t)
{
    double s = 0.0;
    if (x > t[0] && t[1] > t[0]) {
        const double xr = fmin(x, t[1]);
        s += (xr - t[0]) * (xr - t[0]) / (2.0 * (t[1] - t[0]));
    }
    if (x > t[1]) s += fmin(x, t[2]) - t[1];
    if (x > t[2] && t[3] > t[2]) {
        const double xf = fmin(x, t[3]);
        s += ((t[3] - t[2]) * (t[3] - t[2]) - (t[3] - xf) * (t[3] - xf)) / (2.0 * (t[3] - t[2]));
    }
    return s;
}

__device__ inline double row_overlap(int b, double lo, double hi)
{
    const double o = fmin(b + 0.5, hi) - fmax(b - 0.5, lo);
    return o > 0.0 ? o : 0.0;
}

// Footprint of voxel (i, j, k) in view g; false if any projected point lies
// at or behind the source plane.  src: the source in object-frame index
// units; dom: DD's dominant axis of the view (0 = x, 1 = y).
template <int KIND>
__device__ inline bool sf_footprint(const ViewGeo& g, const GeoScalars& s, const double* src,
                                    int dom, int i, int j, int k, SfFootprint& f)
{
    const double fi = i, fj = j, fk = k;
    const double U0 = fma(g.PUd[0], fi, fma(g.PUd[1], fj, fma(g.PUd[2], fk, g.PUd[3])));
    const double V0 = fma(g.PVd[0], fi, fma(g.PVd[1], fj, fma(g.PVd[2], fk, g.PVd[3])));
    const double W0 = fma(g.PWd[0], fi, fma(g.PWd[1], fj, fma(g.PWd[2], fk, g.PWd[3])));
    double t[4];
    if (KIND == kFpSF) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double dx = (c & 1) ? 0.5 : -0.5, dy = (c & 2) ? 0.5 : -0.5;
            const double U = fma(g.PUd[0], dx, fma(g.PUd[1], dy, U0));
            const double W = fma(g.PWd[0], dx, fma(g.PWd[1], dy, W0));
            if (!(W > 0.0)) return false;
            t[c] = U / W + s.cu;
        }
        // sort the four breakpoints (5 compare-exchanges)
#define DP_CX(p, q)                                                  \
    {                                                                \
        const double lo_ = fmin(t[p], t[q]), hi_ = fmax(t[p], t[q]); \
        t[p] = lo_;                                                  \
        t[q] = hi_;                                                  \
    }
        DP_CX(0, 1) DP_CX(2, 3) DP_CX(0, 2) DP_CX(1, 3) DP_CX(1, 2)
#undef DP_CX
    } else {
        double e[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const double off = c ? 0.5 : -0.5;
            const int ax = dom == 0 ? 1 : 0;  // boundaries across the other transaxial axis
            const double U = fma(g.PUd[ax], off, U0), W = fma(g.PWd[ax], off, W0);
            if (!(W > 0.0)) return false;
            e[c] = U / W + s.cu;
        }
        t[0] = t[1] = fmin(e[0], e[1]);
        t[2] = t[3] = fmax(e[0], e[1]);
    }
    double bb[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double dz = c ? 0.5 : -0.5;
        const double V = fma(g.PVd[2], dz, V0), W = fma(g.PWd[2], dz, W0);
        if (!(W > 0.0)) return false;
        bb[c] = V / W + s.cv;
    }
    for (int c = 0; c < 4; ++c) f.tau[c] = t[c];
    f.blo = fmin(bb[0], bb[1]);
    f.bhi = fmax(bb[0], bb[1]);
    // amplitude from d, the line from the source to the centre (mm):
    // SF the chord min_a h_a |d| / |d_a|, DD the slab path h_dom |d| / |d_dom|
    const double h[3] = {s.vx, s.vy, s.vz};
    const double d[3] = {(fi - src[0]) * h[0], (fj - src[1]) * h[1], (fk - src[2]) * h[2]};
    const double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double L;
    if (KIND == kFpSF) {
        L = INFINITY;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (d[c] != 0.0) L = fmin(L, h[c] * n / fabs(d[c]));
    } else {
        L = d[dom] != 0.0 ? h[dom] * n / fabs(d[dom]) : 0.0;
    }
    f.L = L;
    // window, clamped in FP64 before the integer conversion
    f.a0 = (int)fmax(floor(t[0] - 0.5) + 1.0, 0.0);
    f.a1 = (int)fmin(ceil(t[3] + 0.5) - 1.0, (double)(s.nu - 1));
    f.b0 = (int)fmax(floor(f.blo - 0.5) + 1.0, 0.0);
    f.b1 = (int)fmin(ceil(f.bhi + 0.5) - 1.0, (double)(s.nv - 1));
    return true;
}

__device__ inline double sf_col_weight(const SfFootprint& f, int a)
{
    return trap_cdf(a + 0.5, f.tau) - trap_cdf(a - 0.5, f.tau);
}

// Source position in object-frame (unpadded) voxel-index units, and the
// view's dominant transaxial axis for DD (0 = x, 1 = y).
__device__ inline int sf_source(const ViewGeo& g, const GeoScalars& s, double* src)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) src[c] = g.OT[c] - kPadV - s.sad * g.EW[c];
    const double ox = (src[0] - 0.5 * (s.nx - 1)) * s.vx, oy = (src[1] - 0.5 * (s.ny - 1)) * s.vy;
    return fabs(ox) >= fabs(oy) ? 0 : 1;
}

// Gather sum_i a_ij img_i over the footprint (img: [nv][nu]).
__device__ inline double sf_gather(const SfFootprint& f, const float* __restrict__ img, int nu)
{
    double acc = 0.0;
    for (int b = f.b0; b <= f.b1; ++b) {
        const double wb = row_overlap(b, f.blo, f.bhi);
        if (wb == 0.0) continue;
        double row = 0.0;
        for (int a = f.a0; a <= f.a1; ++a) row += sf_col_weight(f, a) * (double)img[(size_t)b * nu + a];
        acc += wb * row;
    }
    return f.L * acc;
}

// Forward scatter.  A wavefront's 64 lanes take 64 neighbouring voxels
// across the view's rays, not along them: lanes along y when the rays run
// closest to the x axis (DD's dominant axis 0), along x otherwise, so their
// footprints cover neighbouring pixels instead of all landing on the same
// ones (their FP32 atomics would serialise).  The flat block index covers
// both tilings of the (x, y) plane; each block decodes it per view.
template <int KIND>
__global__ __launch_bounds__(kSfBx * kSfBy) void sf_fwd_kernel(GeoScalars s, int V,
                                                               const ViewGeo* __restrict__ views,
                                                               const float* __restrict__ vol,
                                                               float* __restrict__ proj)
{
    const int kb = blockIdx.z * kSfCol;
    const int bxx = (s.nx + kSfBx - 1) / kSfBx, byx = (s.ny + kSfBy - 1) / kSfBy;  // lanes along x
    const int bxy = (s.ny + kSfBx - 1) / kSfBx, byy = (s.nx + kSfBy - 1) / kSfBy;  // lanes along y
    const int blk = blockIdx.x;
    for (int v = 0; v < V; ++v) {
        const ViewGeo& g = views[v];
        double src[3];
        const int dom = sf_source(g, s, src);
        int i, j;
        if (dom == 0) {
            if (blk >= bxy * byy) continue;
            j = (blk % bxy) * kSfBx + (int)threadIdx.x;
            i = (blk / bxy) * kSfBy + (int)threadIdx.y;
        } else {
            if (blk >= bxx * byx) continue;
            i = (blk % bxx) * kSfBx + (int)threadIdx.x;
            j = (blk / bxx) * kSfBy + (int)threadIdx.y;
        }
        if (i >= s.nx || j >= s.ny) continue;
        float* img = proj + (size_t)v * s.nu * s.nv;
        for (int kk = 0; kk < kSfCol && kb + kk < s.nz; ++kk) {
            const int k = kb + kk;
            const float mu = vol[((size_t)k * s.ny + j) * s.nx + i];
            if (mu == 0.0f) continue;
            SfFootprint f;
            if (!sf_footprint<KIND>(g, s, src, dom, i, j, k, f)) continue;
            for (int b = f.b0; b <= f.b1; ++b) {
                const double wb = row_overlap(b, f.blo, f.bhi) * f.L * (double)mu;
                if (wb == 0.0) continue;
                for (int a = f.a0; a <= f.a1; ++a) {
                    const double w = wb * sf_col_weight(f, a);
                    if (w != 0.0) atomicAdd(img + (size_t)b * s.nu + a, (float)w);
                }
            }
        }
    }
}

template <int KIND>
__global__ __launch_bounds__(kSfBx * kSfBy) void sf_bp_kernel(GeoScalars s, int V,
                                                              const ViewGeo* __restrict__ views,
                                                              const float* __restrict__ proj,
                                                              float* __restrict__ vol)
{
    const int i = blockIdx.x * kSfBx + threadIdx.x;
    const int j = blockIdx.y * kSfBy + threadIdx.y;
    const int kb = blockIdx.z * kSfCol;
    if (i >= s.nx || j >= s.ny) return;
    double acc[kSfCol];
#pragma unroll
    for (int kk = 0; kk < kSfCol; ++kk) acc[kk] = 0.0;
    for (int v = 0; v < V; ++v) {
        const ViewGeo& g = views[v];
        double src[3];
        const int dom = sf_source(g, s, src);
        const float* img = proj + (size_t)v * s.nu * s.nv;
#pragma unroll
        for (int kk = 0; kk < kSfCol; ++kk) {
            if (kb + kk >= s.nz) break;
            SfFootprint f;
            if (sf_footprint<KIND>(g, s, src, dom, i, j, kb + kk, f)) acc[kk] += sf_gather(f, img, s.nu);
        }
    }
#pragma unroll
    for (int kk = 0; kk < kSfCol; ++kk)
        if (kb + kk < s.nz) vol[((size_t)(kb + kk) * s.ny + j) * s.nx + i] = (float)acc[kk];
}

// Per-view block reduction of C channels into partials[v][blk][C] (fixed
// order: wavefront butterflies, then the 4 wavefronts in sequence).
template <int C>
__device__ inline void sf_reduce_store(float (&r)[C], float (&red)[kSfBy][C], float* out)
{
    const int lane = threadIdx.x, wave = threadIdx.y;
#pragma unroll
    for (int ch = 0; ch < C; ++ch)
        for (int off = 32; off > 0; off >>= 1) r[ch] += __shfl_xor(r[ch], off);
    if (lane == 0) {
#pragma unroll
        for (int ch = 0; ch < C; ++ch) red[wave][ch] = r[ch];
    }
    __syncthreads();
    if (wave == 0 && lane < C) out[lane] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    __syncthreads();
}

__device__ inline float vol_at(const float* __restrict__ v, const GeoScalars& s, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= s.nx || j >= s.ny || k >= s.nz) return 0.0f;
    return v[((size_t)k * s.ny + j) * s.nx + i];
}

template <int KIND>
__global__ __launch_bounds__(kSfBx * kSfBy) void sf_fwd_grad_kernel(GeoScalars s, int V,
                                                                    const ViewGeo* __restrict__ views,
                                                                    const float* __restrict__ vol,
                                                                    const float* __restrict__ grad_proj,
                                                                    float* __restrict__ partials)
{
    __shared__ float red[kSfBy][kRdChannels];
    const int i = blockIdx.x * kSfBx + threadIdx.x;
    const int j = blockIdx.y * kSfBy + threadIdx.y;
    const int kb = blockIdx.z * kSfCol;
    const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    const bool active = i < s.nx && j < s.ny;
    // central-difference gradient (index units: half the neighbour difference)
    float G[kSfCol][3];
#pragma unroll
    for (int kk = 0; kk < kSfCol; ++kk) {
        const int k = kb + kk;
        const bool in = active && k < s.nz;
        G[kk][0] = in ? 0.5f * (vol_at(vol, s, i + 1, j, k) - vol_at(vol, s, i - 1, j, k)) : 0.0f;
        G[kk][1] = in ? 0.5f * (vol_at(vol, s, i, j + 1, k) - vol_at(vol, s, i, j - 1, k)) : 0.0f;
        G[kk][2] = in ? 0.5f * (vol_at(vol, s, i, j, k + 1) - vol_at(vol, s, i, j, k - 1)) : 0.0f;
    }
    const float pi = (float)i - 0.5f * (s.nx - 1), pj = (float)j - 0.5f * (s.ny - 1);
    for (int v = 0; v < V; ++v) {
        const ViewGeo& g = views[v];
        double src[3];
        const int dom = sf_source(g, s, src);
        const float* w = grad_proj + (size_t)v * s.nu * s.nv;
        float r[kRdChannels];
#pragma unroll
        for (int ch = 0; ch < kRdChannels; ++ch) r[ch] = 0.0f;
        if (active) {
#pragma unroll
            for (int kk = 0; kk < kSfCol; ++kk) {
                const int k = kb + kk;
                if (k >= s.nz) break;
                if (G[kk][0] == 0.0f && G[kk][1] == 0.0f && G[kk][2] == 0.0f) continue;
                SfFootprint f;
                if (!sf_footprint<KIND>(g, s, src, dom, i, j, k, f)) continue;
                const float sj = (float)sf_gather(f, w, s.nu);
                const float pk = (float)k - 0.5f * (s.nz - 1);
                const float gx = sj * G[kk][0], gy = sj * G[kk][1], gz = sj * G[kk][2];
                // B_c, then T_xy, T_xz, T_yx, T_yz, T_zx, T_zy (T_ac = sum s P_a G_c)
                r[0] += gx; r[1] += gy; r[2] += gz;
                r[3] = fmaf(pi, gy, r[3]); r[4] = fmaf(pi, gz, r[4]);
                r[5] = fmaf(pj, gx, r[5]); r[6] = fmaf(pj, gz, r[6]);
                r[7] = fmaf(pk, gx, r[7]); r[8] = fmaf(pk, gy, r[8]);
            }
        }
        sf_reduce_store<kRdChannels>(r, red, partials + ((size_t)v * nblk + blk) * kRdChannels);
    }
}

template <int KIND>
__global__ __launch_bounds__(kSfBx * kSfBy) void sf_bp_grad_kernel(GeoScalars s, int V,
                                                                   const ViewGeo* __restrict__ views,
                                                                   const float4* __restrict__ proj4,
                                                                   const float* __restrict__ grad_vol,
                                                                   float* __restrict__ partials)
{
    __shared__ float red[kSfBy][kVdChannels];
    const int i = blockIdx.x * kSfBx + threadIdx.x;
    const int j = blockIdx.y * kSfBy + threadIdx.y;
    const int kb = blockIdx.z * kSfCol;
    const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    const bool active = i < s.nx && j < s.ny;
    const int NU = s.nu + 2 * kPadD, NV = s.nv + 2 * kPadD;
    float e[kSfCol];
#pragma unroll
    for (int kk = 0; kk < kSfCol; ++kk)
        e[kk] = (active && kb + kk < s.nz) ? grad_vol[((size_t)(kb + kk) * s.ny + j) * s.nx + i] : 0.0f;
    const float pi = (float)i - 0.5f * (s.nx - 1), pj = (float)j - 0.5f * (s.ny - 1);
    for (int v = 0; v < V; ++v) {
        const ViewGeo& g = views[v];
        double src[3];
        const int dom = sf_source(g, s, src);
        const float4* img = proj4 + (size_t)v * NU * NV;
        float A1 = 0.f, A2 = 0.f, A3 = 0.f, Z1 = 0.f, Z2 = 0.f, Z3 = 0.f;
#pragma unroll
        for (int kk = 0; kk < kSfCol; ++kk) {
            const int k = kb + kk;
            if (k >= s.nz || e[kk] == 0.0f) continue;
            SfFootprint f;
            if (!sf_footprint<KIND>(g, s, src, dom, i, j, k, f)) continue;
            double da = 0.0, db = 0.0;
            for (int b = f.b0; b <= f.b1; ++b) {
                const double wb = row_overlap(b, f.blo, f.bhi);
                if (wb == 0.0) continue;
                for (int a = f.a0; a <= f.a1; ++a) {
                    const double wgt = wb * sf_col_weight(f, a);
                    const float4 p = img[(size_t)(b + kPadD) * NU + (a + kPadD)];
                    da += wgt * (double)p.y;
                    db += wgt * (double)p.z;
                }
            }
            da *= f.L;
            db *= f.L;
            // projection of the voxel centre: offsets from the detector centre, depth
            const double fi = i, fj = j, fk = k;
            const double U = fma(g.PUd[0], fi, fma(g.PUd[1], fj, fma(g.PUd[2], fk, g.PUd[3])));
            const double Vv = fma(g.PVd[0], fi, fma(g.PVd[1], fj, fma(g.PVd[2], fk, g.PVd[3])));
            const double W = fma(g.PWd[0], fi, fma(g.PWd[1], fj, fma(g.PWd[2], fk, g.PWd[3])));
            const double ec = (double)e[kk] / W;
            const float c1 = (float)(ec * da), c2 = (float)(ec * db);
            const float c3 = (float)(-ec * (da * (U / W) + db * (Vv / W)));
            const float pk = (float)k - 0.5f * (s.nz - 1);
            A1 += c1; A2 += c2; A3 += c3;
            Z1 = fmaf(c1, pk, Z1); Z2 = fmaf(c2, pk, Z2); Z3 = fmaf(c3, pk, Z3);
        }
        float r[kVdChannels] = {A1, A2, A3, pi * A1, pi * A2, pi * A3,
                                pj * A1, pj * A2, pj * A3, Z1, Z2, Z3};
        sf_reduce_store<kVdChannels>(r, red, partials + ((size_t)v * nblk + blk) * kVdChannels);
    }
}

__global__ void sf_zero_kernel(size_t n, float* __restrict__ p)
{
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        p[t] = 0.0f;
}

static dim3 sf_grid(const GeoScalars& s)
{
    return dim3((s.nx + kSfBx - 1) / kSfBx, (s.ny + kSfBy - 1) / kSfBy, (s.nz + kSfCol - 1) / kSfCol);
}

int sf_blocks(const GeoScalars& s)
{
    const dim3 g = sf_grid(s);
    return (int)(g.x * g.y * g.z);
}

#define DP_FP_LAUNCH(KERNEL, ...)                                                           \
    do {                                                                                    \
        if (kind == kFpDD)                                                                  \
            KERNEL<kFpDD><<<sf_grid(s), dim3(kSfBx, kSfBy), 0, st>>>(__VA_ARGS__);          \
        else                                                                                \
            KERNEL<kFpSF><<<sf_grid(s), dim3(kSfBx, kSfBy), 0, st>>>(__VA_ARGS__);          \
    } while (0)

void launch_sf_fwd(const GeoScalars& s, int V, const ViewGeo* views, const float* vol, float* proj,
                   int kind, hipStream_t st)
{
    const size_t n = (size_t)V * s.nu * s.nv;
    const int zb = (int)std::min<size_t>((n + 255) / 256, 65536);
    // flat (x, y) block index large enough for either lane order
    const int bx = std::max(((s.nx + kSfBx - 1) / kSfBx) * ((s.ny + kSfBy - 1) / kSfBy),
                            ((s.ny + kSfBx - 1) / kSfBx) * ((s.nx + kSfBy - 1) / kSfBy));
    const dim3 grid(bx, 1, (s.nz + kSfCol - 1) / kSfCol);
    prof_begin(DP_K_SF, st);
    sf_zero_kernel<<<zb, 256, 0, st>>>(n, proj);
    if (kind == kFpDD)
        sf_fwd_kernel<kFpDD><<<grid, dim3(kSfBx, kSfBy), 0, st>>>(s, V, views, vol, proj);
    else
        sf_fwd_kernel<kFpSF><<<grid, dim3(kSfBx, kSfBy), 0, st>>>(s, V, views, vol, proj);
    prof_end(DP_K_SF, st);
}

void launch_sf_bp(const GeoScalars& s, int V, const ViewGeo* views, const float* proj, float* vol,
                  int kind, hipStream_t st)
{
    prof_begin(DP_K_SF, st);
    DP_FP_LAUNCH(sf_bp_kernel, s, V, views, proj, vol);
    prof_end(DP_K_SF, st);
}

void launch_sf_fwd_grad(const GeoScalars& s, int V, const ViewGeo* views, const float* vol,
                        const float* grad_proj, float* partials, int kind, hipStream_t st)
{
    prof_begin(DP_K_SF, st);
    DP_FP_LAUNCH(sf_fwd_grad_kernel, s, V, views, vol, grad_proj, partials);
    prof_end(DP_K_SF, st);
}

void launch_sf_bp_grad(const GeoScalars& s, int V, const ViewGeo* views, const float4* proj4,
                       const float* grad_vol, float* partials, int kind, hipStream_t st)
{
    prof_begin(DP_K_SF, st);
    DP_FP_LAUNCH(sf_bp_grad_kernel, s, V, views, proj4, grad_vol, partials);
    prof_end(DP_K_SF, st);
}
#undef DP_FP_LAUNCH

}  // namespace dp
