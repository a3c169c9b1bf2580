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
// view's projective map on voxel indices; FP64 anchors per voxel column and
// view, exact FP32 offsets per voxel, see SfColumn):
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

// Footprint of one voxel in one view, in FP32 pixel coordinates relative
// to an integer base pixel (abase, bbase), so that breakpoints of magnitude
// ~1e3 pixels keep ~1e-6 pixel resolution.
struct SfFootprint {
    float tau[4];     // trapezoid breakpoints (column), relative to abase
    float r01, r23;   // 1 / (2 (tau1 - tau0)), 1 / (2 (tau3 - tau2)); 0 for a vertical edge
    float blo, bhi;   // row rectangle, relative to bbase
    float L;          // amplitude
    int abase, bbase;
    int a0, a1, b0, b1;  // pixel window (inclusive, absolute), clipped; empty if a0 > a1 or b0 > b1
};

constexpr double kSfPixClamp = 1048576.0;  // projections beyond 2^20 pixels are off any detector

// Integral of the unit-height trapezoid over [x0, x1] (relative to abase),
// segment by segment: rising edge (x - t0) / (t1 - t0), plateau, falling
// edge (t3 - x) / (t3 - t2).  Each term is a product of short differences,
// so no digits are lost when breakpoints lie far from the cell.
__device__ inline float trap_integral(float x0, float x1, const SfFootprint& f)
{
    const float* t = f.tau;
    float s = fmaxf(fminf(x1, t[2]) - fmaxf(x0, t[1]), 0.0f);
    if (t[1] > t[0]) {
        const float l = fmaxf(x0, t[0]), r = fminf(x1, t[1]);
        if (r > l) s += (r - l) * ((r - t[0]) + (l - t[0])) * f.r01;
    }
    if (t[3] > t[2]) {
        const float l = fmaxf(x0, t[2]), r = fminf(x1, t[3]);
        if (r > l) s += (r - l) * ((t[3] - l) + (t[3] - r)) * f.r23;
    }
    return s;
}

__device__ inline float row_overlap(float b, float lo, float hi)
{
    const float o = fminf(b + 0.5f, hi) - fmaxf(b - 0.5f, lo);
    return o > 0.0f ? o : 0.0f;
}

// The parts every producer shares: sort (SF), slopes, amplitude, window.
// t: column breakpoints (SF: four corners; DD: the two boundaries in t[0],
// t[1]), bb: the two row bounds, both relative to the bases; d: the line
// from the source to the voxel centre (mm).
template <int KIND>
__device__ inline void sf_finish(const GeoScalars& s, int dom, float* t, const float* bb,
                                 const float* d, int abase, int bbase, SfFootprint& f)
{
    if (KIND == kFpSF) {
#define DP_CX(p, q)                                                  \
    {                                                                \
        const float lo_ = fminf(t[p], t[q]), hi_ = fmaxf(t[p], t[q]); \
        t[p] = lo_;                                                  \
        t[q] = hi_;                                                  \
    }
        DP_CX(0, 1) DP_CX(2, 3) DP_CX(0, 2) DP_CX(1, 3) DP_CX(1, 2)
#undef DP_CX
    } else {
        const float lo = fminf(t[0], t[1]), hi = fmaxf(t[0], t[1]);
        t[0] = t[1] = lo;
        t[2] = t[3] = hi;
    }
    for (int c = 0; c < 4; ++c) f.tau[c] = t[c];
    // reciprocals to ~1 ulp (hardware rcp): every quantity here needs only
    // relative precision
    f.r01 = t[1] > t[0] ? 0.5f * __builtin_amdgcn_rcpf(t[1] - t[0]) : 0.0f;
    f.r23 = t[3] > t[2] ? 0.5f * __builtin_amdgcn_rcpf(t[3] - t[2]) : 0.0f;
    f.blo = fminf(bb[0], bb[1]);
    f.bhi = fmaxf(bb[0], bb[1]);
    // amplitude: SF the chord min_a h_a |d| / |d_a|, DD the slab path
    // h_dom |d| / |d_dom|; it scales the weights, so FP32 is enough
    const float h[3] = {(float)s.vx, (float)s.vy, (float)s.vz};
    const float n = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    float L;
    if (KIND == kFpSF) {
        L = INFINITY;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (d[c] != 0.0f) L = fminf(L, h[c] * n * __builtin_amdgcn_rcpf(fabsf(d[c])));
    } else {
        L = d[dom] != 0.0f ? h[dom] * n * __builtin_amdgcn_rcpf(fabsf(d[dom])) : 0.0f;
    }
    f.L = L;
    f.abase = abase;
    f.bbase = bbase;
    // window (the bases and relative offsets are bounded, so no overflow)
    f.a0 = max(abase + (int)floorf(t[0] - 0.5f) + 1, 0);
    f.a1 = min(abase + (int)ceilf(t[3] + 0.5f) - 1, s.nu - 1);
    f.b0 = max(bbase + (int)floorf(f.blo - 0.5f) + 1, 0);
    f.b1 = min(bbase + (int)ceilf(f.bhi + 0.5f) - 1, s.nv - 1);
}

// Column breakpoint line q of voxel column (i, j): SF corner (i +- 1/2,
// j +- 1/2), DD boundary across the non-dominant transaxial axis.
template <int KIND>
__device__ inline void sf_line(int q, int dom, double& dx, double& dy)
{
    if (KIND == kFpSF) {
        dx = (q & 1) ? 0.5 : -0.5;
        dy = (q & 2) ? 0.5 : -0.5;
    } else {
        const double off = q ? 0.5 : -0.5;
        dx = dom == 0 ? 0.0 : off;  // dom x: boundaries across y
        dy = dom == 0 ? off : 0.0;
    }
}

// Per-voxel FP64 footprint of voxel (i, j, k) in view g; false if any
// projected point lies at or behind the source plane.  src: the source in
// object-frame index units; dom: DD's dominant axis of the view.
template <int KIND>
__device__ inline bool sf_footprint(const ViewGeo& g, const GeoScalars& s, const double* src,
                                    int dom, int i, int j, int k, SfFootprint& f)
{
    const double fi = i, fj = j, fk = k;
    const double U0 = fma(g.PUd[0], fi, fma(g.PUd[1], fj, fma(g.PUd[2], fk, g.PUd[3])));
    const double V0 = fma(g.PVd[0], fi, fma(g.PVd[1], fj, fma(g.PVd[2], fk, g.PVd[3])));
    const double W0 = fma(g.PWd[0], fi, fma(g.PWd[1], fj, fma(g.PWd[2], fk, g.PWd[3])));
    constexpr int NL = KIND == kFpSF ? 4 : 2;
    double td[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        double dx, dy;
        sf_line<KIND>(q, dom, dx, dy);
        const double U = fma(g.PUd[0], dx, fma(g.PUd[1], dy, U0));
        const double W = fma(g.PWd[0], dx, fma(g.PWd[1], dy, W0));
        if (!(W > 0.0)) return false;
        td[q] = fmin(fmax(U / W + s.cu, -kSfPixClamp), kSfPixClamp);
    }
    double bd[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double dz = c ? 0.5 : -0.5;
        const double V = fma(g.PVd[2], dz, V0), W = fma(g.PWd[2], dz, W0);
        if (!(W > 0.0)) return false;
        bd[c] = fmin(fmax(V / W + s.cv, -kSfPixClamp), kSfPixClamp);
    }
    const double ab = floor(td[0]), bbv = floor(bd[0]);
    float t[4], bb[2];
#pragma unroll
    for (int q = 0; q < NL; ++q) t[q] = (float)(td[q] - ab);
    bb[0] = (float)(bd[0] - bbv);
    bb[1] = (float)(bd[1] - bbv);
    const float d[3] = {(float)((fi - src[0]) * s.vx), (float)((fj - src[1]) * s.vy),
                        (float)((fk - src[2]) * s.vz)};
    sf_finish<KIND>(s, dom, t, bb, d, (int)ab, (int)bbv, f);
    return true;
}

// FP64 anchors of voxel column (i, j) at height ka for one view.  Along the
// column each breakpoint line and the centre line move only in z, so with
// U(dk) = U0 + dk P_uz and W(dk) = W0 + dk P_wz the projection is exactly
//   U(dk) / W(dk) = U0 / W0 + dk N / W(dk),   N = (P_uz W0 - P_wz U0) / W0,
// and only the small offset dk N / W(dk) is evaluated per voxel, in FP32.
struct SfColumn {
    bool fast;       // false: an anchor within 1 mm of the source plane (per-voxel FP64)
    int abase, bbase;
    float tfr[4], tn[4], tw[4];  // breakpoint lines: anchor offset from abase, N, W0
    float bfr, bn, bw;           // centre line: row offset from bbase, N_v, W0
    float ucfr, ucn;             // centre line: column offset from abase, N_u
    float uco, bco;              // abase - c_u, bbase - c_v (offsets from the detector centre)
    float pwz, ka;
    float d0, d1, d2o;           // source-to-voxel line: x, y (mm) and z offset
};

template <int KIND>
__device__ inline SfColumn sf_column(const ViewGeo& g, const GeoScalars& s, const double* src,
                                     int dom, int i, int j, int ka)
{
    SfColumn c;
    c.fast = false;
    const double fi = i, fj = j, fk = ka;
    constexpr int NL = KIND == kFpSF ? 4 : 2;
    double A[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        double dx, dy;
        sf_line<KIND>(q, dom, dx, dy);
        const double U = fma(g.PUd[0], fi + dx, fma(g.PUd[1], fj + dy, fma(g.PUd[2], fk, g.PUd[3])));
        const double W = fma(g.PWd[0], fi + dx, fma(g.PWd[1], fj + dy, fma(g.PWd[2], fk, g.PWd[3])));
        if (!(W >= 1.0)) return c;
        const double iw = 1.0 / W;
        A[q] = fmin(fmax(U * iw + s.cu, -kSfPixClamp), kSfPixClamp);
        c.tn[q] = (float)((g.PUd[2] * W - g.PWd[2] * U) * iw);
        c.tw[q] = (float)W;
    }
    const double Uc = fma(g.PUd[0], fi, fma(g.PUd[1], fj, fma(g.PUd[2], fk, g.PUd[3])));
    const double V = fma(g.PVd[0], fi, fma(g.PVd[1], fj, fma(g.PVd[2], fk, g.PVd[3])));
    const double W = fma(g.PWd[0], fi, fma(g.PWd[1], fj, fma(g.PWd[2], fk, g.PWd[3])));
    if (!(W >= 1.0)) return c;
    const double iw = 1.0 / W;
    const double B = fmin(fmax(V * iw + s.cv, -kSfPixClamp), kSfPixClamp);
    const double Ac = fmin(fmax(Uc * iw + s.cu, -kSfPixClamp), kSfPixClamp);
    c.bn = (float)((g.PVd[2] * W - g.PWd[2] * V) * iw);
    c.ucn = (float)((g.PUd[2] * W - g.PWd[2] * Uc) * iw);
    c.bw = (float)W;
    const double ab = floor(A[0]), bb = floor(B);
    c.abase = (int)ab;
    c.bbase = (int)bb;
#pragma unroll
    for (int q = 0; q < NL; ++q) c.tfr[q] = (float)(A[q] - ab);
    c.bfr = (float)(B - bb);
    c.ucfr = (float)(Ac - ab);
    c.uco = (float)(ab - s.cu);
    c.bco = (float)(bb - s.cv);
    c.pwz = (float)g.PWd[2];
    c.ka = (float)ka;
    c.d0 = (float)((fi - src[0]) * s.vx);
    c.d1 = (float)((fj - src[1]) * s.vy);
    c.d2o = (float)(-src[2] * s.vz);
    c.fast = true;
    return c;
}

// Footprint of voxel (i, j, k) from its column's anchors (FP32), falling
// back to the per-voxel FP64 footprint when the column has no safe anchor.
template <int KIND>
__device__ inline bool sf_voxel(const SfColumn& c, const ViewGeo& g, const GeoScalars& s,
                                const double* src, int dom, int i, int j, int k, SfFootprint& f)
{
    if (!c.fast) return sf_footprint<KIND>(g, s, src, dom, i, j, k, f);
    constexpr int NL = KIND == kFpSF ? 4 : 2;
    const float dk = (float)k - c.ka;
    float t[4] = {0.f, 0.f, 0.f, 0.f}, bb[2];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const float W = fmaf(dk, c.pwz, c.tw[q]);
        if (!(W > 0.0f)) return false;
        t[q] = fmaf(dk * c.tn[q], __builtin_amdgcn_rcpf(W), c.tfr[q]);  // offset <~ 10 px
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dz = dk + (e ? 0.5f : -0.5f);
        const float W = fmaf(dz, c.pwz, c.bw);
        if (!(W > 0.0f)) return false;
        bb[e] = fmaf(dz * c.bn, __builtin_amdgcn_rcpf(W), c.bfr);
    }
    const float d[3] = {c.d0, c.d1, fmaf((float)k, (float)s.vz, c.d2o)};
    sf_finish<KIND>(s, dom, t, bb, d, c.abase, c.bbase, f);
    return true;
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

// The footprint's pixels column by column: fn(a, b, w) for every pixel of
// the window with a non-zero weight w = column integral x row overlap
// (without the amplitude L); the column integral is evaluated once per
// column.
template <typename Fn>
__device__ inline void sf_for_each(const SfFootprint& f, Fn&& fn)
{
    for (int a = f.a0; a <= f.a1; ++a) {
        const float x = (float)(a - f.abase);
        const float wa = trap_integral(x - 0.5f, x + 0.5f, f);
        if (wa == 0.0f) continue;
        for (int b = f.b0; b <= f.b1; ++b) {
            const float wb = row_overlap((float)(b - f.bbase), f.blo, f.bhi);
            if (wb != 0.0f) fn(a, b, wa * wb);
        }
    }
}

// Gather sum_i a_ij img_i over the footprint (img: [nv][nu]).
__device__ inline float sf_gather(const SfFootprint& f, const float* __restrict__ img, int nu)
{
    float acc = 0.0f;
    sf_for_each(f, [&](int a, int b, float w) { acc = fmaf(w, img[(size_t)b * nu + a], acc); });
    return f.L * acc;
}

// Forward scatter.  A wavefront's 64 lanes take 64 neighbouring voxels
// across the view's rays, not along them: lanes along y when the rays run
// closest to the x axis (DD's dominant axis 0), along x otherwise, so their
// footprints cover neighbouring pixels instead of all landing on the same
// ones (their FP32 atomics would serialise).  The flat block index covers
// both tilings of the (x, y) plane; each block decodes it per view.
template <int KIND>
__global__ __launch_bounds__(kSfBx * kSfBy, 5) void sf_fwd_kernel(GeoScalars s, int V,
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
        const SfColumn col = sf_column<KIND>(g, s, src, dom, i, j, kb + kSfCol / 2);
        for (int kk = 0; kk < kSfCol && kb + kk < s.nz; ++kk) {
            const int k = kb + kk;
            const float mu = vol[((size_t)k * s.ny + j) * s.nx + i];
            if (mu == 0.0f) continue;
            SfFootprint f;
            if (!sf_voxel<KIND>(col, g, s, src, dom, i, j, k, f)) continue;
            const float scale = f.L * mu;
            sf_for_each(f, [&](int a, int b, float w) {
                atomicAdd(img + (size_t)b * s.nu + a, w * scale);
            });
        }
    }
}

template <int KIND>
__global__ __launch_bounds__(kSfBx * kSfBy, 4) void sf_bp_kernel(GeoScalars s, int V,
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
        const SfColumn col = sf_column<KIND>(g, s, src, dom, i, j, kb + kSfCol / 2);
#pragma unroll
        for (int kk = 0; kk < kSfCol; ++kk) {
            if (kb + kk >= s.nz) break;
            SfFootprint f;
            if (sf_voxel<KIND>(col, g, s, src, dom, i, j, kb + kk, f)) acc[kk] += sf_gather(f, img, s.nu);
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
__global__ __launch_bounds__(kSfBx * kSfBy, KIND == kFpDD ? 4 : 1) void sf_fwd_grad_kernel(GeoScalars s, int V,
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
            const SfColumn col = sf_column<KIND>(g, s, src, dom, i, j, kb + kSfCol / 2);
#pragma unroll
            for (int kk = 0; kk < kSfCol; ++kk) {
                const int k = kb + kk;
                if (k >= s.nz) break;
                if (G[kk][0] == 0.0f && G[kk][1] == 0.0f && G[kk][2] == 0.0f) continue;
                SfFootprint f;
                if (!sf_voxel<KIND>(col, g, s, src, dom, i, j, k, f)) continue;
                const float sj = sf_gather(f, w, s.nu);
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

// Views [v0, v0 + Vc); proj4 holds this chunk's detector gradient images.
template <int KIND>
__global__ __launch_bounds__(kSfBx * kSfBy, KIND == kFpDD ? 4 : 1) void sf_bp_grad_kernel(GeoScalars s, int v0, int Vc,
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
    for (int vv = 0; vv < Vc; ++vv) {
        const int v = v0 + vv;
        const ViewGeo& g = views[v];
        double src[3];
        const int dom = sf_source(g, s, src);
        const float4* img = proj4 + (size_t)vv * NU * NV;
        float A1 = 0.f, A2 = 0.f, A3 = 0.f, Z1 = 0.f, Z2 = 0.f, Z3 = 0.f;
        const SfColumn col = sf_column<KIND>(g, s, src, dom, i, j, kb + kSfCol / 2);
#pragma unroll
        for (int kk = 0; kk < kSfCol; ++kk) {
            const int k = kb + kk;
            if (k >= s.nz || e[kk] == 0.0f) continue;
            SfFootprint f;
            if (!sf_voxel<KIND>(col, g, s, src, dom, i, j, k, f)) continue;
            float da = 0.0f, db = 0.0f;
            sf_for_each(f, [&](int a, int b, float w) {
                const float4 p = img[(size_t)(b + kPadD) * NU + (a + kPadD)];
                da = fmaf(w, p.y, da);
                db = fmaf(w, p.z, db);
            });
            da *= f.L;
            db *= f.L;
            // projection of the voxel centre: offsets from the detector centre (pixels), depth
            float ap, bp, Wc;
            if (col.fast) {
                const float dk = (float)k - col.ka;
                Wc = fmaf(dk, col.pwz, col.bw);
                const float iw = __builtin_amdgcn_rcpf(Wc);
                ap = col.uco + fmaf(dk * col.ucn, iw, col.ucfr);
                bp = col.bco + fmaf(dk * col.bn, iw, col.bfr);
            } else {
                const double fi = i, fj = j, fk = k;
                const double U = fma(g.PUd[0], fi, fma(g.PUd[1], fj, fma(g.PUd[2], fk, g.PUd[3])));
                const double Vv = fma(g.PVd[0], fi, fma(g.PVd[1], fj, fma(g.PVd[2], fk, g.PVd[3])));
                const double W = fma(g.PWd[0], fi, fma(g.PWd[1], fj, fma(g.PWd[2], fk, g.PWd[3])));
                Wc = (float)W;
                ap = (float)(U / W);
                bp = (float)(Vv / W);
            }
            const float ec = e[kk] * __builtin_amdgcn_rcpf(Wc);
            const float c1 = ec * da, c2 = ec * db;
            const float c3 = -ec * fmaf(da, ap, db * bp);
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

void launch_sf_bp_grad(const GeoScalars& s, int v0, int Vc, const ViewGeo* views,
                       const float4* proj4, const float* grad_vol, float* partials, int kind,
                       hipStream_t st)
{
    prof_begin(DP_K_SF, st);
    DP_FP_LAUNCH(sf_bp_grad_kernel, s, v0, Vc, views, proj4, grad_vol, partials);
    prof_end(DP_K_SF, st);
}
#undef DP_FP_LAUNCH

}  // namespace dp
