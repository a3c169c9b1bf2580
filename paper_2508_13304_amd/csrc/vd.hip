// Voxel-driven (FDK-style) back-projector and its rigid-motion gradient.
//
// Back-projection (Eq. back, Sec. II-A; mu^j = sum_i a^ij l^i, Sec. II-C):
// every voxel j is moved by M_v, projected with the projective mapping of
// Eq. projmatrix, and picks up W * bilinear(l_v) at its projection, with
// W = 1 (plain) or (D / depth)^2 (FDK weight).
//
// Gradient (Eqs. back_derive / final_back / back_int / dis_back): per
// voxel-view, G_b = grad_d l^T grad_r p grad_M r is back-projected with the
// same bilinear weights and weighted by dL/dmu.  With the Jacobian rows of
// p(r), (P_k w' - P_3 u'_k) / w'^2, the world-frame gradient of one
// contribution is
//   g_r = (W / w') [ l_a (S/du) e_u + l_b (S/dv) e_v - (l_a a' + l_b b' + kappa l) e_w ]
// (a', b' pixel offsets from the detector centre; kappa = 2 carries the
// product-rule term l grad_r W of the FDK weight, 0 without weight).  Since
// grad_M r = [p^T, 1] per row, dL/dM needs only
//   A_k = sum e c_k      and   Q_k = sum e c_k (I - centre)   (k = u, v, w)
// with g_r = sum_k c_k E_k; each thread accumulates them over its voxel
// column and the block reduces them per view (fixed order).
//
// Numerics: each thread owns a column of K voxels along z.  Per view, the
// projection of the column's middle voxel is evaluated in FP64 and split
// into an integer pixel and a fraction; every voxel of the column is then
// placed exactly (no incremental accumulation) by the small FP32 offset
//   a(k) - a(anchor) = dk * N_u / W(k),  N_u = (P_u,z W0 - P_w,z U0) / W0,
// an algebraic identity of the projective division.  The bilinear weights
// thus carry errors of ~1e-6 pixel instead of the ~3e-5 pixel that FP32
// pixel coordinates of magnitude ~500 would carry.
#include <algorithm>

#include "dp_internal.h"

// Voxels per batch of tap loads and the occupancy target (waves per SIMD)
// of the two kernels; measured at 512^3 / 360 views (build-time choices).
#ifndef VD_BP_NB
#define VD_BP_NB 8
#endif
#ifndef VD_GRAD_NB
#define VD_GRAD_NB 2
#endif
#ifndef VD_BP_WPE
#define VD_BP_WPE 3
#endif
#ifndef VD_GRAD_WPE
#define VD_GRAD_WPE 3
#endif

namespace dp {

// Bilinear value from a pixel's cell coefficients (c0, ca, cb, cab) at
// fractional offsets (wa, wb), wab = wa wb.
__device__ inline float cell_value(float c0, float ca, float cb, float cab, float wa, float wb,
                                   float wab)
{
    return fmaf(wab, cab, fmaf(wb, cb, fmaf(wa, ca, c0)));
}

// Largest distance (pixels, per detector axis) from the detector centre at
// which a column's FP64 anchor may project: two detector widths and a margin.
__host__ __device__ inline double anchor_limit(const GeoScalars& s)
{
    return 2.0 * (double)(s.nu > s.nv ? s.nu : s.nv) + 64.0;
}

// FP64 anchor of one voxel column for one view.
struct ColumnAnchor {
    long long off;      // padded-image offset of the anchor pixel (integer part)
    int ai, bi;         // the anchor pixel's padded column and row
    float a0f, b0f;     // fractional part of the anchor's pixel coordinates
    float nu, nv;       // N_u, N_v of the offset formula
    float w0;           // depth of the anchor voxel (mm)
    float ka;           // anchor position in the column
    float alo, ahi, blo, bhi;  // safe window of the padded image, relative to the anchor
    float apc, bpc;     // anchor offsets from the detector centre (pixels)
    bool exact;         // no usable anchor: project every voxel in FP64 instead
};

__device__ inline ColumnAnchor column_anchor(const ViewGeo& g, const GeoScalars& s, int i, int j,
                                             int kb, int K)
{
    ColumnAnchor c;
    int ka = K / 2;
    const double fi = i, fj = j;
    const double Wij = fma(g.PWd[0], fi, fma(g.PWd[1], fj, g.PWd[3]));
    double W0 = fma(g.PWd[2], (double)(kb + ka), Wij);
    c.exact = false;
    if (!(fabs(W0) >= 1.0)) {
        // anchor within 1 mm of the source plane: move it to the column end
        // farther from that plane (the depth is linear along the column)
        const double Wlo = fma(g.PWd[2], (double)kb, Wij), Whi = fma(g.PWd[2], (double)(kb + K - 1), Wij);
        ka = fabs(Wlo) >= fabs(Whi) ? 0 : K - 1;
        W0 = ka == 0 ? Wlo : Whi;
        if (!(fabs(W0) >= 1.0)) {  // the whole column lies within 1 mm of it
            c.exact = true;
            W0 = 1.0;
        }
    }
    const double fk = kb + ka;
    const double U0 = fma(g.PUd[0], fi, fma(g.PUd[1], fj, fma(g.PUd[2], fk, g.PUd[3])));
    const double V0 = fma(g.PVd[0], fi, fma(g.PVd[1], fj, fma(g.PVd[2], fk, g.PVd[3])));
    const double iw0 = 1.0 / W0;
    const double ap = U0 * iw0, bp = V0 * iw0;
    // an anchor projecting far outside the detector (or a non-finite one) is
    // no reference for the offsets of the other voxels of its column: those
    // that land on the detector would carry FP32 offsets of the anchor's
    // magnitude
    const double lim = anchor_limit(s);
    if (!(fabs(ap) <= lim && fabs(bp) <= lim)) c.exact = true;
    const double a0 = c.exact ? 0.0 : ap + s.cu + kPadD;
    const double b0 = c.exact ? 0.0 : bp + s.cv + kPadD;
    const double A0 = floor(a0), B0 = floor(b0);
    const int NU = s.nu + 2 * kPadD;
    c.off = (long long)B0 * NU + (long long)A0;
    c.ai = (int)A0;
    c.bi = (int)B0;
    c.a0f = (float)(a0 - A0);
    c.b0f = (float)(b0 - B0);
    c.nu = (float)((g.PUd[2] * W0 - g.PWd[2] * U0) * iw0);
    c.nv = (float)((g.PVd[2] * W0 - g.PWd[2] * V0) * iw0);
    c.w0 = (float)W0;
    c.ka = (float)ka;
    // small integers and halves: exact in FP32 (no FP64 constants to keep live)
    const float fA0 = (float)A0, fB0 = (float)B0;
    c.alo = ((float)kPadD - 1.5f) - fA0;
    c.ahi = ((float)(s.nu + kPadD) + 0.5f) - fA0;
    c.blo = ((float)kPadD - 1.5f) - fB0;
    c.bhi = ((float)(s.nv + kPadD) + 0.5f) - fB0;
    c.apc = (float)ap;
    c.bpc = (float)bp;
    return c;
}

// floor(x) as an integer in one VALU instruction (|x| far below 2^31 here).
__device__ inline int floor_to_int(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Window clamp: positions more than half a pixel outside the detector (or
// behind the source) land in the zero border; all others are unchanged.
__device__ inline float clampf(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

// One view's contribution to a column of K voxels.  FRONT: the caller has
// checked that every voxel of the column lies in front of the source (W > 0 at
// both ends of the column, W being linear along it), so no per-voxel test.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const f32x4 global_float4;
typedef __attribute__((address_space(1))) const char global_bytes;

// Byte offset of the tap at pixel offset (ia, ib) from a column's anchor,
// relative to its view's image: col = the anchor's byte offset, row = bytes
// per padded image row, BYTES per pixel.  Two 24-bit multiply-adds (every
// operand is far below 2^23 in magnitude); 32-bit wrap-around is exact since
// the tap itself lies inside the image.
__device__ inline unsigned mad_i24(int a, int b, unsigned c)
{
    unsigned r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

template <int BYTES>
__device__ inline unsigned tap_offset(unsigned col, int ia, int ib, int row)
{
    return mad_i24(ib, row, mad_i24(ia, BYTES, col));
}

// A 16-byte load at a byte offset from a wave-uniform base (the base stays
// in scalar registers; each lane supplies only its 32-bit offset).
__device__ inline f32x4 ld16(global_bytes* base, unsigned off)
{
    return *(global_float4*)(base + off);
}

// The taps of NB consecutive voxels are gathered before any of them is
// used, so NB loads are in flight per wavefront.
template <int MODE, int K, bool FRONT>
__device__ inline void bp_column(const ColumnAnchor& c, float pw2, global_float4* __restrict__ img,
                                 int NU, float (&acc)[K])
{
    constexpr int NB = VD_BP_NB;
    static_assert(K % NB == 0, "column length must be a multiple of the batch");
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += NB) {
        f32x4 q[NB];
        float wa[NB], wb[NB], iw[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const float dk = (float)(k0 + u) - c.ka;  // kk - ka, exact: small integers
            const float W = fmaf(dk, pw2, c.w0);
            const bool front = FRONT || W > 0.0f;  // voxels at or behind the source get no ray
            iw[u] = front ? __builtin_amdgcn_rcpf(W) : 0.0f;
            float A = fmaf(dk * c.nu, iw[u], c.a0f);
            const float B0 = fmaf(dk * c.nv, iw[u], c.b0f);
            if (!FRONT) A = front ? A : -1.0e9f;
            A = __builtin_amdgcn_fmed3f(A, c.alo, c.ahi);
            const float B = __builtin_amdgcn_fmed3f(B0, c.blo, c.bhi);
            const int ia = floor_to_int(A), ib = floor_to_int(B);
            wa[u] = __builtin_amdgcn_fractf(A);
            wb[u] = __builtin_amdgcn_fractf(B);
            q[u] = img[ib * NU + ia];
        }
        // keep the batch whole: without this barrier the scheduler moves the
        // first uses of the taps up between the loads, and the wavefront then
        // waits for each load in turn (measured ~1.6x slower)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const float val = cell_value(q[u].x, q[u].y, q[u].z, q[u].w, wa[u], wb[u], wa[u] * wb[u]);
            if (MODE == DP_W_FDK)
                acc[k0 + u] = fmaf(iw[u] * iw[u], val, acc[k0 + u]);
            else
                acc[k0 + u] += val;
        }
    }
}

// A column with no usable FP64 anchor (it lies within 1 mm of the source
// plane, which only happens with the source inside the volume): every voxel
// is projected on its own in FP64, with the same window clamp and weights.
struct ExactVoxel {
    bool front;        // in front of the source
    float A, B;        // padded-image coordinates, window-clamped
    float iw;          // 1 / depth
    float ap, bp;      // pixel offsets from the detector centre
};

// U, V, W: the projective rows at the voxel (FP64, stepped along the column).
__device__ inline ExactVoxel exact_voxel(const GeoScalars& s, double U, double V, double W)
{
    ExactVoxel x;
    x.front = W > 0.0;
    const double iw = x.front ? 1.0 / W : 0.0;
    const double ap = U * iw, bp = V * iw;
    const double a = x.front ? ap + s.cu + kPadD : -1.0e9;
    x.A = (float)fmin(fmax(a, kPadD - 1.5), s.nu + kPadD + 0.5);
    x.B = (float)fmin(fmax(bp + s.cv + kPadD, kPadD - 1.5), s.nv + kPadD + 0.5);
    x.iw = (float)iw;
    x.ap = (float)ap;
    x.bp = (float)bp;
    return x;
}

// Projective rows of voxel (i, j, k) for one view.
__device__ inline void exact_rows(const ViewGeo& g, int i, int j, int k, double& U, double& V, double& W)
{
    const double fi = i, fj = j, fk = k;
    U = fma(g.PUd[0], fi, fma(g.PUd[1], fj, fma(g.PUd[2], fk, g.PUd[3])));
    V = fma(g.PVd[0], fi, fma(g.PVd[1], fj, fma(g.PVd[2], fk, g.PVd[3])));
    W = fma(g.PWd[0], fi, fma(g.PWd[1], fj, fma(g.PWd[2], fk, g.PWd[3])));
}

template <int MODE, int K>
__device__ inline void bp_column_exact(const ViewGeo& g, const GeoScalars& s, int i, int j, int kb,
                                       global_float4* __restrict__ view, int NU, float (&acc)[K])
{
    // a rolled loop keeps the FP64 code (and its registers) out of the fast
    // paths; each voxel's term reaches its register by compile-time selects
    double U, V, W;
    exact_rows(g, i, j, kb, U, V, W);
#pragma unroll 1
    for (int kk = 0; kk < K; ++kk, U += g.PUd[2], V += g.PVd[2], W += g.PWd[2]) {
        const ExactVoxel x = exact_voxel(s, U, V, W);
        const int ia = floor_to_int(x.A), ib = floor_to_int(x.B);
        const float wa = __builtin_amdgcn_fractf(x.A), wb = __builtin_amdgcn_fractf(x.B);
        const f32x4 q = view[ib * NU + ia];
        const float val = cell_value(q.x, q.y, q.z, q.w, wa, wb, wa * wb);
        const float term = MODE == DP_W_FDK ? x.iw * x.iw * val : val;
#pragma unroll
        for (int t = 0; t < K; ++t) acc[t] += t == kk ? term : 0.0f;
    }
}

// One launch covers the views [v0, v0 + Vc) of the detector images in
// `projq` (this chunk's cell-coefficient images).  The column sums run in view order
// and are carried between launches in `vol` unscaled (FIRST: start from
// zero; LAST: apply the FDK constant), so a chunked back-projection is
// bit-identical to a single launch over all views.
template <int MODE, int K>
__global__ __launch_bounds__(kVdBx * kVdBy) __attribute__((amdgpu_waves_per_eu(VD_BP_WPE))) void vd_bp_kernel(GeoScalars s, int v0, int Vc,
                                                              const ViewGeo* __restrict__ views,
                                                              const float4* __restrict__ projq,
                                                              float* __restrict__ vol, int first,
                                                              int last)
{
    const int i = blockIdx.x * kVdBx + threadIdx.x;
    const int j = blockIdx.y * kVdBy + threadIdx.y;
    const int kb = blockIdx.z * K;
    const int NU = s.nu + 2 * kPadD, NV = s.nv + 2 * kPadD;
    const float D2 = (float)(s.sad * s.sad);
    const bool active = i < s.nx && j < s.ny;
    float acc[K];
#pragma unroll
    for (int kk = 0; kk < K; ++kk)
        acc[kk] = (!first && active && kb + kk < s.nz) ? vol[((size_t)(kb + kk) * s.ny + j) * s.nx + i]
                                                        : 0.0f;
    for (int vv = 0; vv < Vc; ++vv) {
        const ViewGeo& g = views[v0 + vv];
        const ColumnAnchor c = column_anchor(g, s, i, j, kb, K);
        const float pw2 = g.PW[2];
        if (c.exact) {
            bp_column_exact<MODE, K>(g, s, i, j, kb, (global_float4*)(projq + (long long)vv * NU * NV),
                                     NU, acc);
            continue;
        }
        const float4* base = projq + ((long long)vv * NU * NV + c.off);  // anchor pixel of this view
        // one 64-bit base per view and column (kept whole, in global memory's
        // address space), so each update adds only its 32-bit pixel offset
        // (measured faster here than a scalar view base with 32-bit offsets,
        // which the gradient kernel uses)
        asm volatile("" : "+v"(base));
        global_float4* img = (global_float4*)base;
        if (fmaf(-c.ka, pw2, c.w0) > 0.0f && fmaf((float)(K - 1) - c.ka, pw2, c.w0) > 0.0f)
            bp_column<MODE, K, true>(c, pw2, img, NU, acc);
        else
            bp_column<MODE, K, false>(c, pw2, img, NU, acc);
    }
    if (active) {
        const float scale = (MODE == DP_W_FDK && last) ? D2 : 1.0f;
#pragma unroll
        for (int kk = 0; kk < K; ++kk)
            if (kb + kk < s.nz)
                vol[((size_t)(kb + kk) * s.ny + j) * s.nx + i] = scale == 1.0f ? acc[kk] : scale * acc[kk];
    }
}

// One view's gradient sums over a column of K voxels (FRONT as in bp_column).
// Per voxel, with ec = e W / w' and (a', b') = (apc + da, bpc + db):
//   c1 = ec l_a,  c2 = ec l_b,  c3 = -(apc c1 + bpc c2 + s),
//   s = c1 da + c2 db + kappa ec l,
// so the column keeps A1 = sum c1, A2 = sum c2, S = sum s and their moments
// Z1', Z2', ZS' about the column's first voxel (weights kk = 0 .. K-1); the
// caller forms A3, the third moment and the shift to the volume centre once
// per column.
// Tap sources of the gradient: the chunk's DetTap3 images in global memory
// (a wave-uniform view base plus 32-bit byte offsets), or one view's
// rectangle of them staged in LDS (offsets clamped to the rectangle).
struct GlobalTaps {
    global_bytes* view;
    int row;  // bytes per padded image row
    __device__ inline void load(unsigned o, float4& l, float4& a, float4& b) const
    {
        const f32x4 tl = ld16(view, o), ta = ld16(view + 16, o), tb = ld16(view + 32, o);
        l = make_float4(tl.x, tl.y, tl.z, tl.w);
        a = make_float4(ta.x, ta.y, ta.z, ta.w);
        b = make_float4(tb.x, tb.y, tb.z, tb.w);
    }
};

struct LdsTaps {
    const DetTap3* stage;  // the staged rectangle, row-major
    int row;               // bytes per staged row
    unsigned hi;           // byte offset of its last pixel
    __device__ inline void load(unsigned o, float4& l, float4& a, float4& b) const
    {
        const DetTap3& t = *(const DetTap3*)((const char*)stage + min(o, hi));
        l = t.l;
        a = t.a;
        b = t.b;
    }
};

template <int MODE, int K, bool FRONT, class Taps>
__device__ inline void grad_column(const ColumnAnchor& c, float pw2, const Taps& taps,
                                   unsigned col, const float (&e)[K], float& A1, float& A2,
                                   float& S, float& Z1, float& Z2, float& ZS)
{
    constexpr int NB = VD_GRAD_NB;  // voxels whose three taps are in flight together
    static_assert(K % NB == 0, "column length must be a multiple of the batch");
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += NB) {
        float4 ql[NB], qa[NB], qb[NB];
        float wa[NB], wb[NB], iw[NB], da[NB], db[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const float dk = (float)(k0 + u) - c.ka;  // kk - ka, exact: small integers
            const float W = fmaf(dk, pw2, c.w0);
            const bool front = FRONT || W > 0.0f;  // voxels at or behind the source get no ray
            iw[u] = front ? __builtin_amdgcn_rcpf(W) : 0.0f;
            const float t = dk * iw[u];
            da[u] = t * c.nu;
            db[u] = t * c.nv;
            float A = c.a0f + da[u];
            if (!FRONT) A = front ? A : -1.0e9f;
            A = __builtin_amdgcn_fmed3f(A, c.alo, c.ahi);
            const float B = __builtin_amdgcn_fmed3f(c.b0f + db[u], c.blo, c.bhi);
            const int ia = floor_to_int(A), ib = floor_to_int(B);
            wa[u] = __builtin_amdgcn_fractf(A);
            wb[u] = __builtin_amdgcn_fractf(B);
            taps.load(tap_offset<48>(col, ia, ib, taps.row), ql[u], qa[u], qb[u]);  // DetTap3: 48 B
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const float wab = wa[u] * wb[u];
            const float l = cell_value(ql[u].x, ql[u].y, ql[u].z, ql[u].w, wa[u], wb[u], wab);
            const float la = cell_value(qa[u].x, qa[u].y, qa[u].z, qa[u].w, wa[u], wb[u], wab);
            const float lb = cell_value(qb[u].x, qb[u].y, qb[u].z, qb[u].w, wa[u], wb[u], wab);
            // e * W / w' (FDK: e D^2 / w'^3, with D^2 folded into e)
            const float ec = MODE == DP_W_FDK ? e[k0 + u] * (iw[u] * iw[u]) * iw[u] : e[k0 + u] * iw[u];
            const float c1 = ec * la, c2 = ec * lb;
            const float sk = MODE == DP_W_FDK ? fmaf(c1, da[u], fmaf(c2, db[u], (ec + ec) * l))
                                              : fmaf(c1, da[u], c2 * db[u]);
            const float kz = (float)(k0 + u);
            A1 += c1; A2 += c2; S += sk;
            Z1 = fmaf(c1, kz, Z1); Z2 = fmaf(c2, kz, Z2); ZS = fmaf(sk, kz, ZS);
        }
    }
}

// Sum 12 channels over the wavefront and add them to out[12] (this
// wavefront's LDS slice for one view).  Channel-halving butterfly: at the
// xor-32 and xor-16 steps each lane keeps half of the channels and receives
// the partner's sums of them, so the 12 channels take 6 + 3 + 4 x 3 = 21
// cross-lane exchanges instead of 72.  Lane 16 q (q = 0..3) ends with
// channels 3 q .. 3 q + 2 of the whole wavefront.
__device__ inline void wave_partials(const float (&r)[kVdChannels], int lane, float* out)
{
    const bool h32 = (lane & 32) != 0, h16 = (lane & 16) != 0;
    float s6[6], s3[3];
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const float keep = h32 ? r[6 + t] : r[t], give = h32 ? r[t] : r[6 + t];
        s6[t] = keep + __shfl_xor(give, 32);
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const float keep = h16 ? s6[3 + t] : s6[t], give = h16 ? s6[t] : s6[3 + t];
        s3[t] = keep + __shfl_xor(give, 16);
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1)
#pragma unroll
        for (int t = 0; t < 3; ++t) s3[t] += __shfl_xor(s3[t], off);
    if ((lane & 15) == 0) {
        float* o = out + (lane >> 4) * 3;
#pragma unroll
        for (int t = 0; t < 3; ++t) o[t] += s3[t];
    }
}

// Per-block partial sums of one view chunk: each wavefront accumulates its
// per-view channel sums over the block's column groups in its own LDS slice;
// the block then adds the four slices in a fixed order and writes (ADD:
// adds) one partial set per view, partials[v][blk][kVdChannels].
constexpr int kVgWaves = kVgBx * kVgBy / 64;
struct VdGradShared {
    float acc[kVgWaves][kVdMaxChunk][kVdChannels];
};

__device__ inline void vd_shared_zero(VdGradShared& sh)
{
    float* a = &sh.acc[0][0][0];
    for (int t = threadIdx.x; t < kVgWaves * kVdMaxChunk * kVdChannels; t += kVgBx * kVgBy) a[t] = 0.0f;
    __syncthreads();
}

template <bool ADD>
__device__ inline void vd_shared_store(const VdGradShared& sh, int v0, int Vc, int blk, int nblk,
                                       const int* __restrict__ only, float* __restrict__ partials)
{
    static_assert(kVgWaves == 4, "fixed-order sum of four wavefront slices");
    __syncthreads();
    for (int t = threadIdx.x; t < Vc * kVdChannels; t += kVgBx * kVgBy) {
        const int vv = t / kVdChannels, c = t - vv * kVdChannels;
        if (only && only[v0 + vv] == 0) continue;
        const float sum = ((sh.acc[0][vv][c] + sh.acc[1][vv][c]) + sh.acc[2][vv][c]) + sh.acc[3][vv][c];
        float* o = partials + ((size_t)(v0 + vv) * nblk + blk) * kVdChannels + c;
        *o = ADD ? *o + sum : sum;
    }
}

// Thread t of a gradient block owns voxel column (x0 + t % kVgBx, y0 + t / kVgBx).
__device__ inline int vg_col_i() { return blockIdx.x * kVgBx + (int)(threadIdx.x % kVgBx); }
__device__ inline int vg_col_j() { return blockIdx.y * kVgBy + (int)(threadIdx.x / kVgBx); }

// Staged detector rectangle of one view: padded pixels [a0, a0 + w) x
// [b0, b0 + h); w = 0 when the block's taps are gathered from global memory.
struct StageRect {
    int a0, b0, w, h;
};

// The rectangle that holds every tap of the block's voxel region (kVgBx x
// kVgBy columns of K voxels from kb, grid faces ignored) for one view, from
// the FP64 projections of the region's 8 corner voxels (the projective map
// is monotone along every segment in front of the source, so the region's
// image lies in the hull of theirs), window-clamped like the voxels, plus a
// safety margin.  Wavefront 0 computes it; w = 0 unless every corner lies at
// least 1 mm in front of the source and the rectangle fits kVgStage pixels.
__device__ inline void stage_rect(const ViewGeo& g, const GeoScalars& s, int kb, int K,
                                  StageRect& out)
{
    const int q = threadIdx.x;  // lanes 0 .. 7 of wavefront 0: the corners
    double amin = 1.0e300, amax = -1.0e300, bmin = 1.0e300, bmax = -1.0e300;
    int ok = 1;
    if (q < 8) {
        const double ci = blockIdx.x * kVgBx + (q & 1) * (kVgBx - 1);
        const double cj = blockIdx.y * kVgBy + ((q >> 1) & 1) * (kVgBy - 1);
        const double ck = kb + (q >> 2) * (K - 1);
        const double U = fma(g.PUd[0], ci, fma(g.PUd[1], cj, fma(g.PUd[2], ck, g.PUd[3])));
        const double V = fma(g.PVd[0], ci, fma(g.PVd[1], cj, fma(g.PVd[2], ck, g.PVd[3])));
        const double W = fma(g.PWd[0], ci, fma(g.PWd[1], cj, fma(g.PWd[2], ck, g.PWd[3])));
        ok = W >= 1.0;
        const double iw = ok ? 1.0 / W : 0.0;
        const double a = fmin(fmax(U * iw + s.cu + kPadD, kPadD - 1.5), s.nu + kPadD + 0.5);
        const double b = fmin(fmax(V * iw + s.cv + kPadD, kPadD - 1.5), s.nv + kPadD + 0.5);
        amin = amax = a;
        bmin = bmax = b;
    }
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
        amin = fmin(amin, __shfl_xor(amin, off));
        amax = fmax(amax, __shfl_xor(amax, off));
        bmin = fmin(bmin, __shfl_xor(bmin, off));
        bmax = fmax(bmax, __shfl_xor(bmax, off));
        ok &= __shfl_xor(ok, off);
    }
    if (q == 0) {
        const int NU = s.nu + 2 * kPadD, NV = s.nv + 2 * kPadD;
        const int a0 = max(0, (int)floor(amin - 1.0e-3)), a1 = min(NU - 1, (int)floor(amax + 1.0e-3) + 1);
        const int b0 = max(0, (int)floor(bmin - 1.0e-3)), b1 = min(NV - 1, (int)floor(bmax + 1.0e-3) + 1);
        const int w = a1 - a0 + 1, h = b1 - b0 + 1;
        const bool fits = ok && w > 0 && h > 0 && w * h <= kVgStage;
        out.a0 = a0;
        out.b0 = b0;
        out.w = fits ? w : 0;
        out.h = fits ? h : 0;
    }
}

// Copy the rectangle's DetTap3 pixels into LDS (row-major, w per row): every
// thread issues its (at most 8) 16-byte loads before its first store.
__device__ inline void stage_copy(const StageRect& r, global_bytes* view, int NU, DetTap3* stage)
{
    constexpr int kPer = (3 * kVgStage + kVgBx * kVgBy - 1) / (kVgBx * kVgBy);
    const int n16 = 3 * r.w * r.h;
    const float invw = 1.0f / (float)r.w;
    f32x4 buf[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int q = (int)threadIdx.x + u * kVgBx * kVgBy;
        if (q < n16) {
            const int p = q / 3, part = q - 3 * p;
            const int row = (int)(((float)p + 0.5f) * invw), cl = p - row * r.w;
            buf[u] = ld16(view, (unsigned)(((r.b0 + row) * NU + r.a0 + cl) * 48 + part * 16));
        }
    }
    f32x4* dst = (f32x4*)stage;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int q = (int)threadIdx.x + u * kVgBx * kVgBy;
        if (q < n16) dst[q] = buf[u];
    }
}

// Block (bx, by, bz) covers kVgBx x kVgBy voxel columns and the zpb
// consecutive column groups of K voxels starting at group bz * zpb.  Per
// view, the detector rectangle under the block's region is staged in LDS
// when it fits (every tap then an LDS read); otherwise the taps come from
// global memory.
template <int MODE, int K>
__global__ __launch_bounds__(kVgBx * kVgBy) __attribute__((amdgpu_waves_per_eu(VD_GRAD_WPE))) void vd_grad_kernel(
    GeoScalars s, int v0, int Vc, int zpb, const ViewGeo* __restrict__ views,
    const DetTap3* __restrict__ det, const float* __restrict__ grad_vol,
    float* __restrict__ partials, int* __restrict__ exact_views)
{
    __shared__ VdGradShared sh;
    __shared__ DetTap3 stage[kVgStage];
    __shared__ StageRect rect;
    const int i = vg_col_i(), j = vg_col_j();
    const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    const int NU = s.nu + 2 * kPadD, NV = s.nv + 2 * kPadD;
    const float D2 = (float)(s.sad * s.sad);
    const float pi = (float)i - 0.5f * (s.nx - 1), pj = (float)j - 0.5f * (s.ny - 1);
    const bool active = i < s.nx && j < s.ny;
    const int lane = threadIdx.x & 63;
    float* mine = &sh.acc[threadIdx.x >> 6][0][0];
    vd_shared_zero(sh);
    for (int zg = 0; zg < zpb; ++zg) {
        const int kb = ((int)blockIdx.z * zpb + zg) * K;
        if (kb >= s.nz) break;  // uniform over the block
        const float pk0 = (float)kb - 0.5f * (s.nz - 1);
        // dL/dmu of this thread's voxel column, kept in registers for all views.
        float e[K];
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
            const bool in = active && kb + kk < s.nz;
            e[kk] = in ? grad_vol[((size_t)(kb + kk) * s.ny + j) * s.nx + i] : 0.0f;
            if (MODE == DP_W_FDK) e[kk] *= D2;
        }
        for (int vv = 0; vv < Vc; ++vv) {
            const ViewGeo& g = views[v0 + vv];
            global_bytes* view = (global_bytes*)(det + (long long)vv * NU * NV);
            if (threadIdx.x < 64) stage_rect(g, s, kb, K, rect);
            __syncthreads();  // rect visible; every reader of the previous view's stage is done
            const StageRect r = rect;
            if (r.w > 0) stage_copy(r, view, NU, stage);
            __syncthreads();  // stage visible (rect is read by everyone before this point)
            const ColumnAnchor c = column_anchor(g, s, i, j, kb, K);
            const float pw2 = g.PW[2];
            float A1 = 0.f, A2 = 0.f, S = 0.f, Z1 = 0.f, Z2 = 0.f, ZS = 0.f;
            if (c.exact) {
                // no usable anchor: vd_grad_exact_kernel adds this column's sums
                exact_views[v0 + vv] = 1;
            } else if (r.w > 0) {
                // every voxel of the region lies in front of the source
                const LdsTaps t{stage, 48 * r.w, (unsigned)(48 * (r.w * r.h - 1))};
                const unsigned col = (unsigned)(((c.bi - r.b0) * r.w + (c.ai - r.a0)) * 48);
                grad_column<MODE, K, true>(c, pw2, t, col, e, A1, A2, S, Z1, Z2, ZS);
            } else {
                const GlobalTaps t{view, 48 * NU};
                const unsigned col = (unsigned)c.off * 48u;  // anchor pixel of this view
                if (fmaf(-c.ka, pw2, c.w0) > 0.0f && fmaf((float)(K - 1) - c.ka, pw2, c.w0) > 0.0f)
                    grad_column<MODE, K, true>(c, pw2, t, col, e, A1, A2, S, Z1, Z2, ZS);
                else
                    grad_column<MODE, K, false>(c, pw2, t, col, e, A1, A2, S, Z1, Z2, ZS);
            }
            // third channel, and moments about the volume centre (k - centre = pk0 + kk)
            const float A3 = -fmaf(c.apc, A1, fmaf(c.bpc, A2, S));
            const float Z3 = fmaf(pk0, A3, -fmaf(c.apc, Z1, fmaf(c.bpc, Z2, ZS)));
            Z1 = fmaf(pk0, A1, Z1);
            Z2 = fmaf(pk0, A2, Z2);
            const float rr[kVdChannels] = {A1, A2, A3, pi * A1, pi * A2, pi * A3,
                                           pj * A1, pj * A2, pj * A3, Z1, Z2, Z3};
            wave_partials(rr, lane, mine + vv * kVdChannels);
        }
    }
    vd_shared_store<false>(sh, v0, Vc, blk, nblk, nullptr, partials);
}

// Columns with no usable FP64 anchor (every voxel within 1 mm of the source
// plane, or an anchor projecting more than anchor_limit() pixels from the
// detector centre; only with the source inside or next to the volume), which
// vd_grad_kernel leaves out and flags per view: their voxels are projected
// one by one in FP64 and their block sums added to the same per-block
// partials (same blocks, same column groups, same fixed order).  Views
// without a flag are skipped; in the others a conservative FP32 test of the
// column ends skips every column that cannot be such a column: if the depth
// keeps its sign and exceeds 2 mm at both ends, it exceeds 1 mm along the
// whole column, so the middle voxel is the anchor, and its projection lies
// between those of the ends (the projective map has no pole in between), so
// it is within the limit when both ends are within 0.9 of it.
template <int MODE, int K>
__global__ __launch_bounds__(kVgBx * kVgBy) void vd_grad_exact_kernel(
    GeoScalars s, int v0, int Vc, int zpb, const ViewGeo* __restrict__ views,
    const DetTap3* __restrict__ det, const float* __restrict__ grad_vol,
    float* __restrict__ partials, const int* __restrict__ exact_views)
{
    // uniform over the launch: nothing to do unless a view of the chunk is flagged
    bool any = false;
    for (int vv = 0; vv < Vc; ++vv) any = any || exact_views[v0 + vv] != 0;
    if (!any) return;
    __shared__ VdGradShared sh;
    const int i = vg_col_i(), j = vg_col_j();
    const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    const int NU = s.nu + 2 * kPadD, NV = s.nv + 2 * kPadD;
    const float escale = MODE == DP_W_FDK ? (float)(s.sad * s.sad) : 1.0f;
    const float kappa = MODE == DP_W_FDK ? 2.0f : 0.0f;
    const float pi = (float)i - 0.5f * (s.nx - 1), pj = (float)j - 0.5f * (s.ny - 1);
    const int lane = threadIdx.x & 63;
    const float lim = 0.9f * (float)anchor_limit(s);
    float* mine = &sh.acc[threadIdx.x >> 6][0][0];
    vd_shared_zero(sh);
    for (int zg = 0; zg < zpb; ++zg) {
        const int kb = ((int)blockIdx.z * zpb + zg) * K;
        if (kb >= s.nz) break;  // uniform over the block
        const float pk0 = (float)kb - 0.5f * (s.nz - 1);
        const float fi = (float)i, fj = (float)j, flo = (float)kb, fhi = (float)(kb + K - 1);
        for (int vv = 0; vv < Vc; ++vv) {
            if (exact_views[v0 + vv] == 0) continue;  // no column of this view was left out
            const ViewGeo& g = views[v0 + vv];
            const float wij = fmaf(g.PW[0], fi, fmaf(g.PW[1], fj, g.PW[3]));
            const float uij = fmaf(g.PU[0], fi, fmaf(g.PU[1], fj, g.PU[3]));
            const float vij = fmaf(g.PV[0], fi, fmaf(g.PV[1], fj, g.PV[3]));
            const float wlo = fmaf(g.PW[2], flo, wij), whi = fmaf(g.PW[2], fhi, wij);
            const float ulo = fmaf(g.PU[2], flo, uij), uhi = fmaf(g.PU[2], fhi, uij);
            const float vlo = fmaf(g.PV[2], flo, vij), vhi = fmaf(g.PV[2], fhi, vij);
            const bool safe = (wlo > 2.0f && whi > 2.0f) || (wlo < -2.0f && whi < -2.0f);
            const float lim_lo = lim * fabsf(wlo), lim_hi = lim * fabsf(whi);
            const bool cand = !(safe && fabsf(ulo) < lim_lo && fabsf(uhi) < lim_hi &&
                                fabsf(vlo) < lim_lo && fabsf(vhi) < lim_hi);
            if (__ballot(cand) == 0) continue;  // wave-uniform: no column of this wavefront
            float A1 = 0.f, A2 = 0.f, A3 = 0.f, Z1 = 0.f, Z2 = 0.f, Z3 = 0.f;
            if (cand && column_anchor(g, s, i, j, kb, K).exact) {
                const DetTap3* view = det + (long long)vv * NU * NV;
                double U, V, W;
                exact_rows(g, i, j, kb, U, V, W);
                for (int kk = 0; kk < K; ++kk, U += g.PUd[2], V += g.PVd[2], W += g.PWd[2]) {
                    const bool in = i < s.nx && j < s.ny && kb + kk < s.nz;
                    const float ek = in ? escale * grad_vol[((size_t)(kb + kk) * s.ny + j) * s.nx + i] : 0.0f;
                    const ExactVoxel x = exact_voxel(s, U, V, W);
                    const int ia = floor_to_int(x.A), ib = floor_to_int(x.B);
                    const float wa = __builtin_amdgcn_fractf(x.A), wb = __builtin_amdgcn_fractf(x.B);
                    const DetTap3* p = view + (ib * NU + ia);
                    const float4 ql = p->l, qa = p->a, qb = p->b;
                    const float wab = wa * wb;
                    const float l = cell_value(ql.x, ql.y, ql.z, ql.w, wa, wb, wab);
                    const float la = cell_value(qa.x, qa.y, qa.z, qa.w, wa, wb, wab);
                    const float lb = cell_value(qb.x, qb.y, qb.z, qb.w, wa, wb, wab);
                    const float ec = MODE == DP_W_FDK ? ek * (x.iw * x.iw) * x.iw : ek * x.iw;
                    const float c1 = ec * la, c2 = ec * lb;
                    const float c3 = -ec * fmaf(la, x.ap, fmaf(lb, x.bp, kappa * l));
                    const float pk = pk0 + (float)kk;
                    A1 += c1; A2 += c2; A3 += c3;
                    Z1 = fmaf(c1, pk, Z1); Z2 = fmaf(c2, pk, Z2); Z3 = fmaf(c3, pk, Z3);
                }
            }
            const float r[kVdChannels] = {A1, A2, A3, pi * A1, pi * A2, pi * A3,
                                          pj * A1, pj * A2, pj * A3, Z1, Z2, Z3};
            wave_partials(r, lane, mine + vv * kVdChannels);
        }
    }
    vd_shared_store<true>(sh, v0, Vc, blk, nblk, exact_views, partials);
}

template <int MODE>
static void vd_bp_dispatch(const GeoScalars& s, int v0, int Vc, const ViewGeo* views,
                           const float4* projq, float* vol, bool first, bool last, hipStream_t st)
{
    dim3 block(kVdBx, kVdBy);
    dim3 grid((s.nx + kVdBx - 1) / kVdBx, (s.ny + kVdBy - 1) / kVdBy, (s.nz + kVdBpCol - 1) / kVdBpCol);
    vd_bp_kernel<MODE, kVdBpCol><<<grid, block, 0, st>>>(s, v0, Vc, views, projq, vol, first, last);
}

void launch_vd_bp(const GeoScalars& s, int v0, int Vc, const ViewGeo* views, const float4* projq,
                  float* vol, int weight_mode, bool first, bool last, hipStream_t st)
{
    prof_begin(DP_K_VD_BP, st);
    if (weight_mode == DP_W_FDK)
        vd_bp_dispatch<DP_W_FDK>(s, v0, Vc, views, projq, vol, first, last, st);
    else
        vd_bp_dispatch<DP_W_NONE>(s, v0, Vc, views, projq, vol, first, last, st);
    prof_end(DP_K_VD_BP, st);
}

__global__ __launch_bounds__(256) void fill_zero_i32_kernel(int* __restrict__ p, int n)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < n) p[t] = 0;
}

void launch_vd_flags_clear(int V, int* flags, hipStream_t st)
{
    fill_zero_i32_kernel<<<(V + 255) / 256, 256, 0, st>>>(flags, V);
}

VdGradGrid vd_grad_grid(const GeoScalars& s)
{
    VdGradGrid g;
    const int gx = (s.nx + kVgBx - 1) / kVgBx, gy = (s.ny + kVgBy - 1) / kVgBy;
    const int groups = (s.nz + kVdGradCol - 1) / kVdGradCol;
    // enough blocks to fill the chip several times over; beyond that, blocks
    // take several column groups each (fewer partial sets to write and sum)
    g.zpb = std::max(1, std::min(8, gx * gy * groups / kVdGradMinBlocks));
    g.gz = (groups + g.zpb - 1) / g.zpb;
    g.blocks = gx * gy * g.gz;
    return g;
}

template <int MODE>
static void vd_grad_dispatch(const GeoScalars& s, int v0, int Vc, const ViewGeo* views,
                             const DetTap3* det, const float* grad_vol, float* partials, int* flags,
                             hipStream_t st)
{
    const VdGradGrid vg = vd_grad_grid(s);
    dim3 block(kVgBx * kVgBy);
    dim3 grid((s.nx + kVgBx - 1) / kVgBx, (s.ny + kVgBy - 1) / kVgBy, vg.gz);
    vd_grad_kernel<MODE, kVdGradCol><<<grid, block, 0, st>>>(s, v0, Vc, vg.zpb, views, det,
                                                             grad_vol, partials, flags);
    vd_grad_exact_kernel<MODE, kVdGradCol><<<grid, block, 0, st>>>(s, v0, Vc, vg.zpb, views, det,
                                                                   grad_vol, partials, flags);
}

void launch_vd_grad(const GeoScalars& s, int v0, int Vc, const ViewGeo* views, const DetTap3* det,
                    const float* grad_vol, float* partials, int* flags, int weight_mode,
                    hipStream_t st)
{
    prof_begin(DP_K_VD_GRAD, st);
    if (weight_mode == DP_W_FDK)
        vd_grad_dispatch<DP_W_FDK>(s, v0, Vc, views, det, grad_vol, partials, flags, st);
    else
        vd_grad_dispatch<DP_W_NONE>(s, v0, Vc, views, det, grad_vol, partials, flags, st);
    prof_end(DP_K_VD_GRAD, st);
}

}  // namespace dp
