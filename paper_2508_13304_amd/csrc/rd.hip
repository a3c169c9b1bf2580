// Ray-driven cone-beam forward projector and its rigid-motion gradient.
//
// Forward (Eq. forward, Sec. II-A; discretised as l^i = sum_j a^ij mu^j,
// Sec. II-C): each lane marches one detector ray through the rigidly moved
// volume.  Samples sit at world-anchored arc lengths k*step from the source
// (k >= 0), are mapped to the object frame by r' = R^T (r - t), and are
// trilinearly interpolated from a zero-padded copy of the volume; the sum
// is scaled by step.
//
// Gradient (Eqs. final_forward / for_int / dis_forward, Sec. II-B/C): the
// same samples are recomputed (never stored), and each per-voxel matrix
// G_f^j = [(R p_j) g_j^T | -R g_j] is projected with the same trilinear
// weights a^ij and weighted by dL/dl -- computed once per sample and shared
// by all 12 entries (the weight-sharing of Sec. II-C).  Because R is common
// to every voxel of a view, the 12 entries collapse exactly to 9 per-ray
// sums in voxel-index units:
//   B_c   = sum phi_j G_c(j)                 (G = central difference / 2 in index units)
//   T_a,c = sum phi_j (I_a(j) - c_a) G_c(j)  (a != c)
// from which the finalize kernel forms dL/dt = -R b and dL/dgamma_a =
// -omega_a . (R tau) with b = B / h and tau = sum phi p x g.
//
// Memory: a block owns a 16x16 pixel tile of one view (4 wavefronts of 8x8
// rays).  Its rays are marched in chunks of M consecutive sample numbers
// k.  The samples of one chunk lie in the convex hull of the tile's four
// corner rays between the chunk's two arc lengths, up to the height of the
// spherical cap spanned by the tile (bounded per tile), so the chunk's
// axis-aligned bounding box is loaded once, coalesced, into LDS and every
// trilinear tap is an LDS read.  All chunk boxes of a tile are planned up
// front, one per thread; M shrinks in steps until every box fits the LDS
// budget, and a tile whose boxes do not fit even at M = 1 (or need more
// chunks than threads) reads its taps from global memory.
//
// Numerics: per-ray setup in FP64; each ray is anchored at its crossing of
// the iso-plane (a point of small magnitude) and, per chunk, re-anchored at
// its first sample of the chunk, X(kb) = X0 + (f + (kb - k0) step) D; the
// chunk's samples are then X(kb) + j (step D) for j < M.  No absolute
// position of ~1000 mm is ever formed in FP32.
#include <type_traits>

#include "dp_internal.h"

namespace dp {

// LDS budgets: forward = one float per voxel; gradient (with or without the
// SSD) = (mu, Gx, Gy, Gz) interleaved per voxel, one 16-byte read per
// trilinear corner.
// Compiled variants: tile shape x chunk class (chunk length before
// adaptation, LDS voxels; listed with the launchers); the autotuner picks
// one per shape class, variant 1 (16x16 tiles, middle class) is the default.
// At most one chunk per thread of the block: thread i plans chunk i and
// keeps its box record in registers (published to the block through a
// two-slot LDS buffer when the chunk comes up).
constexpr int kMaxChunks = kRdThreads;
// 16-byte row loads for interior boxes of volumes with aligned rows (a
// build-time switch for measurements; 1 in the library)
#ifndef RD_VEC_ROWS
#define RD_VEC_ROWS 1
#endif

struct RayState {
    float x0, y0, z0;   // padded voxel index of the iso-plane anchor
    float dx, dy, dz;   // direction in voxel-index units per mm
    float f;            // arc-length offset of sample k0 from the anchor (mm)
    int k0;             // sample number of the anchor's nearest sample
    int klo, khi;       // in-support sample numbers (inclusive); empty if klo > khi
};

// FP64 per-ray setup: anchor, direction, sample offset and the slab clip of
// the samples against the support (-1, n) of the trilinear interpolant.
__device__ inline RayState ray_setup(const GeoScalars& s, const ViewGeo& g, int a, int b)
{
    RayState r;
    const double D = s.sad, S = s.sdd;
    const double xa = (a - s.cu) * s.du, yb = (b - s.cv) * s.dv;
    const double q = D / S;
    const double nrm = sqrt(S * S + xa * xa + yb * yb);
    const double inv = 1.0 / nrm;
    double X0[3], Dir[3];
    for (int c = 0; c < 3; ++c) {
        X0[c] = q * (xa * g.EU[c] + yb * g.EV[c]) + g.OT[c];
        Dir[c] = (S * g.EW[c] + xa * g.EU[c] + yb * g.EV[c]) * inv;
    }
    // Arc length of the anchor from the source: D sqrt(1 + rho^2); sample
    // k0 = round(that / step); f = k0 step - D - D rho^2 / (sqrt(1+rho^2) + 1).
    const double rho2 = (xa * xa + yb * yb) / (S * S);
    const double sq = sqrt(1.0 + rho2);
    const double k0 = rint(D * sq / s.step);
    const double f = (k0 * s.step - D) - D * rho2 / (sq + 1.0);
    const int n[3] = {s.nx, s.ny, s.nz};
    double tlo = -1.0e30, thi = 1.0e30;
    bool empty = !(k0 < 1.0e8);  // also false for NaN geometry
    for (int c = 0; c < 3; ++c) {
        const double lo = kPadV - 1.0, hi = (double)n[c] + kPadV;
        if (fabs(Dir[c]) > 1.0e-12) {
            const double t1 = (lo - X0[c]) / Dir[c], t2 = (hi - X0[c]) / Dir[c];
            tlo = fmax(tlo, fmin(t1, t2));
            thi = fmin(thi, fmax(t1, t2));
        } else if (!(X0[c] > lo && X0[c] < hi)) {
            empty = true;
        }
    }
    // the anchor geometry stays valid for rays without samples: corner rays
    // of a tile bound the chunk boxes whether or not they hit the volume
    r.k0 = k0 < 1.0e8 ? (int)k0 : 0;
    r.klo = 1;
    r.khi = 0;
    if (!empty && tlo < thi) {  // false for NaN inputs
        double mlo = ceil((tlo - f) / s.step), mhi = floor((thi - f) / s.step);
        mlo = fmax(mlo, -k0);  // k = k0 + m >= 0: in front of the source
        if (mlo <= mhi && mhi - mlo < 1.0e7) {
            r.klo = (int)(k0 + mlo);
            r.khi = (int)(k0 + mhi);
        }
    }
    r.x0 = (float)X0[0]; r.y0 = (float)X0[1]; r.z0 = (float)X0[2];
    r.dx = (float)Dir[0]; r.dy = (float)Dir[1]; r.dz = (float)Dir[2];
    r.f = (float)f;
    return r;
}

// Lane -> detector pixel: 4 wavefronts per block, each an 8x8 pixel tile,
// in a block tile TW pixels wide (u) and 256 / TW high (v).
template <int TW>
__device__ inline void rd_pixel(const GeoScalars& s, int tile, int& a, int& b, int& a0, int& b0)
{
    constexpr int TH = kRdThreads / TW, WU = TW / 8;
    const int tiles_u = (s.nu + TW - 1) / TW;
    const int tu = tile % tiles_u, tv = tile / tiles_u;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    a0 = tu * TW;
    b0 = tv * TH;
    a = a0 + (wave % WU) * 8 + (lane & 7);
    b = b0 + (wave / WU) * 8 + (lane >> 3);
}

__device__ inline float lerpf(float a, float b, float w) { return fmaf(w, b - a, a); }

// 16-byte LDS vector with its address space explicit (LDS instructions, not
// flat ones, whatever the pointer it is formed from)
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const v4f lds_v4f;

struct Corner {
    float x0, y0, z0, dx, dy, dz, f, k0;
};

struct Box {
    int ox, oy, oz, bx, by, bz;
    int px, py;  // LDS row and slice pitch in voxels (bx, by rounded up to odd)
};

// Odd LDS pitches: rays of one wavefront that sample neighbouring rows
// (or slices) of a box then read different LDS banks; an even pitch maps
// every other row onto the same banks.
__device__ inline int lds_pitch(int n) { return n | 1; }

// Block-wide state shared by both kernels.
struct TileShared {
    Corner corner[4];
    int klo[4], khi[4], vmax[4];
    unsigned cur[2][3];  // box records of the current and the next chunk
};

// A chunk box packed in three words: (ox | oy << 16, oz | bx << 16,
// by | bz << 16); every field fits 16 bits (padded extents <= 65535).
struct BoxRec {
    unsigned w[3];
};

// Union of the active rays' sample ranges, the tile's four corner rays and
// the margin that covers the spherical cap between them (voxel units).
// `active` rays define the sample range; every in-detector corner lane
// publishes its ray geometry (whether or not it carries samples).
template <int TW>
__device__ inline void tile_setup(const GeoScalars& s, const RayState& r, bool inside, bool active,
                                  int a, int b, int a0, int b0, TileShared& sh, int& Kmin,
                                  int& Kmax, float& margin)
{
    int lo = active && r.klo <= r.khi ? r.klo : INT_MAX;
    int hi = active && r.klo <= r.khi ? r.khi : INT_MIN;
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off));
        hi = max(hi, __shfl_xor(hi, off));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sh.klo[wave] = lo;
        sh.khi[wave] = hi;
    }
    // corner rays: first / last valid pixel of the tile in each direction
    const int a1 = min(a0 + TW - 1, s.nu - 1), b1 = min(b0 + kRdThreads / TW - 1, s.nv - 1);
    // a degenerate tile (one column or row) has coincident corners: every
    // owner writes the same values
    if (inside && (a == a0 || a == a1) && (b == b0 || b == b1)) {
        const Corner c = {r.x0, r.y0, r.z0, r.dx, r.dy, r.dz, r.f, (float)r.k0};
        if (a == a0 && b == b0) sh.corner[0] = c;
        if (a == a1 && b == b0) sh.corner[1] = c;
        if (a == a0 && b == b1) sh.corner[2] = c;
        if (a == a1 && b == b1) sh.corner[3] = c;
    }
    __syncthreads();
    Kmin = min(min(sh.klo[0], sh.klo[1]), min(sh.klo[2], sh.klo[3]));
    Kmax = max(max(sh.khi[0], sh.khi[1]), max(sh.khi[2], sh.khi[3]));
    // Cap height: for unit directions u0, u3 of the diagonal corner rays, the
    // tile's rays deviate from the corner hull by at most
    // lambda (1 - cos(theta/2)) <= 0.31 lambda |u0 - u3|^2 (mm).
    const float S = (float)s.sdd;
    const float xa0 = (float)((a0 - s.cu) * s.du), xa1 = (float)((a1 - s.cu) * s.du);
    const float yb0 = (float)((b0 - s.cv) * s.dv), yb1 = (float)((b1 - s.cv) * s.dv);
    const float n0 = rsqrtf(S * S + xa0 * xa0 + yb0 * yb0), n1 = rsqrtf(S * S + xa1 * xa1 + yb1 * yb1);
    const float e0 = S * (n0 - n1), e1 = xa0 * n0 - xa1 * n1, e2 = yb0 * n0 - yb1 * n1;
    const float hmin = (float)fmin(s.vx, fmin(s.vy, s.vz));
    const float lmax = (float)(fmax((double)Kmax, 0.0) * s.step + s.step);
    margin = 0.31f * lmax * (e0 * e0 + e1 * e1 + e2 * e2) / hmin + 0.02f;
}

// Bounding box (padded voxel indices, clamped to the padded volume) of all
// trilinear taps of the samples k in [K, Ke] of every ray of the tile.
__device__ inline Box chunk_box(const TileShared& sh, int K, int Ke, float step, float margin,
                                int NX, int NY, int NZ)
{
    float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const Corner& q = sh.corner[c];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const float t = fmaf((float)(e ? Ke : K) - q.k0, step, q.f);
            const float p[3] = {fmaf(t, q.dx, q.x0), fmaf(t, q.dy, q.y0), fmaf(t, q.dz, q.z0)};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                lo[d] = fminf(lo[d], p[d]);
                hi[d] = fmaxf(hi[d], p[d]);
            }
        }
    }
    const float cap[3] = {(float)(NX - 1), (float)(NY - 1), (float)(NZ - 1)};
    int o[3], e[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        o[d] = (int)fminf(fmaxf(floorf(lo[d] - margin), 0.0f), cap[d]);
        e[d] = (int)fminf(fmaxf(floorf(hi[d] + margin) + 1.0f, 0.0f), cap[d]);
    }
    Box bx;
    bx.ox = o[0]; bx.oy = o[1]; bx.oz = o[2];
    bx.bx = e[0] - o[0] + 1; bx.by = e[1] - o[1] + 1; bx.bz = e[2] - o[2] + 1;
    bx.px = lds_pitch(bx.bx);
    bx.py = lds_pitch(bx.by);
    return bx;
}

// Plan every chunk of the tile at once (thread i plans chunk i) and return
// the chunk length M for which all boxes fit `cap` voxels, or 0 if none
// does (the tile then reads its taps from global memory).  M shrinks in
// steps of max(2, M / 8) (16 -> 14 -> 12 ...): a tile whose widest box
// overflows by a few percent keeps most of its chunk length.
// Thread i < the chunk count leaves the record of chunk i in `rec`.
__device__ inline int plan_chunks(TileShared& sh, int Kmin, int Kmax, int Mmax, int cap,
                                  float step, float margin, int NX, int NY, int NZ, BoxRec& rec)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int M = Mmax;;) {
        const int nch = (Kmax - Kmin) / M + 1;
        if (nch > kMaxChunks) return 0;
        int vol = 0;
        if ((int)threadIdx.x < nch) {
            const int K = Kmin + (int)threadIdx.x * M;
            const Box b = chunk_box(sh, K, min(K + M - 1, Kmax), step, margin, NX, NY, NZ);
            rec.w[0] = (unsigned)b.ox | (unsigned)b.oy << 16;
            rec.w[1] = (unsigned)b.oz | (unsigned)b.bx << 16;
            rec.w[2] = (unsigned)b.by | (unsigned)b.bz << 16;
            vol = lds_pitch(b.bx) * lds_pitch(b.by) * b.bz;
        }
        for (int off = 32; off > 0; off >>= 1) vol = max(vol, __shfl_xor(vol, off));
        if (lane == 0) sh.vmax[wave] = vol;
        __syncthreads();
        const int vmax = max(max(sh.vmax[0], sh.vmax[1]), max(sh.vmax[2], sh.vmax[3]));
        __syncthreads();
        if (vmax <= cap) return M;
        if (M == 1) return 0;
        M = max(1, M - max(2, M >> 3));
    }
}

// Chunk records travel through the two slots of sh.cur: chunk ci is read
// from slot ci & 1 at the start of the chunk.  Its planner writes it after
// the first barrier of chunk ci - 1 (all reads of that slot, made at the
// start of chunk ci - 2, are done by then) and the second barrier of chunk
// ci - 1 publishes it; chunk 0 is written after planning, before a barrier
// of its own.
__device__ inline void publish_box(TileShared& sh, const BoxRec& rec, int ci)
{
    if ((int)threadIdx.x == ci) {
        unsigned* d = sh.cur[ci & 1];
        d[0] = rec.w[0]; d[1] = rec.w[1]; d[2] = rec.w[2];
    }
}

__device__ inline Box planned_box(const TileShared& sh, int ci)
{
    const unsigned* q = sh.cur[ci & 1];
    Box b;
    b.ox = q[0] & 0xFFFF; b.oy = q[0] >> 16; b.oz = q[1] & 0xFFFF;
    b.bx = q[1] >> 16; b.by = q[2] & 0xFFFF; b.bz = q[2] >> 16;
    b.px = lds_pitch(b.bx);
    b.py = lds_pitch(b.by);
    return b;
}

// Cooperative copy of a chunk box into LDS straight from the caller's volume
// (no padded copy, no precomputed gradient planes).  The box lives in padded
// index space: padded voxel (I, J, K) is grid voxel (I, J, K) - kPadV, and
// everything outside the grid reads as zero.  C floats per voxel, in the
// box's own x-fastest order (LDS index = C * ((z * py + y) * px + x); the
// pitch padding is never read):
//   C == 1: mu (forward);
//   C == 4: (mu, Gx, Gy, Gz) (pose gradient, with or without the SSD);
// G_c = the central difference of mu along c in index units (twice the
// gradient field; the factor 1/2 is applied to the per-ray sums) on grid
// voxels, mu zero-extended; G is zero off the grid.
//
// Interior boxes are staged in items: item i covers up to SEG consecutive
// voxels of one z column of the box (plane position p = i / nseg, z segment
// i mod nseg), so the position decode is paid once per SEG voxels.  Along an
// item the z neighbours slide (mu at z + 1 is the next voxel's centre): the
// gradient staging reads 2 + 5 SEG values per item (-z and the centre of its
// first voxel, then +z, -x, +x, -y, +y of each), the mu staging SEG.  An item
// shorter than SEG (the end of a column) re-reads its last voxel (in bounds,
// never stored).
template <int C>
struct BoxItem {
    static constexpr int SEG = C == 1 ? 8 : 4;
    static constexpr int NV = C == 1 ? SEG : 2 + 5 * SEG;
    float v[NV];
    unsigned slot;  // LDS index of the item's first voxel
    int cnt;        // voxels of the item (0: no item)
};

// Box-wide item decode constants (uniform over the block).
struct BoxItems {
    unsigned nseg, items, mseg, mx;
};

template <int C>
__device__ inline BoxItems box_items(const Box& b)
{
    BoxItems bi;
    bi.nseg = ((unsigned)b.bz + BoxItem<C>::SEG - 1) / BoxItem<C>::SEG;
    bi.items = (unsigned)(b.bx * b.by) * bi.nseg;
    // q = floor(e / d) = umulhi(e, floor(2^32 / d) + 1), exact for e * d < 2^32
    bi.mseg = bi.nseg > 1 ? 0xFFFFFFFFu / bi.nseg + 1u : 0u;
    bi.mx = b.bx > 1 ? 0xFFFFFFFFu / (unsigned)b.bx + 1u : 0u;
    return bi;
}

// Load at a byte offset from the volume base (offsets stay below 4 GiB: the
// volume has at most 2^30 voxels).
__device__ inline float ldv(const float* __restrict__ mu, unsigned boff)
{
    return *(const float*)((const char*)mu + boff);
}

// Issue the loads of item `it` of an interior box.
template <int C>
__device__ inline void item_load(const Box& b, const BoxItems& bi, unsigned it,
                                 const float* __restrict__ mu, int nx, int ny, BoxItem<C>& r)
{
    constexpr int SEG = BoxItem<C>::SEG;
    const unsigned p = bi.nseg > 1 ? __umulhi(it, bi.mseg) : it;
    const unsigned sg = it - p * bi.nseg;
    const unsigned ly = b.bx > 1 ? __umulhi(p, bi.mx) : p;
    const unsigned lx = p - ly * (unsigned)b.bx;
    const unsigned z0 = sg * SEG;
    r.cnt = min(SEG, b.bz - (int)z0);
    const unsigned nx4 = 4u * (unsigned)nx, nxy4 = nx4 * (unsigned)ny;
    const unsigned i = (unsigned)b.ox + lx - kPadV, j = (unsigned)b.oy + ly - kPadV;
    const unsigned k0 = (unsigned)b.oz + z0 - kPadV;
    const unsigned o0 = ((k0 * (unsigned)ny + j) * (unsigned)nx + i) * 4u;
    const unsigned olast = o0 + (unsigned)(r.cnt - 1) * nxy4;
    r.slot = (unsigned)C * ((z0 * (unsigned)b.py + ly) * (unsigned)b.px + lx);
    if constexpr (C == 1) {
#pragma unroll
        for (int q = 0; q < SEG; ++q) r.v[q] = ldv(mu, min(o0 + (unsigned)q * nxy4, olast));
    } else {
        r.v[0] = ldv(mu, o0 - nxy4);
        r.v[1] = ldv(mu, o0);
#pragma unroll
        for (int q = 0; q < SEG; ++q) {
            const unsigned o = min(o0 + (unsigned)q * nxy4, olast);
            r.v[2 + 5 * q + 0] = ldv(mu, o + nxy4);
            r.v[2 + 5 * q + 1] = ldv(mu, o - 4u);
            r.v[2 + 5 * q + 2] = ldv(mu, o + 4u);
            r.v[2 + 5 * q + 3] = ldv(mu, o - nx4);
            r.v[2 + 5 * q + 4] = ldv(mu, o + nx4);
        }
    }
}

template <int C>
__device__ inline void box_store(float* dst, unsigned slot, float m, float gx, float gy, float gz)
{
    float* d = dst + slot;
    static_assert(C == 1 || C == 4, "boxes hold mu or (mu, Gx, Gy, Gz)");
    if constexpr (C == 4) {  // one 16-byte store: lanes 16 B apart, no bank conflict
        *reinterpret_cast<float4*>(d) = make_float4(m, gx, gy, gz);
    } else {
        d[0] = m;
    }
}

// Form the staged values of a loaded item and store them to LDS.
template <int C>
__device__ inline void item_store(const Box& b, const BoxItem<C>& r, float* dst)
{
    constexpr int SEG = BoxItem<C>::SEG;
    const unsigned dslot = (unsigned)(C * b.py * b.px);
    unsigned slot = r.slot;
#pragma unroll
    for (int q = 0; q < SEG; ++q, slot += dslot) {
        if (q >= r.cnt) break;
        if constexpr (C == 1) {
            box_store<C>(dst, slot, r.v[q], 0.f, 0.f, 0.f);
        } else {
            const float c = q == 0 ? r.v[1] : r.v[2 + 5 * (q - 1)];
            const float zm = q == 0 ? r.v[0] : (q == 1 ? r.v[1] : r.v[2 + 5 * (q - 2)]);
            const float* w = &r.v[2 + 5 * q];
            box_store<C>(dst, slot, c, w[2] - w[1], w[4] - w[3], w[0] - zm);
        }
    }
}

// True if every voxel of the box lies on the grid, with a one-voxel margin
// when its neighbours are read too (C >= 3).
template <int C>
__device__ inline bool box_interior(const Box& b, int nx, int ny, int nz)
{
    constexpr int m = C >= 3 ? 1 : 0;
    return b.ox - kPadV >= m && b.oy - kPadV >= m && b.oz - kPadV >= m &&
           b.ox - kPadV + b.bx + m <= nx && b.oy - kPadV + b.by + m <= ny &&
           b.oz - kPadV + b.bz + m <= nz;
}

// Interior box, volume rows 16-byte aligned (nx a multiple of 4 and an
// aligned base), at least kVecSeg voxels deep: the box is covered by aligned
// 4-voxel x segments, and item i is one segment of one box row over kVecSeg
// consecutive z (segment fastest, so a wavefront's loads are contiguous
// 16-byte pieces of a row).  The last z run of a column starts at
// bz - kVecSeg and overlaps the one before it (those voxels are stored
// twice, with the same values), so every item spans kVecSeg planes inside
// the box.  Per z step an item loads the +z, -y and +y rows as 16-byte
// vectors and the two x neighbours of the segment as scalars: 5 loads for 4
// voxels instead of 20.  Segment voxels outside the box (at most 3 at either
// end of a row) are loaded and not stored.
//
// The loads are raw buffer loads over the volume: one per-lane offset per
// item (three with the x neighbours) and the plane and row steps as
// wavefront-uniform offsets, so no per-load address arithmetic.  Every
// address is inside the volume: the box keeps a one-voxel margin to the
// grid faces, and an aligned segment of a row containing a box voxel ends
// inside the row (nx is a multiple of 4); at the row ends the x neighbour
// falls back onto the segment voxel itself, which the margin keeps out of
// the box.
constexpr int kVecSeg = 4;

struct VecItems {
    int gx0;               // first grid x of the box
    unsigned s0, nxs;      // first aligned segment, segments per row
    unsigned nseg, items;  // z runs per column, items of the box
    unsigned mxs, mby;     // division magics for nxs and by
};

__device__ inline VecItems vec_items(const Box& b)
{
    VecItems vi;
    vi.gx0 = b.ox - kPadV;
    vi.s0 = (unsigned)vi.gx0 >> 2;
    vi.nxs = ((unsigned)(vi.gx0 + b.bx - 1) >> 2) - vi.s0 + 1;
    vi.nseg = ((unsigned)b.bz + kVecSeg - 1) / kVecSeg;
    vi.items = vi.nxs * (unsigned)b.by * vi.nseg;
    vi.mxs = vi.nxs > 1 ? 0xFFFFFFFFu / vi.nxs + 1u : 0u;
    vi.mby = b.by > 1 ? 0xFFFFFFFFu / (unsigned)b.by + 1u : 0u;
    return vi;
}

// Raw buffer over the volume (gfx9 descriptor: 32-bit data, no swizzle).
__device__ inline __amdgpu_buffer_rsrc_t vol_rsrc(const float* __restrict__ mu, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void*)mu, (short)0, (int)bytes, 0x00020000);
}

__device__ inline float4 bload4(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

__device__ inline float bload1(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ inline float f4at(const float4& v, int e)
{
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}

template <int C>
__device__ inline void vec_item(const Box& b, const VecItems& vi, unsigned it,
                                __amdgpu_buffer_rsrc_t vr, int nx, int ny, float* dst)
{
    const unsigned t = vi.nxs > 1 ? __umulhi(it, vi.mxs) : it;
    const unsigned xs = it - t * vi.nxs;
    const unsigned zs = b.by > 1 ? __umulhi(t, vi.mby) : t;
    const unsigned ly = t - zs * (unsigned)b.by;
    const int gxs = (int)(vi.s0 + xs) * 4;        // grid x of the segment's first voxel
    const int lx0 = gxs - vi.gx0;                 // its box x (may be negative)
    const unsigned z0 = min(zs * kVecSeg, (unsigned)b.bz - kVecSeg);
    const unsigned nx4 = 4u * (unsigned)nx, nxy4 = nx4 * (unsigned)ny;
    const unsigned j = (unsigned)b.oy + ly - kPadV, k0 = (unsigned)b.oz + z0 - kPadV;
    const unsigned o0 = ((k0 * (unsigned)ny + j) * (unsigned)nx + (unsigned)gxs) * 4u;
    const unsigned dslot = (unsigned)(C * b.py * b.px);
    // LDS index of segment voxel e at the item's first z (only for 0 <= lx0 + e < bx)
    const int slot0 = C * (((int)z0 * b.py + (int)ly) * b.px + lx0);
    // which segment voxels lie in the box (the same at every z of the item)
    bool inb[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) inb[e] = (unsigned)(lx0 + e) < (unsigned)b.bx;
    if constexpr (C == 1) {
        float4 v[kVecSeg];
#pragma unroll
        for (int q = 0; q < kVecSeg; ++q) v[q] = bload4(vr, o0, (unsigned)q * nxy4);
        unsigned sq = (unsigned)slot0;
#pragma unroll
        for (int q = 0; q < kVecSeg; ++q, sq += dslot)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (inb[e]) dst[sq + (unsigned)e] = f4at(v[q], e);
    } else {
        // base: the item's first voxel one plane down (k0 >= 1 in an interior box)
        const unsigned vb = o0 - nxy4;
        const unsigned vl = vb - (gxs > 0 ? 4u : 0u), vrt = vb + (gxs + 4 < nx ? 16u : 12u);
        float4 zc[kVecSeg + 2], ym[kVecSeg], yp[kVecSeg];
        float xl[kVecSeg], xr[kVecSeg];
        zc[0] = bload4(vr, vb, 0u);
        zc[1] = bload4(vr, vb, nxy4);
#pragma unroll
        for (int q = 0; q < kVecSeg; ++q) {
            const unsigned pl = (unsigned)(q + 1) * nxy4;  // plane of voxel row q
            zc[q + 2] = bload4(vr, vb, pl + nxy4);
            ym[q] = bload4(vr, vb, pl - nx4);
            yp[q] = bload4(vr, vb, pl + nx4);
            xl[q] = bload1(vr, vl, pl);
            xr[q] = bload1(vr, vrt, pl);
        }
        // LDS index of the segment's first voxel at plane q of the item
        // (modulo 2^32; voxels outside the box are never stored)
        unsigned sq = (unsigned)slot0;
#pragma unroll
        for (int q = 0; q < kVecSeg; ++q, sq += dslot) {
            const float4 c = zc[q + 1], zm = zc[q], zp = zc[q + 2];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (!inb[e]) continue;
                const float right = e < 3 ? f4at(c, e + 1) : xr[q];
                const float left = e > 0 ? f4at(c, e - 1) : xl[q];
                box_store<C>(dst, sq + (unsigned)(C * e), f4at(c, e), right - left,
                             f4at(yp[q], e) - f4at(ym[q], e), f4at(zp, e) - f4at(zm, e));
            }
        }
    }
}

template <int C>
__device__ inline void load_box_vec(const Box& b, const float* __restrict__ mu, int nx, int ny,
                                    unsigned vol_bytes, float* dst)
{
    const VecItems vi = vec_items(b);
    const __amdgpu_buffer_rsrc_t vr = vol_rsrc(mu, vol_bytes);
    for (unsigned it = threadIdx.x; it < vi.items; it += kRdThreads)
        vec_item<C>(b, vi, it, vr, nx, ny, dst);
}

// Interior box staged in one go: every item loaded and stored, two items per
// thread in flight.
template <int C>
__device__ inline void load_box_interior(const Box& b, const float* __restrict__ mu, int nx,
                                         int ny, float* dst)
{
    const BoxItems bi = box_items<C>(b);
    for (unsigned it = threadIdx.x; it < bi.items; it += 2 * kRdThreads) {
        BoxItem<C> r0, r1;
        r1.cnt = 0;
        item_load<C>(b, bi, it, mu, nx, ny, r0);
        if (it + kRdThreads < bi.items) item_load<C>(b, bi, it + kRdThreads, mu, nx, ny, r1);
        item_store<C>(b, r0, dst);
        if (r1.cnt > 0) item_store<C>(b, r1, dst);
    }
}

// Box touching the grid's faces (or beyond): every voxel tested, neighbour
// offsets clamped onto the voxel itself at the grid faces and their values
// masked, loads only for voxels on the grid.
template <int C>
__device__ inline void load_box_edge(const Box& b, const float* __restrict__ mu, int nx, int ny,
                                     int nz, float* dst)
{
    const int nxy = nx * ny;
    const unsigned dslot = (unsigned)(C * b.py * b.px);
    const BoxItems bi = box_items<C>(b);
    constexpr int SEG = BoxItem<C>::SEG;
    for (unsigned it = threadIdx.x; it < bi.items; it += kRdThreads) {
        const unsigned p = bi.nseg > 1 ? __umulhi(it, bi.mseg) : it;
        const unsigned sg = it - p * bi.nseg;
        const unsigned uly = b.bx > 1 ? __umulhi(p, bi.mx) : p;
        struct { int lx, ly, z0, z1; } w;
        w.lx = (int)(p - uly * (unsigned)b.bx);
        w.ly = (int)uly;
        w.z0 = (int)sg * SEG;
        w.z1 = min(w.z0 + SEG, b.bz);
        const int i = b.ox + w.lx - kPadV, j = b.oy + w.ly - kPadV;
        const bool col = (unsigned)i < (unsigned)nx && (unsigned)j < (unsigned)ny;
        const bool fxm = i > 0, fxp = i + 1 < nx, fym = j > 0, fyp = j + 1 < ny;
        const int oxm = fxm ? -1 : 0, oxp = fxp ? 1 : 0;
        const int oym = fym ? -nx : 0, oyp = fyp ? nx : 0;
        int k = b.oz + w.z0 - kPadV;
        int off = (k * ny + j) * nx + i;  // element offset, meaningful only on the grid
        unsigned slot = (unsigned)C * (((unsigned)w.z0 * (unsigned)b.py + (unsigned)w.ly) *
                                       (unsigned)b.px + (unsigned)w.lx);
        for (int z = w.z0; z < w.z1; ++z, ++k, off += nxy, slot += dslot) {
            float m = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
            if (col && (unsigned)k < (unsigned)nz) {
                const float* pc = mu + off;
                m = pc[0];
                if constexpr (C >= 3) {
                    const bool fzm = k > 0, fzp = k + 1 < nz;
                    const float xm = pc[oxm], xp = pc[oxp], ym = pc[oym], yp = pc[oyp];
                    const float zm = pc[fzm ? -nxy : 0], zp = pc[fzp ? nxy : 0];
                    gx = (fxp ? xp : 0.0f) - (fxm ? xm : 0.0f);
                    gy = (fyp ? yp : 0.0f) - (fym ? ym : 0.0f);
                    gz = (fzp ? zp : 0.0f) - (fzm ? zm : 0.0f);
                }
            }
            box_store<C>(dst, slot, m, gx, gy, gz);
        }
    }
}

// Wait for every outstanding vector-memory load of this wavefront (s_waitcnt
// vmcnt(0), expcnt and lgkmcnt left at their maxima).  A staging step ends
// with it: the items it loaded and stored are complete by then, and the
// compiler's wait tracking otherwise keeps the re-read tails of short items
// (loaded, never stored) pending into the sample loop, where it stalls on
// them at the loop's first LDS reads.
__device__ inline void vm_drain() { __builtin_amdgcn_s_waitcnt(0x0F70); }

template <int C>
__device__ inline void load_box(const Box& b, const float* __restrict__ mu, int nx, int ny, int nz,
                                float* dst)
{
    // uniform over the block; rows of mu are 16-byte aligned when nx % 4 == 0;
    // the buffer loads cover volumes below 4 GiB
    if (box_interior<C>(b, nx, ny, nz)) {
        const size_t vol_bytes = (size_t)nx * ny * nz * sizeof(float);
        if (RD_VEC_ROWS && (nx & 3) == 0 && ((uintptr_t)mu & 15) == 0 && b.bz >= kVecSeg &&
            vol_bytes <= 0xFFFFFFF0u)
            load_box_vec<C>(b, mu, nx, ny, (unsigned)vol_bytes, dst);
        else
            load_box_interior<C>(b, mu, nx, ny, dst);
    } else {
        load_box_edge<C>(b, mu, nx, ny, nz, dst);
    }
    vm_drain();
}


// mu at padded voxel (I, J, K): zero off the grid.
__device__ inline float mu_at(const float* __restrict__ mu, int nx, int ny, int nz, int I, int J,
                              int K)
{
    const int i = I - kPadV, j = J - kPadV, k = K - kPadV;
    if ((unsigned)i >= (unsigned)nx || (unsigned)j >= (unsigned)ny || (unsigned)k >= (unsigned)nz)
        return 0.0f;
    return mu[((size_t)k * ny + j) * nx + i];
}

// mu and (Gx, Gy, Gz) at the 8 trilinear corners of base padded voxel
// (I, J, K), as the box loaders form them, from the 32 voxels they need:
// the 2x2x2 core and, per axis, the two voxels beyond it on the 4 core lines
// along that axis.
__device__ inline void corners_at(const float* __restrict__ mu, int nx, int ny, int nz, int I,
                                  int J, int K, float (&m)[2][2][2], float3 (&q)[2][2][2])
{
    float xo[2][2][2], yo[2][2][2], zo[2][2][2];  // [line][line][-1 / +2 side]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int c = 0; c < 2; ++c) m[a][b][c] = mu_at(mu, nx, ny, nz, I + c, J + b, K + a);
            xo[a][b][0] = mu_at(mu, nx, ny, nz, I - 1, J + b, K + a);  // [dz][dy]
            xo[a][b][1] = mu_at(mu, nx, ny, nz, I + 2, J + b, K + a);
            yo[a][b][0] = mu_at(mu, nx, ny, nz, I + b, J - 1, K + a);  // [dz][dx]
            yo[a][b][1] = mu_at(mu, nx, ny, nz, I + b, J + 2, K + a);
            zo[a][b][0] = mu_at(mu, nx, ny, nz, I + b, J + a, K - 1);  // [dy][dx]
            zo[a][b][1] = mu_at(mu, nx, ny, nz, I + b, J + a, K + 2);
        }
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int i = I + dx - kPadV, j = J + dy - kPadV, k = K + dz - kPadV;
                const bool on = (unsigned)i < (unsigned)nx && (unsigned)j < (unsigned)ny &&
                                (unsigned)k < (unsigned)nz;
                const float xp = dx ? xo[dz][dy][1] : m[dz][dy][1], xm = dx ? m[dz][dy][0] : xo[dz][dy][0];
                const float yp = dy ? yo[dz][dx][1] : m[dz][1][dx], ym = dy ? m[dz][0][dx] : yo[dz][dx][0];
                const float zp = dz ? zo[dy][dx][1] : m[1][dy][dx], zm = dz ? m[0][dy][dx] : zo[dy][dx][0];
                q[dz][dy][dx] = on ? make_float3(xp - xm, yp - ym, zp - zm) : make_float3(0.f, 0.f, 0.f);
            }
}

// LDS voxel index of a sample's base corner from its (integral) float value,
// clamped to [0, hi] with one median-of-three (the planned box holds every
// tap; the clamp only keeps rounding at the box faces inside the array).
__device__ inline int lds_index(float f, float hi)
{
    return (int)__builtin_amdgcn_fmed3f(f, 0.0f, hi);
}

// One chunk of one ray: first local position and per-sample increment.
struct ChunkRay {
    float X, Y, Z;     // local box coordinates of sample kb
    float sx, sy, sz;  // step * direction
    float n;           // number of samples - 1 (negative: none)
};

__device__ inline ChunkRay chunk_ray(const RayState& r, int kb, int ke, const Box& bx, float step)
{
    ChunkRay c;
    const float tb = fmaf((float)(kb - r.k0), step, r.f);
    c.X = fmaf(tb, r.dx, r.x0 - (float)bx.ox);
    c.Y = fmaf(tb, r.dy, r.y0 - (float)bx.oy);
    c.Z = fmaf(tb, r.dz, r.z0 - (float)bx.oz);
    c.sx = step * r.dx; c.sy = step * r.dy; c.sz = step * r.dz;
    c.n = (float)(ke - kb);
    return c;
}

template <int TW, int MCH, int CAP>
__device__ inline void rd_fwd_tile(const GeoScalars& s, const ViewGeo* __restrict__ views,
                                   const float* __restrict__ mu, float* __restrict__ proj,
                                   int v, int tile, float* lds, TileShared& sh)
{
    int a, b, a0, b0;
    rd_pixel<TW>(s, tile, a, b, a0, b0);
    const bool active = a < s.nu && b < s.nv;
    const ViewGeo& g = views[v];
    const RayState r = ray_setup(s, g, min(a, s.nu - 1), min(b, s.nv - 1));
    int Kmin, Kmax;
    float margin;
    tile_setup<TW>(s, r, active, active, a, b, a0, b0, sh, Kmin, Kmax, margin);
    const int NX = s.nx + 2 * kPadV, NY = s.ny + 2 * kPadV, NZ = s.nz + 2 * kPadV;
    const float step = (float)s.step;
    const int klo = active ? r.klo : 1, khi = active ? r.khi : 0;
    float acc = 0.0f;
    BoxRec rec = {};
    const int M = Kmin <= Kmax ? plan_chunks(sh, Kmin, Kmax, MCH, CAP, step, margin, NX, NY, NZ,
                                             rec)
                               : 1;
    if (M > 0) {
        publish_box(sh, rec, 0);
        __syncthreads();
        for (int K = Kmin, ci = 0; K <= Kmax; K += M, ++ci) {
            const int Ke = min(K + M - 1, Kmax);
            const Box bx = planned_box(sh, ci);
            __syncthreads();  // the previous chunk's readers are done
            publish_box(sh, rec, ci + 1);
            load_box<1>(bx, mu, s.nx, s.ny, s.nz, lds);
            __syncthreads();
            const int kb = max(K, klo), ke = min(Ke, khi);
            const ChunkRay c = chunk_ray(r, kb, ke, bx, step);
            const int BX = bx.px, BXY = bx.px * bx.py;
            const float fbx = (float)bx.px, fby = (float)bx.py;
            const float fimax = (float)(CAP - 1 - (BXY + BX + 1));
            // sample j of the chunk, its position measured from (X0, Y0, Z0)
            auto sample = [&](float j, float X0, float Y0, float Z0) {
                const float X = fmaf(j, c.sx, X0), Y = fmaf(j, c.sy, Y0), Z = fmaf(j, c.sz, Z0);
                const float fx = floorf(X), fy = floorf(Y), fz = floorf(Z);
                const float wx = X - fx, wy = Y - fy, wz = Z - fz;
                const int idx = lds_index(fmaf(fmaf(fz, fby, fy), fbx, fx), fimax);
                const float* p = lds + idx;
                const float c00 = lerpf(p[0], p[1], wx);
                const float c10 = lerpf(p[BX], p[BX + 1], wx);
                const float c01 = lerpf(p[BXY], p[BXY + 1], wx);
                const float c11 = lerpf(p[BXY + BX], p[BXY + BX + 1], wx);
                acc += lerpf(lerpf(c00, c10, wy), lerpf(c01, c11, wy), wz);
            };
            // two samples per trip (the second from the next sample's origin),
            // then the odd one
            const float X1 = c.X + c.sx, Y1 = c.Y + c.sy, Z1 = c.Z + c.sz, n1 = c.n - 1.0f;
            float j = 0.0f;
            for (; j <= n1; j += 2.0f) {
                sample(j, c.X, c.Y, c.Z);
                sample(j, X1, Y1, Z1);
            }
            if (j <= c.n) sample(j, c.X, c.Y, c.Z);
        }
    } else {
        // chunk boxes too large for LDS: taps straight from the volume
        const float xmax = NX - 1.001f, ymax = NY - 1.001f, zmax = NZ - 1.001f;
        for (int k = klo; k <= khi; ++k) {
            const float t = fmaf((float)(k - r.k0), step, r.f);
            const float X = fminf(fmaxf(fmaf(t, r.dx, r.x0), 0.0f), xmax);
            const float Y = fminf(fmaxf(fmaf(t, r.dy, r.y0), 0.0f), ymax);
            const float Z = fminf(fmaxf(fmaf(t, r.dz, r.z0), 0.0f), zmax);
            const float fx = floorf(X), fy = floorf(Y), fz = floorf(Z);
            const float wx = X - fx, wy = Y - fy, wz = Z - fz;
            const int I = (int)fx, J = (int)fy, Kz = (int)fz;
            float m[2][2][2];
#pragma unroll
            for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 2; ++dx)
                        m[dz][dy][dx] = mu_at(mu, s.nx, s.ny, s.nz, I + dx, J + dy, Kz + dz);
            const float c00 = lerpf(m[0][0][0], m[0][0][1], wx);
            const float c10 = lerpf(m[0][1][0], m[0][1][1], wx);
            const float c01 = lerpf(m[1][0][0], m[1][0][1], wx);
            const float c11 = lerpf(m[1][1][0], m[1][1][1], wx);
            acc += lerpf(lerpf(c00, c10, wy), lerpf(c01, c11, wy), wz);
        }
    }
    if (active) proj[((size_t)v * s.nv + b) * s.nu + a] = acc * step;
}

// Deterministic block reduction of C channels: butterfly within each
// wavefront, then a fixed-order sum over the 4 wavefronts through `red`
// (4 C floats of LDS; the kernels pass their box array, whose readers the
// leading barrier waits for).
template <int C>
__device__ inline void block_reduce_store(float (&v)[C], float* red, float* __restrict__ out)
{
#pragma unroll
    for (int c = 0; c < C; ++c)
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) red[wave * C + c] = v[c];
    }
    __syncthreads();
    if (threadIdx.x < C) {
        const int c = threadIdx.x;
        out[c] = ((red[c] + red[C + c]) + red[2 * C + c]) + red[3 * C + c];
    }
}

// Trilinear weights phi[dz][dy][dx] of the 8 corners around a sample with
// fractional offsets (wx, wy, wz), formed with 13 operations (products of
// the y-z pair weights with wx, complements by subtraction).
struct Tri {
    float p[2][2][2];
};

__device__ inline Tri tri_weights(float wx, float wy, float wz)
{
    Tri t;
    const float yz11 = wy * wz, yz01 = wz - yz11, yz10 = wy - yz11;  // [dy][dz]
    const float yz00 = (1.0f - wz) - yz10;
    const float pr[2][2] = {{yz00, yz10}, {yz01, yz11}};              // [dz][dy]
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            t.p[dz][dy][1] = pr[dz][dy] * wx;
            t.p[dz][dy][0] = pr[dz][dy] - t.p[dz][dy][1];
        }
    return t;
}

// sum_j phi_j m_j (formed on its own, so that a running sum it is added to
// takes one rounding per sample)
__device__ inline float tri_dot(const Tri& t, const float (&m)[2][2][2])
{
    float v = t.p[0][0][0] * m[0][0][0];
#pragma unroll
    for (int q = 1; q < 8; ++q) v = fmaf(t.p[q >> 2][(q >> 1) & 1][q & 1], m[q >> 2][(q >> 1) & 1][q & 1], v);
    return v;
}

// Per-ray gradient sums.  add() takes the 8 corner gradient vectors q (index
// units), their trilinear weights and the base corner's index P in some
// frame; T accumulates sum phi P_a G_c + sum phi delta_a G_c.  A change of
// frame P -> P + d moves the sums with T_ac += d_a B_c (shift()).
struct GradAcc {
    float Bx = 0.f, By = 0.f, Bz = 0.f;
    float Txy = 0.f, Txz = 0.f, Tyx = 0.f, Tyz = 0.f, Tzx = 0.f, Tzy = 0.f;

    // One channel: value v = sum phi g and the moments ma = sum_{delta_a = 1}
    // phi g, mb = sum_{delta_b = 1} phi g over its two other axes a, b.  The
    // weights come in four pairs by (delta_a, delta_b); the (1, 1) pair is
    // shared by both moments.
    __device__ static inline void channel(const float (&ph)[2][2][2], const float (&gv)[2][2][2],
                                          float& v, float& ma, float& mb)
    {
        // ph, gv indexed [delta_b][delta_a][delta_c]
        const float s11 = fmaf(ph[1][1][1], gv[1][1][1], ph[1][1][0] * gv[1][1][0]);
        const float s01 = fmaf(ph[0][1][1], gv[0][1][1], ph[0][1][0] * gv[0][1][0]);  // a only
        const float s10 = fmaf(ph[1][0][1], gv[1][0][1], ph[1][0][0] * gv[1][0][0]);  // b only
        ma = s11 + s01;
        mb = s11 + s10;
        v = fmaf(ph[0][0][1], gv[0][0][1], fmaf(ph[0][0][0], gv[0][0][0], ma + s10));
    }

    __device__ inline void add(const float3 (&q)[2][2][2], const Tri& t, float Px, float Py,
                               float Pz)
    {
        // Regroup weights and values per channel as [delta_b][delta_a][delta_c].
        float px[2][2][2], gxv[2][2][2];  // Gx: a = y, b = z
        float py[2][2][2], gyv[2][2][2];  // Gy: a = x, b = z
        float pz[2][2][2], gzv[2][2][2];  // Gz: a = x, b = y
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    const float w = t.p[dz][dy][dx];
                    px[dz][dy][dx] = w; gxv[dz][dy][dx] = q[dz][dy][dx].x;
                    py[dz][dx][dy] = w; gyv[dz][dx][dy] = q[dz][dy][dx].y;
                    pz[dy][dx][dz] = w; gzv[dy][dx][dz] = q[dz][dy][dx].z;
                }
        float Gx, Myx, Mzx, Gy, Mxy, Mzy, Gz, Mxz, Myz;
        channel(px, gxv, Gx, Myx, Mzx);
        channel(py, gyv, Gy, Mxy, Mzy);
        channel(pz, gzv, Gz, Mxz, Myz);
        Bx += Gx; By += Gy; Bz += Gz;
        Txy = fmaf(Px, Gy, Txy) + Mxy; Txz = fmaf(Px, Gz, Txz) + Mxz;
        Tyx = fmaf(Py, Gx, Tyx) + Myx; Tyz = fmaf(Py, Gz, Tyz) + Myz;
        Tzx = fmaf(Pz, Gx, Tzx) + Mzx; Tzy = fmaf(Pz, Gy, Tzy) + Mzy;
    }

    // Re-express the sums in the frame P + d.
    __device__ inline void shift(float dx, float dy, float dz)
    {
        Txy = fmaf(dx, By, Txy); Txz = fmaf(dx, Bz, Txz);
        Tyx = fmaf(dy, Bx, Tyx); Tyz = fmaf(dy, Bz, Tyz);
        Tzx = fmaf(dz, Bx, Tzx); Tzy = fmaf(dz, By, Tzy);
    }
};

template <int TW, int MCH, int CAP, bool FUSED, bool HESS = false>
__device__ inline void rd_grad_tile(const GeoScalars& s, const ViewGeo* __restrict__ views,
                                    const float* __restrict__ mu,
                                    const float4* __restrict__ inter,
                                    const float* __restrict__ gin,
                                    float* __restrict__ proj_out,
                                    float* __restrict__ partials, int v, int tile, int tiles,
                                    float* lds, TileShared& sh)
{
    // FUSED: gin is the target image y, and the ray also integrates mu: l is
    // written to proj_out and the SSD weight w = 2 (l - y) is applied to the
    // gradient sums at the end.  Otherwise gin is dL/dl.  The chunk boxes
    // hold (mu, Gx, Gy, Gz) per voxel in both modes, formed from mu while
    // loading: one aligned 16-byte LDS read per corner (the gradient-only
    // mode ignores mu).  Tiles whose boxes do not fit the LDS gather the same
    // values per trilinear corner: one float4 per corner from `inter` (a
    // padded (mu, Gx, Gy, Gz) copy the caller makes for sparse-ray
    // geometries, where such tiles are common), else from mu directly.
    constexpr int C = 4;
    int a, b, a0, b0;
    rd_pixel<TW>(s, tile, a, b, a0, b0);
    const bool inside = a < s.nu && b < s.nv;
    const size_t pix = ((size_t)v * s.nv + min(b, s.nv - 1)) * s.nu + min(a, s.nu - 1);
    const float gpix = inside ? gin[pix] : 0.0f;
    const ViewGeo& g = views[v];
    const RayState r = ray_setup(s, g, min(a, s.nu - 1), min(b, s.nv - 1));
    // unfused: rays with dL/dl = 0 contribute nothing, they only help load
    // the boxes; fused: w is known only after the march
    const bool active = FUSED ? inside : (inside && gpix != 0.0f);
    float lsum = 0.0f;
    int Kmin, Kmax;
    float margin;
    tile_setup<TW>(s, r, inside, active, a, b, a0, b0, sh, Kmin, Kmax, margin);
    const int NX = s.nx + 2 * kPadV, NY = s.ny + 2 * kPadV, NZ = s.nz + 2 * kPadV;
    const float step = (float)s.step;
    // Padded index of the grid centre: P_a(j) = I_a(j) - centre_a.
    const float ccx = 0.5f * (s.nx - 1) + kPadV, ccy = 0.5f * (s.ny - 1) + kPadV,
                ccz = 0.5f * (s.nz - 1) + kPadV;
    const int klo = active ? r.klo : 1, khi = active ? r.khi : 0;
    GradAcc G;
    BoxRec rec = {};
    const int M = Kmin <= Kmax ? plan_chunks(sh, Kmin, Kmax, MCH, CAP, step, margin, NX, NY, NZ,
                                             rec)
                               : 1;
    if (M > 0) {
        publish_box(sh, rec, 0);
        __syncthreads();
        // G runs through the chunks in the base-corner frame of the current
        // chunk's box (P = local box index); it moves to the next box's
        // frame at each chunk and to the grid-centred frame at the end.
        int fox = 0, foy = 0, foz = 0;  // origin of G's frame (G is zero at first)
        for (int K = Kmin, ci = 0; K <= Kmax; K += M, ++ci) {
            const int Ke = min(K + M - 1, Kmax);
            const Box bx = planned_box(sh, ci);
            G.shift((float)(fox - bx.ox), (float)(foy - bx.oy), (float)(foz - bx.oz));
            fox = bx.ox; foy = bx.oy; foz = bx.oz;
            __syncthreads();  // the previous chunk's readers are done
            publish_box(sh, rec, ci + 1);
            load_box<C>(bx, mu, s.nx, s.ny, s.nz, lds);
            __syncthreads();
            const int kb = max(K, klo), ke = min(Ke, khi);
            const ChunkRay c = chunk_ray(r, kb, ke, bx, step);
            const int BXC = C * bx.px, BXYC = C * bx.px * bx.py;
            const float fbx = (float)bx.px, fby = (float)bx.py;
            // largest base voxel whose 2x2x2 corners stay inside the box
            const float fvmax = (float)(CAP - 2 - (bx.px * bx.py + bx.px));
            // sample j of the chunk, its position measured from (X0, Y0, Z0)
            auto sample = [&](float j, float X0, float Y0, float Z0) {
                const float X = fmaf(j, c.sx, X0), Y = fmaf(j, c.sy, Y0), Z = fmaf(j, c.sz, Z0);
                const float fx = floorf(X), fy = floorf(Y), fz = floorf(Z);
                const int idx = C * lds_index(fmaf(fmaf(fz, fby, fy), fbx, fx), fvmax);
                const float* p = lds + idx;
                float3 q[2][2][2];
                float m[2][2][2];
#pragma unroll
                for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 2; ++dx) {
                            const float* o = p + dz * BXYC + dy * BXC + C * dx;
                            const v4f t = *(lds_v4f*)o;
                            m[dz][dy][dx] = t[0];
                            q[dz][dy][dx] = make_float3(t[1], t[2], t[3]);
                        }
                const Tri t = tri_weights(X - fx, Y - fy, Z - fz);
                if (FUSED) lsum += tri_dot(t, m);
                G.add(q, t, fx, fy, fz);
                if constexpr (!FUSED) {
                    // The gradient-only mode has no use for mu; this empty statement
                    // keeps its 8 lanes live to the end of the sample, so that the
                    // reads stay whole 16-byte ds_read_b128 and their registers are
                    // not reused while a read is still in flight (which would make
                    // the wavefront wait for each read in turn).
                    asm volatile("" ::"v"(m[0][0][0]), "v"(m[0][0][1]), "v"(m[0][1][0]),
                                 "v"(m[0][1][1]), "v"(m[1][0][0]), "v"(m[1][0][1]),
                                 "v"(m[1][1][0]), "v"(m[1][1][1]));
                }
            };
            // two samples per trip (the second from the next sample's origin),
            // then the odd one
            const float X1 = c.X + c.sx, Y1 = c.Y + c.sy, Z1 = c.Z + c.sz, n1 = c.n - 1.0f;
            float j = 0.0f;
            for (; j <= n1; j += 2.0f) {
                sample(j, c.X, c.Y, c.Z);
                sample(j, X1, Y1, Z1);
            }
            if (j <= c.n) sample(j, c.X, c.Y, c.Z);
        }
        G.shift((float)fox - ccx, (float)foy - ccy, (float)foz - ccz);
    } else {
        const float xmax = NX - 1.001f, ymax = NY - 1.001f, zmax = NZ - 1.001f;
        // clamped padded position of sample k
        auto position = [&](int k, float& X, float& Y, float& Z) {
            const float tk = fmaf((float)(k - r.k0), step, r.f);
            X = fminf(fmaxf(fmaf(tk, r.dx, r.x0), 0.0f), xmax);
            Y = fminf(fmaxf(fmaf(tk, r.dy, r.y0), 0.0f), ymax);
            Z = fminf(fmaxf(fmaf(tk, r.dz, r.z0), 0.0f), zmax);
        };
        auto accumulate = [&](float X, float Y, float Z, const float (&m)[2][2][2],
                              const float3 (&q)[2][2][2]) {
            const float fx = floorf(X), fy = floorf(Y), fz = floorf(Z);
            const Tri t = tri_weights(X - fx, Y - fy, Z - fz);
            if (FUSED) lsum += tri_dot(t, m);
            G.add(q, t, fx - ccx, fy - ccy, fz - ccz);
        };
        if (inter) {
            // the 8 corner vectors of sample k from the padded (mu, G) copy
            const int NXY = NX * NY;
            auto gather = [&](float X, float Y, float Z, float (&m)[2][2][2],
                              float3 (&q)[2][2][2]) {
                const int idx = ((int)floorf(Z) * NY + (int)floorf(Y)) * NX + (int)floorf(X);
#pragma unroll
                for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 2; ++dx) {
                            const float4 e = inter[(size_t)idx + dz * NXY + dy * NX + dx];
                            m[dz][dy][dx] = e.x;
                            q[dz][dy][dx] = make_float3(e.y, e.z, e.w);
                        }
            };
            // two samples per trip: the 16 corner loads of both are in flight
            // before either sample's arithmetic waits for them
            int k = klo;
            for (; k < khi; k += 2) {
                float X0, Y0, Z0, X1, Y1, Z1;
                position(k, X0, Y0, Z0);
                position(k + 1, X1, Y1, Z1);
                float m0[2][2][2], m1[2][2][2];
                float3 q0[2][2][2], q1[2][2][2];
                gather(X0, Y0, Z0, m0, q0);
                gather(X1, Y1, Z1, m1, q1);
                accumulate(X0, Y0, Z0, m0, q0);
                accumulate(X1, Y1, Z1, m1, q1);
            }
            if (k == khi) {
                float X0, Y0, Z0;
                position(k, X0, Y0, Z0);
                float m0[2][2][2];
                float3 q0[2][2][2];
                gather(X0, Y0, Z0, m0, q0);
                accumulate(X0, Y0, Z0, m0, q0);
            }
        } else {
            for (int k = klo; k <= khi; ++k) {
                float X, Y, Z;
                position(k, X, Y, Z);
                float3 q[2][2][2];
                float m[2][2][2];
                corners_at(mu, s.nx, s.ny, s.nz, (int)floorf(X), (int)floorf(Y), (int)floorf(Z), m, q);
                accumulate(X, Y, Z, m, q);
            }
        }
    }
    constexpr int NC = FUSED ? (HESS ? kRdChannelsGN : kRdChannels + 1) : kRdChannels;
    float acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0f;
    float w = gpix;
    if (FUSED && inside) {
        const float l = lsum * step;
        proj_out[pix] = l;
        const float res = l - gpix;
        w = 2.0f * res;
        acc[kRdChannels] = res * res;  // SSD of this ray
    }
    if (active) {
        // the staged G is twice the gradient field: its 1/2 enters here
        const float hstep = 0.5f * step;
        const float ws = w * hstep;
        acc[0] = G.Bx * ws; acc[1] = G.By * ws; acc[2] = G.Bz * ws;
        acc[3] = G.Txy * ws; acc[4] = G.Txz * ws; acc[5] = G.Tyx * ws;
        acc[6] = G.Tyz * ws; acc[7] = G.Tzx * ws; acc[8] = G.Tzy * ws;
        if (HESS) {
            // This ray's Jacobian dl/dtheta: the finalize map (dL/dt = -R b,
            // dL/dgamma_a = -omega_a . R tau) applied to its own step-scaled
            // sums; then the 21 products of 2 J J^T (Gauss-Newton matrix of
            // the SSD), accumulated in channels kRdChannels + 1 ...
            const float hx = (float)s.vx, hy = (float)s.vy, hz = (float)s.vz;
            const float b3[3] = {G.Bx * hstep / hx, G.By * hstep / hy, G.Bz * hstep / hz};
            const float t3[3] = {(hy / hz * G.Tyz - hz / hy * G.Tzy) * hstep,
                                 (hz / hx * G.Tzx - hx / hz * G.Txz) * hstep,
                                 (hx / hy * G.Txy - hy / hx * G.Tyx) * hstep};
            float J[6];
#pragma unroll
            for (int r3 = 0; r3 < 3; ++r3)
                J[r3] = -((float)g.R[3 * r3] * b3[0] + (float)g.R[3 * r3 + 1] * b3[1] +
                          (float)g.R[3 * r3 + 2] * b3[2]);
            float Rt[3];
#pragma unroll
            for (int r3 = 0; r3 < 3; ++r3)
                Rt[r3] = (float)g.R[3 * r3] * t3[0] + (float)g.R[3 * r3 + 1] * t3[1] +
                         (float)g.R[3 * r3 + 2] * t3[2];
#pragma unroll
            for (int a3 = 0; a3 < 3; ++a3)
                J[3 + a3] = -((float)g.omega[3 * a3] * Rt[0] + (float)g.omega[3 * a3 + 1] * Rt[1] +
                              (float)g.omega[3 * a3 + 2] * Rt[2]);
            int o = kRdChannels + 1;
#pragma unroll
            for (int i6 = 0; i6 < 6; ++i6)
#pragma unroll
                for (int j6 = i6; j6 < 6; ++j6) acc[o++] = 2.0f * J[i6] * J[j6];
        }
    }
    block_reduce_store<NC>(acc, lds, partials + ((size_t)v * tiles + tile) * NC);
}

template <int TW, int MCH, int CAP>
__global__ __launch_bounds__(kRdThreads) void rd_fwd_kernel(GeoScalars s,
                                                            const ViewGeo* __restrict__ views,
                                                            const float* __restrict__ mu,
                                                            float* __restrict__ proj)
{
    __shared__ float lds[CAP];
    __shared__ TileShared sh;
    rd_fwd_tile<TW, MCH, CAP>(s, views, mu, proj, blockIdx.y, blockIdx.x, lds, sh);
}

template <int TW, int MCH, int CAP>
__global__ __launch_bounds__(kRdThreads) void rd_grad_kernel(GeoScalars s,
                                                             const ViewGeo* __restrict__ views,
                                                             const float* __restrict__ mu,
                                                             const float4* __restrict__ inter,
                                                             const float* __restrict__ grad_proj,
                                                             float* __restrict__ partials)
{
    __shared__ __attribute__((aligned(16))) float lds[4 * CAP];
    __shared__ TileShared sh;
    rd_grad_tile<TW, MCH, CAP, false>(s, views, mu, inter, grad_proj, nullptr, partials,
                                      blockIdx.y, blockIdx.x, gridDim.x, lds, sh);
}

// Forward projection, SSD loss and its pose gradient in one march (HESS:
// also the per-view Gauss-Newton matrix of the SSD).
// Both fused kernels are held to 128 VGPRs (four wavefronts per SIMD), which
// the 40 KB LDS classes need for four blocks per compute unit.
template <int TW, int MCH, int CAP, bool HESS>
__global__ __launch_bounds__(kRdThreads, 4) void rd_fused_kernel(GeoScalars s,
                                                              const ViewGeo* __restrict__ views,
                                                              const float* __restrict__ mu,
                                                              const float4* __restrict__ inter,
                                                              const float* __restrict__ target,
                                                              float* __restrict__ proj,
                                                              float* __restrict__ partials)
{
    __shared__ __attribute__((aligned(16))) float lds[4 * CAP];
    __shared__ TileShared sh;
    rd_grad_tile<TW, MCH, CAP, true, HESS>(s, views, mu, inter, target, proj, partials,
                                           blockIdx.y, blockIdx.x, gridDim.x, lds, sh);
}

// Uneven batch: one launch covers every (problem, view, tile) of up to
// kRdMaxBatch problems; the descriptors travel as kernel arguments, so the
// launch needs no device-side table and can be captured in a graph.  Block
// b belongs to the last problem whose first block is <= b.
__device__ inline int batch_problem(const RdBatch& bt)
{
    int p = 0;
    for (int q = 1; q < bt.n; ++q)
        if ((int)blockIdx.x >= bt.it[q].first) p = q;
    return p;
}

template <int TW, int MCH, int CAP>
__global__ __launch_bounds__(kRdThreads) void rd_fwd_batch_kernel(RdBatch bt)
{
    __shared__ float lds[CAP];
    __shared__ TileShared sh;
    const int p = batch_problem(bt);
    const RdBatchItem& it = bt.it[p];
    const int local = (int)blockIdx.x - it.first;
    rd_fwd_tile<TW, MCH, CAP>(it.s, it.views, it.vol, it.out, local / it.tiles,
                              local % it.tiles, lds, sh);
}

template <int TW, int MCH, int CAP>
__global__ __launch_bounds__(kRdThreads, 4) void rd_grad_batch_kernel(RdBatch bt)
{
    __shared__ __attribute__((aligned(16))) float lds[4 * CAP];
    __shared__ TileShared sh;
    const int p = batch_problem(bt);
    const RdBatchItem& it = bt.it[p];
    const int local = (int)blockIdx.x - it.first;
    rd_grad_tile<TW, MCH, CAP, false>(it.s, it.views, it.vol, it.inter, it.gin, nullptr, it.out,
                                      local / it.tiles, local % it.tiles, it.tiles, lds, sh);
}

// Single-pass SSD with the Gauss-Newton matrix over an uneven batch.
template <int TW, int MCH, int CAP>
__global__ __launch_bounds__(kRdThreads, 4) void rd_fused_batch_kernel(RdBatch bt)
{
    __shared__ __attribute__((aligned(16))) float lds[4 * CAP];
    __shared__ TileShared sh;
    const int p = batch_problem(bt);
    const RdBatchItem& it = bt.it[p];
    const int local = (int)blockIdx.x - it.first;
    rd_grad_tile<TW, MCH, CAP, true, true>(it.s, it.views, it.vol, it.inter, it.gin, it.proj,
                                           it.out, local / it.tiles, local % it.tiles, it.tiles,
                                           lds, sh);
}

// Chunk classes (chunk length before adaptation, LDS voxels) per kernel kind:
//   forward : (16, 4096) (32, 4928) (64, 12288)  (middle class: 19.9 KB, eight blocks per CU)
//   gradient: ( 8, 2048) (16, 2520) (32, 4096)
//   fused   : ( 8, 2048) (16, 2520) (32, 4096)  (both: four channels per voxel)
// The fused and gradient kernels' first two classes take at most 40,520
// bytes of LDS per block, which measures as four blocks (16 wavefronts) per
// compute unit (40,904 bytes measures as three); the third runs two.
struct FwdClasses {
    static constexpr int mch[3] = {16, 32, 64}, cap[3] = {4096, 4928, 12288};
};
struct GradClasses {
    static constexpr int mch[3] = {8, 16, 32}, cap[3] = {2048, 2520, 4096};
};
struct FusedClasses {
    static constexpr int mch[3] = {8, 16, 32}, cap[3] = {2048, 2520, 4096};
};

template <int N>
using IntC = std::integral_constant<int, N>;

// Calls f(IntC<tile width>, IntC<chunk class>) for a variant in
// [0, kRdVariants) (anything else: the default, 16x16 tiles and class 1).
template <class F>
static void rd_dispatch(int variant, F&& f)
{
    switch (variant) {
    case 0: f(IntC<16>(), IntC<0>()); break;
    case 2: f(IntC<16>(), IntC<2>()); break;
    case 3: f(IntC<32>(), IntC<0>()); break;
    case 4: f(IntC<32>(), IntC<1>()); break;
    case 5: f(IntC<32>(), IntC<2>()); break;
    case 6: f(IntC<8>(), IntC<0>()); break;
    case 7: f(IntC<8>(), IntC<1>()); break;
    case 8: f(IntC<8>(), IntC<2>()); break;
    default: f(IntC<16>(), IntC<1>()); break;
    }
}

void launch_rd_fwd(const GeoScalars& s, int V, const ViewGeo* views, const float* mu,
                   float* proj, int variant, hipStream_t st)
{
    const dim3 grid(rd_tiles(s, rd_variant_shape(variant)), V);
    prof_begin(DP_K_RD_FWD, st);
    rd_dispatch(variant, [&](auto tw, auto cl) {
        constexpr int c = decltype(cl)::value;
        rd_fwd_kernel<decltype(tw)::value, FwdClasses::mch[c], FwdClasses::cap[c]>
            <<<grid, kRdThreads, 0, st>>>(s, views, mu, proj);
    });
    prof_end(DP_K_RD_FWD, st);
}

void launch_rd_grad(const GeoScalars& s, int V, const ViewGeo* views, const float* mu,
                    const float4* inter, const float* grad_proj, float* partials, int variant,
                    hipStream_t st)
{
    const dim3 grid(rd_tiles(s, rd_variant_shape(variant)), V);
    prof_begin(DP_K_RD_GRAD, st);
    rd_dispatch(variant, [&](auto tw, auto cl) {
        constexpr int c = decltype(cl)::value;
        rd_grad_kernel<decltype(tw)::value, GradClasses::mch[c], GradClasses::cap[c]>
            <<<grid, kRdThreads, 0, st>>>(s, views, mu, inter, grad_proj, partials);
    });
    prof_end(DP_K_RD_GRAD, st);
}

void launch_rd_fused(const GeoScalars& s, int V, const ViewGeo* views, const float* mu,
                     const float4* inter, const float* target, float* proj, float* partials,
                     bool hess, int variant, hipStream_t st)
{
    const dim3 grid(rd_tiles(s, rd_variant_shape(variant)), V);
    prof_begin(DP_K_RD_FUSED, st);
    rd_dispatch(variant, [&](auto tw, auto cl) {
        constexpr int t = decltype(tw)::value, c = decltype(cl)::value;
        constexpr int m = FusedClasses::mch[c], cap = FusedClasses::cap[c];
        if (hess)
            rd_fused_kernel<t, m, cap, true><<<grid, kRdThreads, 0, st>>>(s, views, mu, inter,
                                                                         target, proj, partials);
        else
            rd_fused_kernel<t, m, cap, false><<<grid, kRdThreads, 0, st>>>(s, views, mu, inter,
                                                                          target, proj, partials);
    });
    prof_end(DP_K_RD_FUSED, st);
}

void launch_rd_fwd_batch(const RdBatch& bt, int blocks, int variant, hipStream_t st)
{
    prof_begin(DP_K_RD_FWD, st);
    rd_dispatch(variant, [&](auto tw, auto cl) {
        constexpr int c = decltype(cl)::value;
        rd_fwd_batch_kernel<decltype(tw)::value, FwdClasses::mch[c], FwdClasses::cap[c]>
            <<<blocks, kRdThreads, 0, st>>>(bt);
    });
    prof_end(DP_K_RD_FWD, st);
}

void launch_rd_fused_batch(const RdBatch& bt, int blocks, int variant, hipStream_t st)
{
    prof_begin(DP_K_RD_FUSED, st);
    rd_dispatch(variant, [&](auto tw, auto cl) {
        constexpr int c = decltype(cl)::value;
        rd_fused_batch_kernel<decltype(tw)::value, FusedClasses::mch[c], FusedClasses::cap[c]>
            <<<blocks, kRdThreads, 0, st>>>(bt);
    });
    prof_end(DP_K_RD_FUSED, st);
}

void launch_rd_grad_batch(const RdBatch& bt, int blocks, int variant, hipStream_t st)
{
    prof_begin(DP_K_RD_GRAD, st);
    rd_dispatch(variant, [&](auto tw, auto cl) {
        constexpr int c = decltype(cl)::value;
        rd_grad_batch_kernel<decltype(tw)::value, GradClasses::mch[c], GradClasses::cap[c]>
            <<<blocks, kRdThreads, 0, st>>>(bt);
    });
    prof_end(DP_K_RD_GRAD, st);
}

}  // namespace dp
