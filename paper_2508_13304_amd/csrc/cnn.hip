// Learned pose proposal: the layers of a small strided CNN on BF16 matrix
// cores (MFMA) with FP32 accumulation.  The network regresses a 6-DoF pose
// offset from a pair of DRRs rendered by the forward projector; its output
// initialises the analytic-gradient registration.
//
// Layout: activations are NHWC (row m = (n, y, x), column = channel), so a
// 3x3 strided convolution is
//   col  = im2col(x)            [M = N Ho Wo][K = 9 Ci], K index (ky, kx, ci)
//   z    = col . W^T            W [Co][K]                  (GEMM, MFMA)
//   y    = relu(z + b)          fused epilogue, BF16 out
// and its backward is
//   dz   = dy * (y > 0)
//   dW   = dz^T . col           [Co][K]                    (GEMM, MFMA)
//   db   = column sums of dz
//   dcol = dz . W               [M][K]                     (GEMM, MFMA)
//   dx   = col2im(dcol)         gather of the overlapping windows.
//
// GEMM: C[M][N] (FP32) = op(A) op(B) (+ C if accumulate), A/B BF16.  A block
// computes a 64x64 tile with 4 wavefronts (32x32 each = 2x2 MFMA 16x16x32
// tiles); K advances by 32 through LDS.  Operand lane layout of
// v_mfma_f32_16x16x32_bf16: lane l supplies row (l % 16) of A and column
// (l % 16) of B, each with the 8 consecutive k = 8 (l / 16) .. +7; it receives
// D rows 4 (l / 16) .. +3 of column (l % 16).
#include <algorithm>

#include "dp_internal.h"

namespace dp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kGT = 64;   // block tile (M and N)
constexpr int kGK = 32;   // K step
constexpr int kGPad = 8;  // k-major tile: row padding (bf16) against bank conflicts
// row-major tile: pitch 80 bf16 = 40 dwords, so the four k rows one 16-lane
// group of a transpose read touches start 8 banks apart
constexpr int kTPad = 16;
constexpr int kSK = kGK + kGPad;  // pitch of a k-major tile S[row][k]
constexpr int kST = kGT + kTPad;  // pitch of a row-major tile T[k][row]
constexpr int kTileElems = kGT * kSK > kGK * kST ? kGT * kSK : kGK * kST;

__device__ inline __bf16 to_bf16(float x) { return (__bf16)x; }

// Stage a 64 x 32 (rows x k) tile of one operand into LDS.
// KC: the operand is stored k-contiguous (element (r, k) at P[r * ld + k])
// and lands in S[row][k] (pitch kSK); else it is row-contiguous (at
// P[k * ld + r]) and keeps that layout, T[k][row] (pitch kST): the
// transpose happens when the fragments are read.  VEC: ld is a multiple of 8
// and P 16-byte aligned, so each thread moves 8 contiguous elements with one
// 16-byte load and one 16-byte store (ragged edges fall back to guarded
// element loads).
template <bool KC, bool VEC>
__device__ inline void stage_tile(const __bf16* __restrict__ P, int ld, int rows, int row0, int k0,
                                  int kend, __bf16* S, int tid)
{
    if (VEC) {
        if (KC) {
            const int r = tid >> 2, c = (tid & 3) * 8, row = row0 + r, k = k0 + c;
            if (row < rows && k + 8 <= kend) {
                *(uint4*)&S[r * kSK + c] = *(const uint4*)(P + (size_t)row * ld + k);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    S[r * kSK + c + j] =
                        (row < rows && k + j < kend) ? P[(size_t)row * ld + k + j] : to_bf16(0.f);
            }
        } else {
            const int kk = tid >> 3, c = (tid & 7) * 8, k = k0 + kk, row = row0 + c;
            if (k < kend && row + 8 <= rows) {
                *(uint4*)&S[kk * kST + c] = *(const uint4*)(P + (size_t)k * ld + row);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    S[kk * kST + c + j] =
                        (k < kend && row + j < rows) ? P[(size_t)k * ld + row + j] : to_bf16(0.f);
            }
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int idx = tid + e * 256;  // 0 .. 2047
        int r, c;
        if (KC) { r = idx >> 5; c = idx & 31; }  // coalesced along k
        else    { r = idx & 63; c = idx >> 6; }  // coalesced along rows
        const int row = row0 + r, k = k0 + c;
        const __bf16 v = (row < rows && k < kend)
                             ? (KC ? P[(size_t)row * ld + k] : P[(size_t)k * ld + row])
                             : to_bf16(0.f);
        S[KC ? r * kSK + c : c * kST + r] = v;
    }
}

typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

// MFMA operand fragment of rows rb .. rb + 15: lane l gets row rb + (l % 16),
// k = 8 (l / 16) .. + 7.  From a k-major tile that is one 16-byte read.
// From a row-major tile it is two transpose reads (ds_read_b64_tr_b16):
// within each 16-lane group, the lane i' = 4 j + q addresses the four rows
// 4 q .. 4 q + 3 at one k (8 bytes) and lane i receives, as element j, the
// element i % 4 of lane 4 j + i / 4's four; so lane i gets row i at the four
// k the group's lanes addressed.
template <bool KC>
__device__ inline bf16x8 load_frag(const __bf16* S, int rb, int lane)
{
    if constexpr (KC) {
        return *(const bf16x8*)&S[(rb + (lane & 15)) * kSK + (lane >> 4) * 8];
    } else {
        const int i = lane & 15, k = (lane >> 4) * 8 + (i >> 2);
        typedef __attribute__((address_space(3))) i16x4 lds_i16x4;
        const __bf16* p = S + k * kST + rb + 4 * (i & 3);
        const i16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4*)p);
        const i16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4*)(p + 4 * kST));
        const i16x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        return __builtin_bit_cast(bf16x8, v);
    }
}

// Exact unsigned division by a divisor fixed at launch (multiply-high and
// shift; Granlund and Montgomery's method with a 33-bit magic number split
// into a 32-bit multiplier and an add-and-halve step).  Valid for every
// 32-bit dividend.
struct FastDiv {
    unsigned d, mul, sh;
    FastDiv() = default;
    explicit FastDiv(unsigned div) : d(div), mul(0), sh(0)
    {
        while ((1ull << sh) < div) ++sh;  // sh = ceil(log2 d)
        if (sh > 0) mul = (unsigned)((((1ull << sh) - div) << 32) / div + 1);
    }
    __device__ unsigned div(unsigned n) const
    {
        if (sh == 0) return n;
        const unsigned t = __umulhi(n, mul);
        return (t + ((n - t) >> 1)) >> (sh - 1);
    }
};

// ---------------------------------------------------------------------------
// Operand sources.  A source stages the 64 x 32 (rows x k) tile of its
// operand at (row0, k0) into LDS, zero outside [0, rows) x [k0, kend): S[row][k]
// if KC, else T[k][row].  init() computes what a thread can keep over the
// K loop.
// ---------------------------------------------------------------------------

// A dense BF16 matrix (k-contiguous if KC).
template <bool KC_, bool VEC>
struct DenseSrc {
    static constexpr bool KC = KC_;
    const __bf16* P;
    int ld, rows;
    struct St {};
    __device__ St init(int, int) const { return {}; }
    __device__ void stage(const St&, __bf16* S, int row0, int k0, int kend, int tid) const
    {
        stage_tile<KC, VEC>(P, ld, rows, row0, k0, kend, S, tid);
    }
};

// 3x3 convolution geometry (padding 1, stride s) on NHWC BF16 input with C
// channels, C a multiple of 8: output pixel m = (n, yo, xo), column
// k = (3 ky + kx) C + ci of the implicit im2col matrix; column 9 C is the
// ones column if `ones`, further columns are zero.
struct ConvGeo {
    int H, W, C, s, Ho, Wo, M;  // M = N Ho Wo output pixels
    int ones;
    FastDiv hw, w, c;            // by Ho Wo, Wo, C
};

// 8 consecutive columns k .. k + 7 (k a multiple of 8) of im2col row m.
__device__ inline uint4 im2col8(const __bf16* __restrict__ x, const ConvGeo& g, int n, int yo,
                                int xo, int k)
{
    const int K9 = 9 * g.C;
    if (k >= K9) {
        uint4 z = make_uint4(0u, 0u, 0u, 0u);
        if (g.ones && k == K9) z.x = 0x3F80u;  // BF16 1.0 in the low half
        return z;
    }
    const unsigned t = g.c.div((unsigned)k), ci = (unsigned)k - t * (unsigned)g.C;
    const int ky = (int)t / 3, kx = (int)t - 3 * ky;
    const int y = yo * g.s + ky - 1, xx = xo * g.s + kx - 1;
    if ((unsigned)y >= (unsigned)g.H || (unsigned)xx >= (unsigned)g.W)
        return make_uint4(0u, 0u, 0u, 0u);
    return *(const uint4*)(x + ((size_t)((n * g.H + y) * g.W + xx)) * g.C + ci);
}

// The im2col matrix of the input x as the GEMM's A (rows = output pixels,
// KC): each thread keeps its row's pixel over the K loop.
struct Im2colA {
    static constexpr bool KC = true;
    const __bf16* x;
    ConvGeo g;
    struct St { int n, yo, xo; bool ok; };
    __device__ St init(int row0, int tid) const
    {
        const int m = row0 + (tid >> 2);
        St st;
        st.ok = m < g.M;
        const unsigned n = g.hw.div((unsigned)m), r = (unsigned)m - n * (unsigned)(g.Ho * g.Wo);
        st.n = (int)n;
        st.yo = (int)g.w.div(r);
        st.xo = (int)r - st.yo * g.Wo;
        return st;
    }
    __device__ void stage(const St& st, __bf16* S, int, int k0, int kend, int tid) const
    {
        const int r = tid >> 2, c = (tid & 3) * 8, k = k0 + c;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (st.ok && k < kend) v = im2col8(x, g, st.n, st.yo, st.xo, k);  // kend % 8 == 0
        *(uint4*)&S[r * kSK + c] = v;
    }
};

// The im2col matrix as the B of the weight gradient dW = dz^T . col: rows =
// im2col columns (the GEMM's N), k = output pixels (row-major tile T[k][row]).
struct Im2colB {
    static constexpr bool KC = false;
    const __bf16* x;
    ConvGeo g;
    int ncols;  // columns of the product (row length of dW)
    struct St {};
    __device__ St init(int, int) const { return {}; }
    __device__ void stage(const St&, __bf16* S, int row0, int k0, int kend, int tid) const
    {
        const int kk = tid >> 3, c = (tid & 7) * 8, m = k0 + kk, col = row0 + c;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (m < kend && col < ncols) {  // ncols % 8 == 0
            const unsigned n = g.hw.div((unsigned)m), r = (unsigned)m - n * (unsigned)(g.Ho * g.Wo);
            const int yo = (int)g.w.div(r), xo = (int)r - yo * g.Wo;
            v = im2col8(x, g, (int)n, yo, xo, col);
        }
        *(uint4*)&S[kk * kST + c] = v;
    }
};

// Input gradient of a 3x3 convolution, one parity class (py, px) of input
// pixels y = s y' + py, x = s x' + px at a time: such a pixel receives tap
// (ky, kx) exactly when s divides py + 1 - ky and px + 1 - kx, from output
// pixel (y' + (py + 1 - ky) / s, x' + (px + 1 - kx) / s).  So the class is
// the product dx[m'][ci] = sum_{(t, co)} dz[pixel(m', t)][co] W[co][tap t][ci]
// over its taps t, with no overlap between classes (no col2im).
struct DgradClass {
    int H, W, Ci, Co, s, Ho, Wo;
    int py, px, Hc, Wc, M;      // class pixels: N Hc Wc
    int nky, nkx;               // taps of the class
    int ky[3], kx[3], dy[3], dx[3];
    FastDiv hw, w, co, nkxd;    // by Hc Wc, Wc, Co, nkx
};

struct DgradA {
    static constexpr bool KC = true;
    const __bf16* dz;  // [N][Ho][Wo][Co]
    DgradClass c;
    struct St { int n, yc, xc; bool ok; };
    __device__ St init(int row0, int tid) const
    {
        const int m = row0 + (tid >> 2);
        St st;
        st.ok = m < c.M;
        const unsigned n = c.hw.div((unsigned)m), r = (unsigned)m - n * (unsigned)(c.Hc * c.Wc);
        st.n = (int)n;
        st.yc = (int)c.w.div(r);
        st.xc = (int)r - st.yc * c.Wc;
        return st;
    }
    __device__ void stage(const St& st, __bf16* S, int, int k0, int kend, int tid) const
    {
        const int r = tid >> 2, q = (tid & 3) * 8, k = k0 + q;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (st.ok && k < kend) {
            const unsigned t = c.co.div((unsigned)k), co = (unsigned)k - t * (unsigned)c.Co;
            const unsigned ty = c.nkxd.div(t), tx = t - ty * (unsigned)c.nkx;
            const int yo = st.yc + c.dy[ty], xo = st.xc + c.dx[tx];
            if ((unsigned)yo < (unsigned)c.Ho && (unsigned)xo < (unsigned)c.Wo)
                v = *(const uint4*)(dz + ((size_t)((st.n * c.Ho + yo) * c.Wo + xo)) * c.Co + co);
        }
        *(uint4*)&S[r * kSK + q] = v;
    }
};

// The weights as the class's B: element (k = (t, co), ci) = W[co][tap t][ci]
// of the [Co][ldw] weight rows (row-major tile T[k][ci]).
struct DgradB {
    static constexpr bool KC = false;
    const __bf16* w;
    int ldw;
    DgradClass c;
    struct St {};
    __device__ St init(int, int) const { return {}; }
    __device__ void stage(const St&, __bf16* S, int row0, int k0, int kend, int tid) const
    {
        const int kk = tid >> 3, q = (tid & 7) * 8, k = k0 + kk, ci = row0 + q;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (k < kend && ci < c.Ci) {  // Ci % 8 == 0
            const unsigned t = c.co.div((unsigned)k), co = (unsigned)k - t * (unsigned)c.Co;
            const unsigned ty = c.nkxd.div(t), tx = t - ty * (unsigned)c.nkx;
            const int tap = 3 * c.ky[ty] + c.kx[tx];
            v = *(const uint4*)(w + (size_t)co * ldw + tap * c.Ci + ci);
        }
        *(uint4*)&S[kk * kST + q] = v;
    }
};

// ---------------------------------------------------------------------------
// Epilogues: store4(m, n, v, N) receives v[q] = C[m][n + q] for the four
// consecutive columns n .. n + 3 (n a multiple of 4, n < N) a lane holds.
// ---------------------------------------------------------------------------

// C (+ C if accumulating), FP32; v4: rows 16-byte aligned (one vector store).
struct EpF32 {
    float* C;
    int ldc, accumulate, v4;
    __device__ void store4(int m, int n, const f32x4& v, int N) const
    {
        float* c = C + (size_t)m * ldc + n;
        if (v4 && n + 3 < N) {
            float4 o = make_float4(v[0], v[1], v[2], v[3]);
            if (accumulate) {
                const float4 a = *(const float4*)c;
                o.x += a.x; o.y += a.y; o.z += a.z; o.w += a.w;
            }
            *(float4*)c = o;
            return;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (n + q < N) c[q] = accumulate ? c[q] + v[q] : v[q];
    }
};

// This block's split-K partial tile into the workspace [splits][M][N].
struct EpPartial {
    float* ws;
    int M, N;
    __device__ void store4(int m, int n, const f32x4& v, int) const
    {
        float* c = ws + ((size_t)blockIdx.z * M + m) * N + n;
        if ((N & 3) == 0) {
            *(float4*)c = make_float4(v[0], v[1], v[2], v[3]);
            return;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (n + q < N) c[q] = v[q];
    }
};

__device__ inline void store_bf16x4(__bf16* p, const float (&y)[4], bool vec, int count)
{
    if (vec && count == 4) {
        union { uint2 u; __bf16 h[4]; } o;
#pragma unroll
        for (int q = 0; q < 4; ++q) o.h[q] = to_bf16(y[q]);
        *(uint2*)p = o.u;
        return;
    }
    for (int q = 0; q < count; ++q) p[q] = to_bf16(y[q]);
}

// act(C + bias) to BF16 (the forward convolution's epilogue); v4: rows of Y
// 8-byte aligned.
struct EpBiasAct {
    const float* bias;  // bias of column n at bias[n * bias_stride]
    int bias_stride, relu;
    __bf16* Y;
    int ldy, v4;
    __device__ void store4(int m, int n, const f32x4& v, int N) const
    {
        const int cnt = min(4, N - n);
        float y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            y[q] = q < cnt ? v[q] + bias[(size_t)(n + q) * bias_stride] : 0.f;
            if (relu) y[q] = fmaxf(y[q], 0.f);
        }
        store_bf16x4(Y + (size_t)m * ldy + n, y, v4 != 0, cnt);
    }
};

// Input gradient of one parity class, with the ReLU backward of the layer
// below applied (dz_below = dx where y_below > 0) and written as BF16 at the
// class pixel's place in [N][H][W][Ci] (Ci a multiple of 8: 8-byte groups).
struct EpDgradAct {
    DgradClass c;
    const __bf16* y;  // activation of the layer below (NULL: no activation)
    int relu;
    __bf16* out;
    __device__ void store4(int m, int n, const f32x4& v, int) const
    {
        const unsigned b = c.hw.div((unsigned)m), r = (unsigned)m - b * (unsigned)(c.Hc * c.Wc);
        const int yc = (int)c.w.div(r), xc = (int)r - yc * c.Wc;
        const size_t p = ((size_t)((b * c.H + c.s * yc + c.py) * c.W + c.s * xc + c.px)) * c.Ci + n;
        float o[4] = {v[0], v[1], v[2], v[3]};
        if (relu) {
            union { uint2 u; __bf16 h[4]; } a;
            a.u = *(const uint2*)(y + p);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (!((float)a.h[q] > 0.f)) o[q] = 0.f;
        }
        store_bf16x4(out + p, o, true, 4);
    }
};

// C[M][N] = A B over k: 64 x 64 block tiles, 4 wavefronts of 32 x 32 (2 x 2
// MFMA 16x16x32 tiles each), K advancing by 32 through LDS.  With several
// z blocks (split-K) block z covers its own contiguous k range.
template <class AS, class BS, class EP>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, AS as, BS bs, EP ep)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[kTileElems];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[kTileElems];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * kGT, n0 = blockIdx.y * kGT;
    const int ksplit = (K + (int)gridDim.z - 1) / (int)gridDim.z;
    const int kbeg = (int)blockIdx.z * ((ksplit + kGK - 1) / kGK * kGK);
    const int kend = min(K, kbeg + (ksplit + kGK - 1) / kGK * kGK);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const auto sa = as.init(m0, tid);
    const auto sb = bs.init(n0, tid);
    for (int k0 = kbeg; k0 < kend; k0 += kGK) {
        // (Prefetching the next step's tiles into registers during the
        // products measured slower: a step's products are too short to hide
        // the loads.)
        as.stage(sa, As, m0, k0, kend, tid);
        bs.stage(sb, Bs, n0, k0, kend, tid);
        __syncthreads();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = load_frag<AS::KC>(As, wm + i * 16, lane);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = load_frag<BS::KC>(Bs, wn + j * 16, lane);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                // B's fragment as the instruction's first operand: the
                // result is the transposed tile, so a lane holds four
                // consecutive columns n of one row m (vector stores)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a[i], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int m = m0 + wm + i * 16 + (lane & 15);
            const int n = n0 + wn + j * 16 + (lane >> 4) * 4;
            if (m < M && n < N) ep.store4(m, n, acc[i][j], N);
        }
}

// C (+)= the sum of the split-K partial tiles, in split order (the result
// does not depend on which block finished first).
__global__ __launch_bounds__(256) void splitk_reduce_kernel(int M, int N, int S,
                                                            const float* __restrict__ ws,
                                                            float* __restrict__ C, int ldc,
                                                            int accumulate)
{
    const size_t total = (size_t)M * N;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        for (int z = 0; z < S; ++z) v += ws[(size_t)z * total + i];
        float* c = C + (i / N) * ldc + i % N;
        *c = accumulate ? *c + v : v;
    }
}

// The same sum for many splits: a block covers 16 consecutive outputs with
// 16 threads each; thread g sums its contiguous range of splits in order,
// and the 16 range sums are added in range order (fixed order, so still
// independent of block timing).
constexpr int kRedOut = 16, kRedGroups = 16;
__global__ __launch_bounds__(256) void splitk_reduce_grouped_kernel(int M, int N, int S,
                                                                    const float* __restrict__ ws,
                                                                    float* __restrict__ C, int ldc,
                                                                    int accumulate)
{
    __shared__ float part[kRedGroups][kRedOut];
    const size_t total = (size_t)M * N;
    const int o = threadIdx.x % kRedOut, grp = threadIdx.x / kRedOut;
    const size_t i = (size_t)blockIdx.x * kRedOut + o;
    const int per = (S + kRedGroups - 1) / kRedGroups;
    const int z0 = grp * per, z1 = min(S, z0 + per);
    float v = 0.f;
    if (i < total)
        for (int z = z0; z < z1; ++z) v += ws[(size_t)z * total + i];
    part[grp][o] = v;
    __syncthreads();
    if (grp == 0 && i < total) {
        float t = part[0][o];
        for (int q = 1; q < kRedGroups; ++q) t += part[q][o];
        float* c = C + (i / N) * ldc + i % N;
        *c = accumulate ? *c + t : t;
    }
}

// Split-K for few output tiles and a long reduction (the weight gradients):
// about 1024 blocks, each reducing at least 1024 rows.
static int gemm_splits(int M, int N, int K)
{
    const long long tiles = (long long)((M + kGT - 1) / kGT) * ((N + kGT - 1) / kGT);
    if (tiles < 512 && K >= 2048)
        return (int)std::max<long long>(1, std::min<long long>((1024 + tiles - 1) / tiles, K / 1024));
    return 1;
}

size_t gemm_ws_bytes(int M, int N, int K)
{
    const int s = gemm_splits(M, N, K);
    return s > 1 ? (size_t)s * M * N * sizeof(float) : 0;
}

// Runs C (+)= A B with the split-K decision of gemm_splits: the partial
// tiles go to ws and are reduced in split order (one pass if ws is too
// small or NULL).
template <class AS, class BS>
static void run_gemm_f32(int M, int N, int K, const AS& as, const BS& bs, float* C, int ldc,
                         bool accumulate, float* ws, size_t ws_bytes, hipStream_t st)
{
    const int tm = (M + kGT - 1) / kGT, tn = (N + kGT - 1) / kGT;
    int splits = gemm_splits(M, N, K);
    // (partial tiles take 16-byte stores: the workspace must be aligned)
    if (splits > 1 && (!ws || ws_bytes < gemm_ws_bytes(M, N, K) || ((uintptr_t)ws & 15)))
        splits = 1;
    if (splits > 1) {
        gemm_kernel<<<dim3(tm, tn, splits), 256, 0, st>>>(M, N, K, as, bs, EpPartial{ws, M, N});
        const size_t total = (size_t)M * N;
        if (splits >= 2 * kRedGroups) {
            const size_t blocks = (total + kRedOut - 1) / kRedOut;
            splitk_reduce_grouped_kernel<<<(unsigned)blocks, 256, 0, st>>>(M, N, splits, ws, C, ldc,
                                                                          accumulate ? 1 : 0);
        } else {
            const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
            splitk_reduce_kernel<<<blocks, 256, 0, st>>>(M, N, splits, ws, C, ldc,
                                                         accumulate ? 1 : 0);
        }
    } else {
        const int v4 = ldc % 4 == 0 && ((uintptr_t)C & 15) == 0;
        gemm_kernel<<<dim3(tm, tn, 1), 256, 0, st>>>(M, N, K, as, bs,
                                                     EpF32{C, ldc, accumulate ? 1 : 0, v4});
    }
}

static bool gemm_vec(int lda, int ldb, const void* A, const void* B)
{
    return lda % 8 == 0 && ldb % 8 == 0 && ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0;
}

// Dense operands: A stored [M][K] unless ta ([K][M]), B stored [K][N] unless
// tb ([N][K]); VEC when both take 16-byte moves.
template <bool VEC, class F>
static void with_dense(bool ta, bool tb, const __bf16* a, int lda, int M, const __bf16* b, int ldb,
                       int N, F&& f)
{
    if (!ta && !tb) f(DenseSrc<true, VEC>{a, lda, M}, DenseSrc<false, VEC>{b, ldb, N});
    else if (!ta && tb) f(DenseSrc<true, VEC>{a, lda, M}, DenseSrc<true, VEC>{b, ldb, N});
    else if (ta && !tb) f(DenseSrc<false, VEC>{a, lda, M}, DenseSrc<false, VEC>{b, ldb, N});
    else f(DenseSrc<false, VEC>{a, lda, M}, DenseSrc<true, VEC>{b, ldb, N});
}

void launch_gemm_bf16(bool ta, bool tb, int M, int N, int K, const void* A, int lda, const void* B,
                      int ldb, float* C, int ldc, bool accumulate, float* ws, size_t ws_bytes,
                      hipStream_t st)
{
    const __bf16* a = (const __bf16*)A;
    const __bf16* b = (const __bf16*)B;
    auto go = [&](const auto& as, const auto& bs) {
        run_gemm_f32(M, N, K, as, bs, C, ldc, accumulate, ws, ws_bytes, st);
    };
    if (gemm_vec(lda, ldb, A, B)) with_dense<true>(ta, tb, a, lda, M, b, ldb, N, go);
    else with_dense<false>(ta, tb, a, lda, M, b, ldb, N, go);
}

void launch_gemm_bias_act(int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                          const float* bias, int bias_stride, bool relu, void* Y, int ldy,
                          hipStream_t st)
{
    const dim3 grid((M + kGT - 1) / kGT, (N + kGT - 1) / kGT, 1);
    const EpBiasAct ep{bias, bias_stride, relu ? 1 : 0, (__bf16*)Y, ldy,
                       ldy % 4 == 0 && ((uintptr_t)Y & 7) == 0};
    const __bf16* a = (const __bf16*)A;
    const __bf16* b = (const __bf16*)B;
    if (gemm_vec(lda, ldb, A, B))
        gemm_kernel<<<grid, 256, 0, st>>>(M, N, K, DenseSrc<true, true>{a, lda, M},
                                          DenseSrc<true, true>{b, ldb, N}, ep);
    else
        gemm_kernel<<<grid, 256, 0, st>>>(M, N, K, DenseSrc<true, false>{a, lda, M},
                                          DenseSrc<true, false>{b, ldb, N}, ep);
}

// ---------------------------------------------------------------------------
// Implicit-GEMM 3x3 convolutions (C a multiple of 8; no im2col matrix)
// ---------------------------------------------------------------------------

static ConvGeo conv_geo(int N, int H, int W, int C, int s, bool ones)
{
    ConvGeo g;
    g.H = H; g.W = W; g.C = C; g.s = s;
    g.Ho = (H - 1) / s + 1;
    g.Wo = (W - 1) / s + 1;
    g.M = N * g.Ho * g.Wo;
    g.ones = ones ? 1 : 0;
    g.hw = FastDiv((unsigned)(g.Ho * g.Wo));
    g.w = FastDiv((unsigned)g.Wo);
    g.c = FastDiv((unsigned)C);
    return g;
}

void launch_conv_fwd(int N, int H, int W, int Ci, int Co, int s, const void* x, const void* w,
                     int ldw, const float* bias, int bias_stride, bool relu, void* y, hipStream_t st)
{
    const ConvGeo g = conv_geo(N, H, W, Ci, s, false);
    const dim3 grid((g.M + kGT - 1) / kGT, (Co + kGT - 1) / kGT, 1);
    gemm_kernel<<<grid, 256, 0, st>>>(g.M, Co, 9 * Ci, Im2colA{(const __bf16*)x, g},
                                      DenseSrc<true, true>{(const __bf16*)w, ldw, Co},
                                      EpBiasAct{bias, bias_stride, relu ? 1 : 0, (__bf16*)y, Co,
                                                Co % 4 == 0 && ((uintptr_t)y & 7) == 0});
}

size_t conv_wgrad_ws_bytes(int N, int H, int W, int Ci, int Co, int s, int ldw)
{
    const ConvGeo g = conv_geo(N, H, W, Ci, s, false);
    return gemm_ws_bytes(Co, ldw, g.M);
}

void launch_conv_wgrad(int N, int H, int W, int Ci, int Co, int s, const void* x, const void* dz,
                       int ldw, bool ones, float* dw, float* ws, size_t ws_bytes, hipStream_t st)
{
    const ConvGeo g = conv_geo(N, H, W, Ci, s, ones);
    run_gemm_f32(Co, ldw, g.M, DenseSrc<false, true>{(const __bf16*)dz, Co, Co},
                 Im2colB{(const __bf16*)x, g, ldw}, dw, ldw, false, ws, ws_bytes, st);
}

void launch_conv_dgrad_act(int N, int H, int W, int Ci, int Co, int s, const void* dz,
                           const void* w, int ldw, const void* y, bool relu, void* out,
                           hipStream_t st)
{
    DgradClass c{};
    c.H = H; c.W = W; c.Ci = Ci; c.Co = Co; c.s = s;
    c.Ho = (H - 1) / s + 1;
    c.Wo = (W - 1) / s + 1;
    c.co = FastDiv((unsigned)Co);
    for (int py = 0; py < s && py < H; ++py)
        for (int px = 0; px < s && px < W; ++px) {
            c.py = py; c.px = px;
            c.Hc = (H - py + s - 1) / s;
            c.Wc = (W - px + s - 1) / s;
            c.M = N * c.Hc * c.Wc;
            c.nky = c.nkx = 0;
            for (int k = 0; k < 3; ++k) {
                if ((py + 1 - k) % s == 0) { c.ky[c.nky] = k; c.dy[c.nky++] = (py + 1 - k) / s; }
                if ((px + 1 - k) % s == 0) { c.kx[c.nkx] = k; c.dx[c.nkx++] = (px + 1 - k) / s; }
            }
            c.hw = FastDiv((unsigned)(c.Hc * c.Wc));
            c.w = FastDiv((unsigned)c.Wc);
            c.nkxd = FastDiv((unsigned)c.nkx);
            const int K = c.nky * c.nkx * Co;
            const dim3 grid((c.M + kGT - 1) / kGT, (Ci + kGT - 1) / kGT, 1);
            gemm_kernel<<<grid, 256, 0, st>>>(c.M, Ci, K, DgradA{(const __bf16*)dz, c},
                                              DgradB{(const __bf16*)w, ldw, c},
                                              EpDgradAct{c, (const __bf16*)y, relu ? 1 : 0,
                                                         (__bf16*)out});
        }
}

// im2col of a 3x3 convolution (stride s, padding 1) on NHWC BF16 input:
// col[m][t C + c] = x[n][yo s + ky - 1][xo s + kx - 1][c] (zero outside),
// t = 3 ky + kx.  One thread per (output pixel m, tap t, group of G
// channels); G = 8 copies 16 bytes at a time.  Index math is 32-bit (the
// host checks that every index space fits).
template <int G>
__global__ __launch_bounds__(256) void im2col_kernel(int N, int H, int W, int C, int s, int Ho,
                                                     int Wo, const __bf16* __restrict__ x,
                                                     __bf16* __restrict__ col, int ld)
{
    const unsigned groups = (unsigned)(C / G);
    const unsigned total = (unsigned)N * Ho * Wo * 9u * groups;
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const unsigned g = i % groups, r = i / groups;
        const unsigned t = r % 9u, m = r / 9u;
        const int xo = (int)(m % (unsigned)Wo);
        const unsigned q = m / (unsigned)Wo;
        const int yo = (int)(q % (unsigned)Ho), n = (int)(q / (unsigned)Ho);
        const int ky = (int)t / 3, kx = (int)t - 3 * ky;
        const int yi = yo * s + ky - 1, xi = xo * s + kx - 1;
        __bf16* dst = col + (size_t)m * ld + t * C + g * G;
        const bool in = yi >= 0 && yi < H && xi >= 0 && xi < W;
        const __bf16* src = x + (((size_t)n * H + yi) * W + xi) * C + g * G;
        if constexpr (G == 8) {
            *reinterpret_cast<uint4*>(dst) = in ? *reinterpret_cast<const uint4*>(src) : make_uint4(0, 0, 0, 0);
        } else {
#pragma unroll
            for (int c = 0; c < G; ++c) dst[c] = in ? src[c] : to_bf16(0.f);
        }
    }
}

// Columns [9 C, ld) of each im2col row: 1 in column 9 C when `ones` (so that
// the weight-gradient product dz^T col also yields the bias gradient, the
// column sums of dz), 0 elsewhere.
__global__ __launch_bounds__(256) void col_tail_kernel(unsigned rows, int K9, int ld, int ones,
                                                       __bf16* __restrict__ col)
{
    const unsigned w = (unsigned)(ld - K9), total = rows * w;
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const unsigned m = i / w, c = i - m * w;
        col[(size_t)m * ld + K9 + c] = to_bf16(ones && c == 0 ? 1.f : 0.f);
    }
}

// dx = col2im(dcol): each input element gathers the window entries that read
// it (taps in ky, kx order).  One thread per (n, yi, xi, group of G
// channels); G = 4 moves float4.
// ACT: the result is the gradient of the layer below's BF16 activation y, and
// the kernel applies that layer's ReLU backward and writes the BF16 operand
// dz = dx * (y > 0) instead of FP32 dx.
template <int G, bool ACT>
__global__ __launch_bounds__(256) void col2im_kernel(int N, int H, int W, int C, int s, int Ho,
                                                     int Wo, const float* __restrict__ dcol,
                                                     float* __restrict__ dx,
                                                     const __bf16* __restrict__ y, int relu,
                                                     __bf16* __restrict__ dz)
{
    const unsigned groups = (unsigned)(C / G);
    const unsigned total = (unsigned)N * H * W * groups;
    const int K = 9 * C;
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const unsigned g = i % groups, p = i / groups;
        const int xi = (int)(p % (unsigned)W);
        const unsigned q = p / (unsigned)W;
        const int yi = (int)(q % (unsigned)H), n = (int)(q / (unsigned)H);
        float acc[G];
#pragma unroll
        for (int c = 0; c < G; ++c) acc[c] = 0.f;
        for (int ky = 0; ky < 3; ++ky) {
            const int ty = yi + 1 - ky;  // = yo * s
            if (ty < 0 || ty % s) continue;
            const int yo = ty / s;
            if (yo >= Ho) continue;
            for (int kx = 0; kx < 3; ++kx) {
                const int tx = xi + 1 - kx;
                if (tx < 0 || tx % s) continue;
                const int xo = tx / s;
                if (xo >= Wo) continue;
                const float* src = dcol + ((size_t)((n * Ho + yo) * Wo + xo)) * K + (ky * 3 + kx) * C + g * G;
                if constexpr (G == 4) {
                    const float4 v = *reinterpret_cast<const float4*>(src);
                    acc[0] += v.x; acc[1] += v.y; acc[2] += v.z; acc[3] += v.w;
                } else {
#pragma unroll
                    for (int c = 0; c < G; ++c) acc[c] += src[c];
                }
            }
        }
        if constexpr (ACT) {
            const size_t o = (size_t)p * C + g * G;
            union { uint2 u; __bf16 h[4]; } yv, dv;
            if constexpr (G == 4) {
                yv.u = *reinterpret_cast<const uint2*>(y + o);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    dv.h[c] = to_bf16(relu ? ((float)yv.h[c] > 0.f ? acc[c] : 0.f) : acc[c]);
                *reinterpret_cast<uint2*>(dz + o) = dv.u;
            } else {
#pragma unroll
                for (int c = 0; c < G; ++c)
                    dz[o + c] = to_bf16(relu ? ((float)y[o + c] > 0.f ? acc[c] : 0.f) : acc[c]);
            }
        } else {
            float* dst = dx + (size_t)p * C + g * G;
            if constexpr (G == 4) {
                *reinterpret_cast<float4*>(dst) = make_float4(acc[0], acc[1], acc[2], acc[3]);
            } else {
#pragma unroll
                for (int c = 0; c < G; ++c) dst[c] = acc[c];
            }
        }
    }
}

// y = relu(z + b) -> BF16 (and FP32 copy for the head); z [M][C] FP32.
__global__ __launch_bounds__(256) void bias_relu_kernel(size_t total, int C, const float* __restrict__ z,
                                                        const float* __restrict__ b, int relu,
                                                        __bf16* __restrict__ y)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        float v = z[i] + b[i % C];
        if (relu) v = fmaxf(v, 0.f);
        y[i] = to_bf16(v);
    }
}

// dz = dy * (y > 0) -> BF16 operand for the GEMMs; y is the layer's BF16 output.
__global__ __launch_bounds__(256) void relu_bwd_kernel(size_t total, const float* __restrict__ dy,
                                                       const __bf16* __restrict__ y, int relu,
                                                       __bf16* __restrict__ dz)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const float g = dy[i];
        dz[i] = to_bf16(relu ? ((float)y[i] > 0.f ? g : 0.f) : g);
    }
}

// db[c] = sum over rows of dz (BF16 operand as used by the weight GEMM).
// Grid-stride over rows with consecutive threads on consecutive elements:
// for C < 256 a block covers R = 256 / C rows per pass (thread t: column
// t % C, row offset t / C), for C >= 256 strips of 256 columns.  Each block
// adds its column sums to db with FP32 atomics (db zeroed first), so the
// summation order, and the last bits, vary from run to run.
__global__ __launch_bounds__(256) void colsum_kernel(int M, int C, const __bf16* __restrict__ dz,
                                                     float* __restrict__ db)
{
    __shared__ float red[256];
    const int t = threadIdx.x;
    const bool narrow = C < 256;
    const int R = narrow ? 256 / C : 1;
    for (int c0 = 0; c0 < C; c0 += 256) {
        const int c = narrow ? t % C : c0 + t;
        const int ro = narrow ? t / C : 0;
        const bool act = narrow ? t < R * C : c < C;
        float acc = 0.f;
        if (act)
            for (size_t r = (size_t)blockIdx.x * R + ro; r < (size_t)M; r += (size_t)gridDim.x * R)
                acc += (float)dz[r * C + c];
        if (narrow) {
            red[t] = acc;
            __syncthreads();
            if (t < C) {
                float sum = 0.f;
                for (int k = 0; k < R; ++k) sum += red[k * C + t];
                atomicAdd(db + t, sum);
            }
            __syncthreads();
        } else if (act) {
            atomicAdd(db + c, acc);
        }
    }
}

// One Adam step over a flat parameter buffer (every layer at once): moments
// m, v and the FP32 master p updated in place, and p rounded to BF16 for the
// next products.  c1, c2: the bias corrections 1 - beta^t.
__global__ __launch_bounds__(256) void adam_kernel(size_t n, float* __restrict__ p,
                                                   const float* __restrict__ g, float* __restrict__ m,
                                                   float* __restrict__ v, __bf16* __restrict__ pb,
                                                   float lr, float b1, float b2, float eps, float c1,
                                                   float c2)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
        const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        pb[i] = to_bf16(pi);
    }
}

__global__ __launch_bounds__(256) void fill_zero_kernel(int n, float* __restrict__ p)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

static int grid_for(size_t total)
{
    const size_t b = (total + 255) / 256;
    return (int)(b < 65536 ? (b == 0 ? 1 : b) : 65536);
}

void launch_im2col(int N, int H, int W, int C, int s, int Ho, int Wo, const void* x, void* col,
                   int ld, bool ones, hipStream_t st)
{
    const bool vec = C % 8 == 0 && ld % 8 == 0 && (uintptr_t)x % 16 == 0 && (uintptr_t)col % 16 == 0;
    const size_t total = (size_t)N * Ho * Wo * 9 * (vec ? C / 8 : C);
    if (vec)
        im2col_kernel<8><<<grid_for(total), 256, 0, st>>>(N, H, W, C, s, Ho, Wo, (const __bf16*)x,
                                                          (__bf16*)col, ld);
    else
        im2col_kernel<1><<<grid_for(total), 256, 0, st>>>(N, H, W, C, s, Ho, Wo, (const __bf16*)x,
                                                          (__bf16*)col, ld);
    if (ld > 9 * C) {
        const unsigned rows = (unsigned)N * Ho * Wo;
        col_tail_kernel<<<grid_for((size_t)rows * (ld - 9 * C)), 256, 0, st>>>(rows, 9 * C, ld, ones ? 1 : 0,
                                                                              (__bf16*)col);
    }
}

void launch_col2im(int N, int H, int W, int C, int s, int Ho, int Wo, const float* dcol, float* dx,
                   const void* y, bool relu, void* dz, hipStream_t st)
{
    const bool act = y != nullptr;
    const bool vec = C % 4 == 0 && (uintptr_t)dcol % 16 == 0 &&
                     (act ? ((uintptr_t)y % 8 == 0 && (uintptr_t)dz % 8 == 0) : (uintptr_t)dx % 16 == 0);
    const size_t total = (size_t)N * H * W * (vec ? C / 4 : C);
    const __bf16* yb = (const __bf16*)y;
    __bf16* dzb = (__bf16*)dz;
    const int r = relu ? 1 : 0;
    if (act) {
        if (vec)
            col2im_kernel<4, true><<<grid_for(total), 256, 0, st>>>(N, H, W, C, s, Ho, Wo, dcol, dx, yb, r, dzb);
        else
            col2im_kernel<1, true><<<grid_for(total), 256, 0, st>>>(N, H, W, C, s, Ho, Wo, dcol, dx, yb, r, dzb);
    } else {
        if (vec)
            col2im_kernel<4, false><<<grid_for(total), 256, 0, st>>>(N, H, W, C, s, Ho, Wo, dcol, dx, yb, r, dzb);
        else
            col2im_kernel<1, false><<<grid_for(total), 256, 0, st>>>(N, H, W, C, s, Ho, Wo, dcol, dx, yb, r, dzb);
    }
}

void launch_adam(size_t n, float* p, const float* g, float* m, float* v, void* pb, float lr,
                 float b1, float b2, float eps, float c1, float c2, hipStream_t st)
{
    adam_kernel<<<grid_for(n), 256, 0, st>>>(n, p, g, m, v, (__bf16*)pb, lr, b1, b2, eps, c1, c2);
}

void launch_bias_relu(size_t total, int C, const float* z, const float* b, bool relu, void* y,
                      hipStream_t st)
{
    bias_relu_kernel<<<grid_for(total), 256, 0, st>>>(total, C, z, b, relu ? 1 : 0, (__bf16*)y);
}

void launch_relu_bwd(size_t total, const float* dy, const void* y, bool relu, void* dz,
                     hipStream_t st)
{
    relu_bwd_kernel<<<grid_for(total), 256, 0, st>>>(total, dy, (const __bf16*)y, relu ? 1 : 0,
                                                     (__bf16*)dz);
}

void launch_colsum(int M, int C, const void* dz, float* db, hipStream_t st)
{
    const int R = C < 256 ? 256 / C : 1;
    const int blocks = (int)std::min<long long>(1024, ((long long)M + R - 1) / R);
    fill_zero_kernel<<<(C + 255) / 256, 256, 0, st>>>(C, db);
    colsum_kernel<<<blocks, 256, 0, st>>>(M, C, (const __bf16*)dz, db);
}

}  // namespace dp
