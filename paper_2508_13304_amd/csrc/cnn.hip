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

// Output modes of the GEMM kernel: FP32 C (+ C if accumulating); this
// block's split-K partial tile into a workspace slice; or act(C + bias) to
// BF16 (the forward convolution's epilogue).
enum { kOutF32 = 0, kOutPartial = 1, kOutBiasAct = 2 };

struct GemmOut {
    float* C;            // kOutF32: C; kOutPartial: the workspace [splits][M][N]
    int ldc;
    int accumulate;
    const float* bias;   // kOutBiasAct: bias of column n at bias[n * bias_stride]
    int bias_stride;
    int relu;
    __bf16* Y;           // kOutBiasAct: BF16 output, row stride ldy
    int ldy;
};

template <bool TA, bool TB, bool VEC, int OUT>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K,
                                                        const __bf16* __restrict__ A, int lda,
                                                        const __bf16* __restrict__ B, int ldb,
                                                        GemmOut o)
{
    // A is k-major in LDS unless stored transposed (TA), B k-major if TB.
    constexpr bool AK = !TA, BK = TB;
    __shared__ __attribute__((aligned(16))) __bf16 As[kTileElems];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[kTileElems];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * kGT, n0 = blockIdx.y * kGT;
    // split-K: block z covers k in [kbeg, kend) and writes its own partial tile
    const int ksplit = (K + (int)gridDim.z - 1) / (int)gridDim.z;
    const int kbeg = (int)blockIdx.z * ((ksplit + kGK - 1) / kGK * kGK);
    const int kend = min(K, kbeg + (ksplit + kGK - 1) / kGK * kGK);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += kGK) {
        // A stored [M][K] (k-contiguous) unless TA; B stored [N][K] if TB.
        // (Prefetching the next step's tiles into registers during the
        // products measured slower: a step's products are too short to hide
        // the loads.)
        stage_tile<AK, VEC>(A, lda, M, m0, k0, kend, As, tid);
        stage_tile<BK, VEC>(B, ldb, N, n0, k0, kend, Bs, tid);
        __syncthreads();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = load_frag<AK>(As, wm + i * 16, lane);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = load_frag<BK>(Bs, wn + j * 16, lane);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + q;
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (m < M && n < N) {
                    const float v = acc[i][j][q];
                    if constexpr (OUT == kOutPartial) {
                        o.C[((size_t)blockIdx.z * M + m) * N + n] = v;
                    } else if constexpr (OUT == kOutBiasAct) {
                        float y = v + o.bias[(size_t)n * o.bias_stride];
                        if (o.relu) y = fmaxf(y, 0.f);
                        o.Y[(size_t)m * o.ldy + n] = to_bf16(y);
                    } else {
                        float* c = o.C + (size_t)m * o.ldc + n;
                        *c = o.accumulate ? *c + v : v;
                    }
                }
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

template <int OUT>
static void gemm_dispatch(bool ta, bool tb, bool vec, dim3 grid, int M, int N, int K,
                          const __bf16* a, int lda, const __bf16* b, int ldb, const GemmOut& o,
                          hipStream_t st)
{
#define DP_GEMM(TA_, TB_)                                                                          \
    do {                                                                                           \
        if (vec)                                                                                   \
            gemm_bf16_kernel<TA_, TB_, true, OUT><<<grid, 256, 0, st>>>(M, N, K, a, lda, b, ldb, o); \
        else                                                                                       \
            gemm_bf16_kernel<TA_, TB_, false, OUT><<<grid, 256, 0, st>>>(M, N, K, a, lda, b, ldb, o); \
    } while (0)
    if (!ta && !tb) DP_GEMM(false, false);
    else if (!ta && tb) DP_GEMM(false, true);
    else if (ta && !tb) DP_GEMM(true, false);
    else DP_GEMM(true, true);
#undef DP_GEMM
}

static bool gemm_vec(int lda, int ldb, const void* A, const void* B)
{
    return lda % 8 == 0 && ldb % 8 == 0 && ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0;
}

void launch_gemm_bf16(bool ta, bool tb, int M, int N, int K, const void* A, int lda, const void* B,
                      int ldb, float* C, int ldc, bool accumulate, float* ws, size_t ws_bytes,
                      hipStream_t st)
{
    const int tm = (M + kGT - 1) / kGT, tn = (N + kGT - 1) / kGT;
    int splits = gemm_splits(M, N, K);
    if (splits > 1 && (!ws || ws_bytes < gemm_ws_bytes(M, N, K))) splits = 1;  // no workspace: one pass
    const __bf16* a = (const __bf16*)A;
    const __bf16* b = (const __bf16*)B;
    const bool vec = gemm_vec(lda, ldb, A, B);
    GemmOut o{};
    if (splits > 1) {
        o.C = ws;
        gemm_dispatch<kOutPartial>(ta, tb, vec, dim3(tm, tn, splits), M, N, K, a, lda, b, ldb, o, st);
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
        o.C = C;
        o.ldc = ldc;
        o.accumulate = accumulate ? 1 : 0;
        gemm_dispatch<kOutF32>(ta, tb, vec, dim3(tm, tn, 1), M, N, K, a, lda, b, ldb, o, st);
    }
}

void launch_gemm_bias_act(int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                          const float* bias, int bias_stride, bool relu, void* Y, int ldy,
                          hipStream_t st)
{
    const int tm = (M + kGT - 1) / kGT, tn = (N + kGT - 1) / kGT;
    GemmOut o{};
    o.bias = bias;
    o.bias_stride = bias_stride;
    o.relu = relu ? 1 : 0;
    o.Y = (__bf16*)Y;
    o.ldy = ldy;
    gemm_dispatch<kOutBiasAct>(false, true, gemm_vec(lda, ldb, A, B), dim3(tm, tn, 1), M, N, K,
                               (const __bf16*)A, lda, (const __bf16*)B, ldb, o, st);
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
