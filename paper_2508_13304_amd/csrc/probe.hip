// Read probes: the LDS, cache-hierarchy and HBM read bandwidths against
// which the gather-bound ray kernels are rated.  Not part of the projection
// method; the kernels only read a buffer and write one sum per thread.
#include "dp_internal.h"

namespace dp {

namespace {

constexpr uint32_t kProbeThreads = 256;
constexpr uint32_t kProbeUnroll = 8;
constexpr uint32_t kProbeStep = kProbeThreads * kProbeUnroll;  // float4 per block per iteration

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline float sum4(float4 v) { return (v.x + v.y) + (v.z + v.w); }

// shared != 0: every block streams the whole footprint (n_vec float4, a power
// of two, at least kProbeStep) `reps` times, starting at its own offset.
// After the first pass each XCD's L2 holds the footprint; with a footprint far
// above a CU's L1 nearly every load misses L1, so the loads measure the
// L2 -> CU read path.
// shared == 0: block b streams its own contiguous slab of `per` float4 (a
// multiple of kProbeStep) with nontemporal loads, and the blocks then share
// the ragged tail past gridDim.x * per grid-stride; every float4 is read once
// per pass.  With a buffer far above L2 and the last-level cache this is HBM
// streaming.
__global__ __launch_bounds__(kProbeThreads) void read_probe_kernel(const float4* __restrict__ buf,
                                                                   uint32_t n_vec, int reps,
                                                                   int shared,
                                                                   float* __restrict__ out)
{
    float acc[kProbeUnroll] = {};
    const uint32_t t = threadIdx.x;
    if (shared) {
        const uint32_t mask = n_vec - 1;
        // Fibonacci hashing spreads the blocks' starting rows over the footprint,
        // so blocks sharing a CU do not walk the same lines in step.
        const uint32_t start = (blockIdx.x * 2654435761u) & mask & ~(kProbeThreads - 1);
        for (int r = 0; r < reps; ++r) {
            for (uint32_t k = 0; k < n_vec; k += kProbeStep) {
                float4 v[kProbeUnroll];
#pragma unroll
                for (uint32_t u = 0; u < kProbeUnroll; ++u)
                    v[u] = buf[(start + k + u * kProbeThreads + t) & mask];
#pragma unroll
                for (uint32_t u = 0; u < kProbeUnroll; ++u) acc[u] += sum4(v[u]);
            }
        }
    } else {
        const uint32_t per = n_vec / (gridDim.x * kProbeStep) * kProbeStep;
        const f32x4* slab = (const f32x4*)(buf + (size_t)blockIdx.x * per);
        const uint32_t tail0 = gridDim.x * per;  // <= n_vec
        const uint32_t stride = gridDim.x * kProbeThreads;
        for (int r = 0; r < reps; ++r) {
            for (uint32_t k = 0; k < per; k += kProbeStep) {
                f32x4 v[kProbeUnroll];
#pragma unroll
                for (uint32_t u = 0; u < kProbeUnroll; ++u)
                    v[u] = __builtin_nontemporal_load(slab + k + u * kProbeThreads + t);
#pragma unroll
                for (uint32_t u = 0; u < kProbeUnroll; ++u)
                    acc[u] += (v[u].x + v[u].y) + (v[u].z + v[u].w);
            }
            // n_vec + stride < 2^32 (checked by the caller): i cannot wrap
            for (uint32_t i = tail0 + blockIdx.x * kProbeThreads + t; i < n_vec; i += stride)
                acc[0] += sum4(buf[i]);
        }
    }
    float total = 0.f;
#pragma unroll
    for (uint32_t u = 0; u < kProbeUnroll; ++u) total += acc[u];
    out[blockIdx.x * kProbeThreads + t] = total;
}

// LDS read probe: each block fills kLdsProbeVec float4 of LDS, then every
// thread reads 16-byte vectors (consecutive lanes, consecutive vectors: no
// bank conflicts), kProbeUnroll per step, `reps` steps, and writes its sum.
// Bytes read = n_blocks * 256 * reps * kProbeUnroll * 16.
constexpr uint32_t kLdsProbeVec = 2048;  // 32 KiB per block

__global__ __launch_bounds__(kProbeThreads) void lds_probe_kernel(int reps, float* __restrict__ out)
{
    __shared__ float4 lds[kLdsProbeVec];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < kLdsProbeVec; i += kProbeThreads)
        lds[i] = make_float4((float)i, 1.0f, 2.0f, 3.0f);
    __syncthreads();
    float acc[kProbeUnroll] = {};
    uint32_t base = t;
    for (int r = 0; r < reps; ++r) {
        float4 v[kProbeUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kProbeUnroll; ++u)
            v[u] = lds[(base + u * kProbeThreads) & (kLdsProbeVec - 1)];
#pragma unroll
        for (uint32_t u = 0; u < kProbeUnroll; ++u) acc[u] += sum4(v[u]);
        base += 64;  // a new window each step (the loads cannot be hoisted), lanes still consecutive
    }
    float total = 0.f;
#pragma unroll
    for (uint32_t u = 0; u < kProbeUnroll; ++u) total += acc[u];
    out[blockIdx.x * kProbeThreads + t] = total;
}

}  // namespace

void launch_lds_probe(int reps, int n_blocks, float* out, hipStream_t st)
{
    lds_probe_kernel<<<n_blocks, kProbeThreads, 0, st>>>(reps, out);
}

void launch_read_probe(const void* buf, uint32_t n_vec, int reps, bool shared, int n_blocks,
                       float* out, hipStream_t st)
{
    read_probe_kernel<<<n_blocks, kProbeThreads, 0, st>>>((const float4*)buf, n_vec, reps,
                                                          shared ? 1 : 0, out);
}

}  // namespace dp
