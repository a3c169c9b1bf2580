// Elementwise detector-image preparation passes (HBM-bound, coalesced along u):
//   - per padded detector pixel, the 2x2 bilinear footprint of the
//     zero-extended image as one float4, for the back-projection;
//   - detector gradient field (central differences of l, Sec. II-C) stored
//     as float4 (l, dl/da, dl/db, 0) in pixel-index units, zero outside
//     (footprint projectors), or as the 2x2 bilinear footprints of the three
//     fields (voxel-driven back-projection gradient).
#include "dp_internal.h"

namespace dp {

__device__ inline float pix_at(const float* __restrict__ img, int nu, int nv, int a, int b)
{
    if (a < 0 || b < 0 || a >= nu || b >= nv) return 0.0f;
    return img[(size_t)b * nu + a];
}

// Per padded pixel (A, B), the 2x2 bilinear footprint {(A, B), (A+1, B),
// (A, B+1), (A+1, B+1)} of the zero-extended image as one float4, so that a
// back-projection update gathers one 16-byte vector instead of two rows.
__global__ __launch_bounds__(256) void det_pad_kernel(int nu, int nv, const float* __restrict__ proj,
                                                      float4* __restrict__ projq)
{
    const int NU = nu + 2 * kPadD, NV = nv + 2 * kPadD;
    const int A = blockIdx.x * blockDim.x + threadIdx.x;
    const int B = blockIdx.y, v = blockIdx.z;
    if (A >= NU) return;
    const float* img = proj + (size_t)v * nu * nv;
    const int a = A - kPadD, b = B - kPadD;
    projq[((size_t)v * NV + B) * NU + A] =
        make_float4(pix_at(img, nu, nv, a, b), pix_at(img, nu, nv, a + 1, b),
                    pix_at(img, nu, nv, a, b + 1), pix_at(img, nu, nv, a + 1, b + 1));
}

__global__ __launch_bounds__(256) void det_grad_kernel(int nu, int nv, const float* __restrict__ proj,
                                                       float4* __restrict__ proj4)
{
    const int NU = nu + 2 * kPadD, NV = nv + 2 * kPadD;
    const int A = blockIdx.x * blockDim.x + threadIdx.x;
    const int B = blockIdx.y, v = blockIdx.z;
    if (A >= NU) return;
    const float* img = proj + (size_t)v * nu * nv;
    const int a = A - kPadD, b = B - kPadD;
    float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
    if (a >= 0 && b >= 0 && a < nu && b < nv) {
        o.x = img[(size_t)b * nu + a];
        o.y = 0.5f * (pix_at(img, nu, nv, a + 1, b) - pix_at(img, nu, nv, a - 1, b));
        o.z = 0.5f * (pix_at(img, nu, nv, a, b + 1) - pix_at(img, nu, nv, a, b - 1));
    }
    proj4[((size_t)v * NV + B) * NU + A] = o;
}

// l, dl/da, dl/db at pixel (a, b) of the zero-extended image (derivatives:
// half the central difference on grid pixels, zero elsewhere).
__device__ inline float3 lgrad_at(const float* __restrict__ img, int nu, int nv, int a, int b)
{
    if (a < 0 || b < 0 || a >= nu || b >= nv) return make_float3(0.f, 0.f, 0.f);
    return make_float3(img[(size_t)b * nu + a],
                       0.5f * (pix_at(img, nu, nv, a + 1, b) - pix_at(img, nu, nv, a - 1, b)),
                       0.5f * (pix_at(img, nu, nv, a, b + 1) - pix_at(img, nu, nv, a, b - 1)));
}

// Per padded pixel (A, B), the 2x2 bilinear footprints of l, dl/da and
// dl/db, so that a back-projection gradient update gathers three 16-byte
// vectors, every lane of them used.
__global__ __launch_bounds__(256) void det_tap3_kernel(int nu, int nv, const float* __restrict__ proj,
                                                       DetTap3* __restrict__ det)
{
    const int NU = nu + 2 * kPadD, NV = nv + 2 * kPadD;
    const int A = blockIdx.x * blockDim.x + threadIdx.x;
    const int B = blockIdx.y, v = blockIdx.z;
    if (A >= NU) return;
    const float* img = proj + (size_t)v * nu * nv;
    const int a = A - kPadD, b = B - kPadD;
    const float3 q00 = lgrad_at(img, nu, nv, a, b), q10 = lgrad_at(img, nu, nv, a + 1, b);
    const float3 q01 = lgrad_at(img, nu, nv, a, b + 1), q11 = lgrad_at(img, nu, nv, a + 1, b + 1);
    DetTap3 t;
    t.l = make_float4(q00.x, q10.x, q01.x, q11.x);
    t.a = make_float4(q00.y, q10.y, q01.y, q11.y);
    t.b = make_float4(q00.z, q10.z, q01.z, q11.z);
    det[((size_t)v * NV + B) * NU + A] = t;
}

void launch_det_tap3(const GeoScalars& s, int V, const float* proj, DetTap3* det, hipStream_t st)
{
    const int NU = s.nu + 2 * kPadD;
    dim3 grid((NU + 255) / 256, s.nv + 2 * kPadD, V);
    prof_begin(DP_K_DET_PREP, st);
    det_tap3_kernel<<<grid, 256, 0, st>>>(s.nu, s.nv, proj, det);
    prof_end(DP_K_DET_PREP, st);
}

void launch_det_pad(const GeoScalars& s, int V, const float* proj, float4* projq, hipStream_t st)
{
    const int NU = s.nu + 2 * kPadD;
    dim3 grid((NU + 255) / 256, s.nv + 2 * kPadD, V);
    prof_begin(DP_K_DET_PREP, st);
    det_pad_kernel<<<grid, 256, 0, st>>>(s.nu, s.nv, proj, projq);
    prof_end(DP_K_DET_PREP, st);
}

void launch_det_grad(const GeoScalars& s, int V, const float* proj, float4* proj4, hipStream_t st)
{
    const int NU = s.nu + 2 * kPadD;
    dim3 grid((NU + 255) / 256, s.nv + 2 * kPadD, V);
    prof_begin(DP_K_DET_PREP, st);
    det_grad_kernel<<<grid, 256, 0, st>>>(s.nu, s.nv, proj, proj4);
    prof_end(DP_K_DET_PREP, st);
}

}  // namespace dp
