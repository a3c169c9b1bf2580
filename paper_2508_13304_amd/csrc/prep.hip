// Elementwise preparation passes (HBM-bound, coalesced along x / u):
//   - zero-padded copy of the volume for the forward march;
//   - volume gradient field (central differences, Sec. II-C: the volume
//     gradient in G_f is approximated by a central finite difference),
//     stored as three zero-padded planes Gx, Gy, Gz in voxel-index units
//     (half the neighbour difference), zero outside the grid, optionally
//     with the padded mu plane, and the same values interleaved per voxel;
//   - per padded detector pixel, the 2x2 bilinear footprint of the
//     zero-extended image as one float4, for the back-projection;
//   - detector gradient field (central differences of l, Sec. II-C) stored
//     as float4 (l, dl/da, dl/db, 0) in pixel-index units, zero outside.
#include "dp_internal.h"

namespace dp {

__device__ inline float vol_at(const float* __restrict__ v, int nx, int ny, int nz, int i, int j,
                               int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= nx || j >= ny || k >= nz) return 0.0f;
    return v[((size_t)k * ny + j) * nx + i];
}

__global__ __launch_bounds__(256) void vol_pad_kernel(int nx, int ny, int nz,
                                                      const float* __restrict__ vol,
                                                      float* __restrict__ volp)
{
    const int NX = nx + 2 * kPadV, NY = ny + 2 * kPadV, NZ = nz + 2 * kPadV;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y, K = blockIdx.z;
    if (I >= NX) return;
    (void)NZ;
    volp[((size_t)K * NY + J) * NX + I] = vol_at(vol, nx, ny, nz, I - kPadV, J - kPadV, K - kPadV);
}

// One pass for the gradient marches: the central-difference planes Gx, Gy,
// Gz (and, for the single-pass SSD, the padded mu plane) that the LDS boxes
// are loaded from, plus the same values interleaved per voxel as float4
// (mu, Gx, Gy, Gz) for tiles whose rays are too sparse to stage: there each
// trilinear corner is one 16-byte gather instead of four scattered ones.
template <bool MU>
__global__ __launch_bounds__(256) void vol_prep_kernel(int nx, int ny, int nz,
                                                       const float* __restrict__ vol,
                                                       float* __restrict__ mu_plane,
                                                       float* __restrict__ g3,
                                                       float4* __restrict__ inter)
{
    const int NX = nx + 2 * kPadV, NY = ny + 2 * kPadV, NZ = nz + 2 * kPadV;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y, K = blockIdx.z;
    if (I >= NX) return;
    const int i = I - kPadV, j = J - kPadV, k = K - kPadV;
    float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i >= 0 && j >= 0 && k >= 0 && i < nx && j < ny && k < nz) {
        o.x = vol[((size_t)k * ny + j) * nx + i];
        o.y = 0.5f * (vol_at(vol, nx, ny, nz, i + 1, j, k) - vol_at(vol, nx, ny, nz, i - 1, j, k));
        o.z = 0.5f * (vol_at(vol, nx, ny, nz, i, j + 1, k) - vol_at(vol, nx, ny, nz, i, j - 1, k));
        o.w = 0.5f * (vol_at(vol, nx, ny, nz, i, j, k + 1) - vol_at(vol, nx, ny, nz, i, j, k - 1));
    }
    const size_t plane = (size_t)NX * NY * NZ;
    const size_t e = ((size_t)K * NY + J) * NX + I;
    if (MU) mu_plane[e] = o.x;
    g3[e] = o.y;
    g3[plane + e] = o.z;
    g3[2 * plane + e] = o.w;
    inter[e] = o;
}

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

void launch_vol_pad(const GeoScalars& s, const float* vol, float* volp, hipStream_t st)
{
    const int NX = s.nx + 2 * kPadV;
    dim3 grid((NX + 255) / 256, s.ny + 2 * kPadV, s.nz + 2 * kPadV);
    prof_begin(DP_K_VOL_PREP, st);
    vol_pad_kernel<<<grid, 256, 0, st>>>(s.nx, s.ny, s.nz, vol, volp);
    prof_end(DP_K_VOL_PREP, st);
}

void launch_vol_prep(const GeoScalars& s, const float* vol, float* mu_plane, float* g3,
                     float4* inter, hipStream_t st)
{
    const int NX = s.nx + 2 * kPadV;
    dim3 grid((NX + 255) / 256, s.ny + 2 * kPadV, s.nz + 2 * kPadV);
    prof_begin(DP_K_VOL_PREP, st);
    if (mu_plane)
        vol_prep_kernel<true><<<grid, 256, 0, st>>>(s.nx, s.ny, s.nz, vol, mu_plane, g3, inter);
    else
        vol_prep_kernel<false><<<grid, 256, 0, st>>>(s.nx, s.ny, s.nz, vol, nullptr, g3, inter);
    prof_end(DP_K_VOL_PREP, st);
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
