// Elementwise preparation passes (HBM-bound, coalesced along x / u): the
// (mu, G) interleave of sparse-ray geometries, and detector images:
//   - per padded detector pixel, the bilinear coefficients of the
//     zero-extended image on the cell to its lower right as one float4, for
//     the back-projection;
//   - detector gradient field (central differences of l, Sec. II-C) stored
//     as float4 (l, dl/da, dl/db, 0) in pixel-index units, zero outside
//     (footprint projectors), or as the cell coefficients of the three fields
//     (voxel-driven back-projection gradient).
// Cell coefficients of pixel (A, B): with v_xy the image at (A + x, B + y),
//   (v00, v10 - v00, v01 - v00, v11 - v10 - v01 + v00),
// so that the bilinear value at (A + wa, B + wb) is
//   c0 + wa ca + wb cb + wa wb cab  (three FMAs per field).
#include "dp_internal.h"

namespace dp {

__device__ inline float pix_at(const float* __restrict__ img, int nu, int nv, int a, int b)
{
    if (a < 0 || b < 0 || a >= nu || b >= nv) return 0.0f;
    return img[(size_t)b * nu + a];
}

__device__ inline float4 cell_coef(float v00, float v10, float v01, float v11)
{
    return make_float4(v00, v10 - v00, v01 - v00, (v11 - v10) - (v01 - v00));
}

// Per padded pixel (A, B), the cell coefficients of the zero-extended image,
// so that a back-projection update gathers one 16-byte vector instead of two
// rows.
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
        cell_coef(pix_at(img, nu, nv, a, b), pix_at(img, nu, nv, a + 1, b),
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

// Per padded pixel (A, B), the cell coefficients of l, dl/da and dl/db, so
// that a back-projection gradient update gathers three 16-byte vectors,
// every lane of them used.
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
    t.l = cell_coef(q00.x, q10.x, q01.x, q11.x);
    t.a = cell_coef(q00.y, q10.y, q01.y, q11.y);
    t.b = cell_coef(q00.z, q10.z, q01.z, q11.z);
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

__device__ inline float vox_at(const float* __restrict__ v, int nx, int ny, int nz, int i, int j,
                               int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= nx || j >= ny || k >= nz) return 0.0f;
    return v[((size_t)k * ny + j) * nx + i];
}

// Per padded voxel (I, J, K) (pad kPadV), (mu, Gx, Gy, Gz) with G the central
// difference of the zero-extended volume on grid voxels (the ray kernels'
// staging convention: not halved), zero in the pad.  For the gradient
// kernels' tiles whose rays are too sparse to stage a box: one 16-byte
// gather per trilinear corner.
__global__ __launch_bounds__(256) void vol_inter_kernel(int nx, int ny, int nz,
                                                        const float* __restrict__ vol,
                                                        float4* __restrict__ inter)
{
    const int NX = nx + 2 * kPadV, NY = ny + 2 * kPadV;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y, K = blockIdx.z;
    if (I >= NX) return;
    const int i = I - kPadV, j = J - kPadV, k = K - kPadV;
    float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i >= 0 && j >= 0 && k >= 0 && i < nx && j < ny && k < nz) {
        o.x = vol[((size_t)k * ny + j) * nx + i];
        o.y = vox_at(vol, nx, ny, nz, i + 1, j, k) - vox_at(vol, nx, ny, nz, i - 1, j, k);
        o.z = vox_at(vol, nx, ny, nz, i, j + 1, k) - vox_at(vol, nx, ny, nz, i, j - 1, k);
        o.w = vox_at(vol, nx, ny, nz, i, j, k + 1) - vox_at(vol, nx, ny, nz, i, j, k - 1);
    }
    inter[((size_t)K * NY + J) * NX + I] = o;
}

void launch_vol_inter(const GeoScalars& s, const float* vol, float4* inter, hipStream_t st)
{
    const int NX = s.nx + 2 * kPadV;
    dim3 grid((NX + 255) / 256, s.ny + 2 * kPadV, s.nz + 2 * kPadV);
    prof_begin(DP_K_VOL_PREP, st);
    vol_inter_kernel<<<grid, 256, 0, st>>>(s.nx, s.ny, s.nz, vol, inter);
    prof_end(DP_K_VOL_PREP, st);
}

// A 16 x 16 tile's rays are sparse when the tile spans more than 13 voxels at
// the isocentre (pixel footprint above 0.85 voxel): chunk boxes of oblique
// views then outgrow the LDS even one sample deep.
bool sparse_rays(const GeoScalars& s)
{
    const double pix = (s.du > s.dv ? s.du : s.dv) * s.sad / s.sdd;
    const double h = s.vx < s.vy ? (s.vx < s.vz ? s.vx : s.vz) : (s.vy < s.vz ? s.vy : s.vz);
    return pix > 0.85 * h;
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
