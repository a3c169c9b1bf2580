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
// Numerics: per-ray setup in FP64; each ray is anchored at its crossing of
// the iso-plane (a point of small magnitude), and the FP32 march evaluates
// X(m) = X0 + (f + m*step) * D with one rounding per FMA, so no absolute
// positions of ~1000 mm are ever formed in FP32.
#include "dp_internal.h"

namespace dp {

struct RayMarch {
    float x0, y0, z0;   // padded voxel index of the iso-plane anchor
    float dx, dy, dz;   // direction in voxel-index units per mm
    float f;            // arc-length offset of sample k0 from the anchor (mm)
    int m_lo, m_hi;     // sample range relative to k0 (inclusive); empty if m_lo > m_hi
};

// FP64 per-ray setup: anchor, direction, sample offset and the slab clip of
// the samples against the support (-1, n) of the trilinear interpolant.
__device__ inline RayMarch ray_setup(const GeoScalars& s, const ViewGeo& g, int a, int b)
{
    RayMarch r;
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
    bool empty = false;
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
    r.m_lo = 1;
    r.m_hi = 0;
    if (!empty && tlo < thi) {  // false for NaN inputs
        double mlo = ceil((tlo - f) / s.step), mhi = floor((thi - f) / s.step);
        mlo = fmax(mlo, -k0);  // k = k0 + m >= 0: in front of the source
        if (mlo <= mhi && mhi - mlo < 1.0e7) {
            r.m_lo = (int)mlo;
            r.m_hi = (int)mhi;
        }
    }
    r.x0 = (float)X0[0]; r.y0 = (float)X0[1]; r.z0 = (float)X0[2];
    r.dx = (float)Dir[0]; r.dy = (float)Dir[1]; r.dz = (float)Dir[2];
    r.f = (float)f;
    return r;
}

// Lane -> detector pixel: 4 wavefronts per block, each an 8x8 pixel tile.
__device__ inline void rd_pixel(const GeoScalars& s, int tile, int& a, int& b)
{
    const int tiles_u = (s.nu + kRdTile - 1) / kRdTile;
    const int tu = tile % tiles_u, tv = tile / tiles_u;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    a = tu * kRdTile + (wave & 1) * 8 + (lane & 7);
    b = tv * kRdTile + (wave >> 1) * 8 + (lane >> 3);
}

__global__ __launch_bounds__(kRdThreads) void rd_fwd_kernel(GeoScalars s,
                                                            const ViewGeo* __restrict__ views,
                                                            const float* __restrict__ volp,
                                                            float* __restrict__ proj)
{
    const int v = blockIdx.y;
    int a, b;
    rd_pixel(s, blockIdx.x, a, b);
    if (a >= s.nu || b >= s.nv) return;
    const ViewGeo& g = views[v];
    const RayMarch r = ray_setup(s, g, a, b);
    const int NX = s.nx + 2 * kPadV, NY = s.ny + 2 * kPadV, NZ = s.nz + 2 * kPadV;
    const int NXY = NX * NY;
    // Clamp bounds keep every tap inside the padded buffer even for
    // positions that FP32 rounding pushes across the support boundary.
    const float xmax = NX - 1.001f, ymax = NY - 1.001f, zmax = NZ - 1.001f;
    const float step = (float)s.step;
    float acc = 0.0f;
    for (int m = r.m_lo; m <= r.m_hi; ++m) {
        const float t = fmaf((float)m, step, r.f);
        const float X = fminf(fmaxf(fmaf(t, r.dx, r.x0), 0.0f), xmax);
        const float Y = fminf(fmaxf(fmaf(t, r.dy, r.y0), 0.0f), ymax);
        const float Z = fminf(fmaxf(fmaf(t, r.dz, r.z0), 0.0f), zmax);
        const float fx = floorf(X), fy = floorf(Y), fz = floorf(Z);
        const float wx = X - fx, wy = Y - fy, wz = Z - fz;
        const int idx = ((int)fz * NY + (int)fy) * NX + (int)fx;
        const float* p = volp + idx;
        const float c000 = p[0], c100 = p[1];
        const float c010 = p[NX], c110 = p[NX + 1];
        const float c001 = p[NXY], c101 = p[NXY + 1];
        const float c011 = p[NXY + NX], c111 = p[NXY + NX + 1];
        const float c00 = fmaf(wx, c100 - c000, c000);
        const float c10 = fmaf(wx, c110 - c010, c010);
        const float c01 = fmaf(wx, c101 - c001, c001);
        const float c11 = fmaf(wx, c111 - c011, c011);
        const float c0 = fmaf(wy, c10 - c00, c00);
        const float c1 = fmaf(wy, c11 - c01, c01);
        acc += fmaf(wz, c1 - c0, c0);
    }
    proj[((size_t)v * s.nv + b) * s.nu + a] = acc * step;
}

__device__ inline float lerpf(float a, float b, float w) { return fmaf(w, b - a, a); }

// Deterministic block reduction of C channels: butterfly within each
// wavefront, then a fixed-order sum over the 4 wavefronts.
template <int C>
__device__ inline void block_reduce_store(float (&v)[C], float* __restrict__ out)
{
    __shared__ float red[4][C];
#pragma unroll
    for (int c = 0; c < C; ++c)
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) red[wave][c] = v[c];
    }
    __syncthreads();
    if (threadIdx.x < C) {
        const int c = threadIdx.x;
        out[c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    }
}

__global__ __launch_bounds__(kRdThreads) void rd_grad_kernel(GeoScalars s,
                                                             const ViewGeo* __restrict__ views,
                                                             const float4* __restrict__ vol4,
                                                             const float* __restrict__ grad_proj,
                                                             float* __restrict__ partials)
{
    const int v = blockIdx.y;
    int a, b;
    rd_pixel(s, blockIdx.x, a, b);
    float acc[kRdChannels];
#pragma unroll
    for (int c = 0; c < kRdChannels; ++c) acc[c] = 0.0f;
    const float w = (a < s.nu && b < s.nv) ? grad_proj[((size_t)v * s.nv + b) * s.nu + a] : 0.0f;
    if (w != 0.0f) {
        const ViewGeo& g = views[v];
        const RayMarch r = ray_setup(s, g, a, b);
        const int NX = s.nx + 2 * kPadV, NY = s.ny + 2 * kPadV, NZ = s.nz + 2 * kPadV;
        const int NXY = NX * NY;
        const float xmax = NX - 1.001f, ymax = NY - 1.001f, zmax = NZ - 1.001f;
        // Padded index of the grid centre: P_a(j) = I_a(j) - centre_a.
        const float ccx = 0.5f * (s.nx - 1) + kPadV, ccy = 0.5f * (s.ny - 1) + kPadV,
                    ccz = 0.5f * (s.nz - 1) + kPadV;
        const float step = (float)s.step;
        float Bx = 0.f, By = 0.f, Bz = 0.f;
        float Txy = 0.f, Txz = 0.f, Tyx = 0.f, Tyz = 0.f, Tzx = 0.f, Tzy = 0.f;
        for (int m = r.m_lo; m <= r.m_hi; ++m) {
            const float t = fmaf((float)m, step, r.f);
            const float X = fminf(fmaxf(fmaf(t, r.dx, r.x0), 0.0f), xmax);
            const float Y = fminf(fmaxf(fmaf(t, r.dy, r.y0), 0.0f), ymax);
            const float Z = fminf(fmaxf(fmaf(t, r.dz, r.z0), 0.0f), zmax);
            const float fx = floorf(X), fy = floorf(Y), fz = floorf(Z);
            const float wx = X - fx, wy = Y - fy, wz = Z - fz;
            const int idx = ((int)fz * NY + (int)fy) * NX + (int)fx;
            const float4* p = vol4 + idx;
            const float4 q000 = p[0], q100 = p[1];
            const float4 q010 = p[NX], q110 = p[NX + 1];
            const float4 q001 = p[NXY], q101 = p[NXY + 1];
            const float4 q011 = p[NXY + NX], q111 = p[NXY + NX + 1];
            // Channel Gx: lerp along x first; moments along y and z.
            float Gx, Mxy, Mxz;  // sum phi Gx, sum phi dy Gx, sum phi dz Gx
            {
                const float L00 = lerpf(q000.x, q100.x, wx), L10 = lerpf(q010.x, q110.x, wx);
                const float L01 = lerpf(q001.x, q101.x, wx), L11 = lerpf(q011.x, q111.x, wx);
                const float Y0 = lerpf(L00, L01, wz), Y1 = lerpf(L10, L11, wz);
                Gx = lerpf(Y0, Y1, wy);
                Mxy = wy * Y1;
                Mxz = wz * lerpf(L01, L11, wy);
            }
            // Channel Gy: lerp along y first; moments along x and z.
            float Gy, Myx, Myz;
            {
                const float L00 = lerpf(q000.y, q010.y, wy), L10 = lerpf(q100.y, q110.y, wy);
                const float L01 = lerpf(q001.y, q011.y, wy), L11 = lerpf(q101.y, q111.y, wy);
                const float X0 = lerpf(L00, L01, wz), X1 = lerpf(L10, L11, wz);
                Gy = lerpf(X0, X1, wx);
                Myx = wx * X1;
                Myz = wz * lerpf(L01, L11, wx);
            }
            // Channel Gz: lerp along z first; moments along x and y.
            float Gz, Mzx, Mzy;
            {
                const float L00 = lerpf(q000.z, q001.z, wz), L10 = lerpf(q100.z, q101.z, wz);
                const float L01 = lerpf(q010.z, q011.z, wz), L11 = lerpf(q110.z, q111.z, wz);
                const float X0 = lerpf(L00, L01, wy), X1 = lerpf(L10, L11, wy);
                Gz = lerpf(X0, X1, wx);
                Mzx = wx * X1;
                Mzy = wy * lerpf(L01, L11, wx);
            }
            const float Px = fx - ccx, Py = fy - ccy, Pz = fz - ccz;
            Bx += Gx; By += Gy; Bz += Gz;
            // T_a,c += P_a(base) * sum phi G_c + sum phi delta_a G_c
            Txy += fmaf(Px, Gy, Myx); Txz += fmaf(Px, Gz, Mzx);
            Tyx += fmaf(Py, Gx, Mxy); Tyz += fmaf(Py, Gz, Mzy);
            Tzx += fmaf(Pz, Gx, Mxz); Tzy += fmaf(Pz, Gy, Myz);
        }
        const float ws = w * step;
        acc[0] = Bx * ws; acc[1] = By * ws; acc[2] = Bz * ws;
        acc[3] = Txy * ws; acc[4] = Txz * ws; acc[5] = Tyx * ws;
        acc[6] = Tyz * ws; acc[7] = Tzx * ws; acc[8] = Tzy * ws;
    }
    const int tiles = gridDim.x;
    block_reduce_store<kRdChannels>(acc, partials + ((size_t)v * tiles + blockIdx.x) * kRdChannels);
}

void launch_rd_fwd(const GeoScalars& s, int V, const ViewGeo* views, const float* volp,
                   float* proj, hipStream_t st)
{
    dim3 grid(rd_tiles(s), V);
    prof_begin(DP_K_RD_FWD, st);
    rd_fwd_kernel<<<grid, kRdThreads, 0, st>>>(s, views, volp, proj);
    prof_end(DP_K_RD_FWD, st);
}

void launch_rd_grad(const GeoScalars& s, int V, const ViewGeo* views, const float4* vol4,
                    const float* grad_proj, float* partials, hipStream_t st)
{
    dim3 grid(rd_tiles(s), V);
    prof_begin(DP_K_RD_GRAD, st);
    rd_grad_kernel<<<grid, kRdThreads, 0, st>>>(s, views, vol4, grad_proj, partials);
    prof_end(DP_K_RD_GRAD, st);
}

}  // namespace dp
