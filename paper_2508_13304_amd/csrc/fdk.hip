// FDK pre-filter and image-sharpness loss for motion-compensated
// reconstruction (the paper's motion-compensated FBP task, Sec. III-B).
//
// Pre-filter: the projections are referred to a virtual detector through
// the isocentre (pitch tau = du SAD/SDD), multiplied by the cosine weight
// SAD / sqrt(SAD^2 + u'^2 + v'^2), and each row is convolved with the
// band-limited ramp (Ram-Lak) kernel
//   h[0] = 1/(4 tau^2),  h[k] = -1/(pi^2 k^2 tau^2) for odd k,  0 for even k != 0,
//   q[a] = scale tau sum_n p_w[n] h[a - n]      (rows zero outside the detector).
// One block per detector row: the weighted row sits zero-padded in LDS and
// the odd-k kernel values in an LDS table, so every tap is two LDS reads and
// one FP64 FMA (the ramp's cancellation between h[0] and the odd taps would
// cost FP32 several digits on smooth rows).
//
// Sharpness: S = -sum over x, y, z forward differences d of d^2 (pairs
// inside the grid); dS/dmu_j = sum over axes of 2 (mu[j+e] - mu_j) where j+e
// exists, minus 2 (mu_j - mu[j-e]) where j-e exists.  FP32 per voxel, FP32
// block sums, FP64 fixed-order total.
//
// Gradient entropy (the sharpness criterion of the paper's motion-compensated
// FBP experiment): g_j = sqrt(dx^2 + dy^2 + dz^2 + eps) from the same forward
// differences, Z = sum g, GE = -sum (g/Z) log(g/Z) = log Z - (sum g log g) / Z.
// Pass 1 reduces sum g and sum g log g per block; a one-block kernel forms Z
// and GE in FP64; pass 2 writes dGE/dmu_i = sum over axes of
// c_{i-e} d_{i-e} - c_i d_i with c_j = -(log g_j - log Z + GE) / (Z g_j),
// recomputing g at i and at its three backward neighbours.
#include <cmath>

#include "dp_internal.h"

namespace dp {

constexpr int kFdkThreads = 256;
constexpr int kFdkMaxNu = 4000;  // LDS: 3 nu floats + nu/2 doubles <= 64 KiB

__global__ __launch_bounds__(kFdkThreads) void fdk_filter_kernel(
    int nu, int nv, double cu, double cv, double du_iso, double dv_iso, double sad, double tau,
    double scale, const float* proj, float* out)  // proj == out allowed (row staged first)
{
    // row[nu .. 2 nu) holds the weighted row; nu zeros on either side
    extern __shared__ __align__(16) unsigned char smem[];
    double* hodd = reinterpret_cast<double*>(smem);            // h[2 i + 1], i < nu / 2
    float* row = reinterpret_cast<float*>(smem + sizeof(double) * (nu / 2 + 1));
    const int r = blockIdx.x;  // row index over all views: v * nv + b
    const int b = r % nv;
    const float* src = proj + (size_t)r * nu;
    const double vv = ((double)b - cv) * dv_iso;
    for (int i = threadIdx.x; i < 3 * nu; i += kFdkThreads) {
        const int a = i - nu;
        float val = 0.0f;
        if (a >= 0 && a < nu) {
            const double uu = ((double)a - cu) * du_iso;
            val = (float)((double)src[a] * sad / sqrt(sad * sad + uu * uu + vv * vv));
        }
        row[i] = val;
    }
    const double pi2tau2 = M_PI * M_PI * tau * tau;
    for (int i = threadIdx.x; i < (nu + 1) / 2; i += kFdkThreads) {
        const double k = 2.0 * i + 1.0;
        hodd[i] = -1.0 / (pi2tau2 * k * k);
    }
    __syncthreads();
    const double h0 = 1.0 / (4.0 * tau * tau);
    float* dst = out + (size_t)r * nu;
    for (int a = threadIdx.x; a < nu; a += kFdkThreads) {
        const float* c = row + nu + a;
        double acc = h0 * (double)c[0];
        // odd offsets k = 2 i + 1 < nu: both neighbours a - k and a + k (zero padded)
        for (int i = 0; 2 * i + 1 < nu; ++i) {
            const int k = 2 * i + 1;
            acc = fma(hodd[i], (double)c[-k] + (double)c[k], acc);
        }
        dst[a] = (float)(scale * tau * acc);
    }
}

size_t fdk_filter_lds_bytes(int nu)
{
    return sizeof(double) * (nu / 2 + 1) + sizeof(float) * 3 * (size_t)nu;
}

void launch_fdk_filter(const GeoScalars& s, int V, const float* proj, float* out, double scale,
                       hipStream_t st)
{
    const double mag = s.sad / s.sdd;
    const double du_iso = s.du * mag, dv_iso = s.dv * mag;
    const size_t lds = fdk_filter_lds_bytes(s.nu);
    fdk_filter_kernel<<<(unsigned)(V * s.nv), kFdkThreads, lds, st>>>(
        s.nu, s.nv, s.cu, s.cv, du_iso, dv_iso, s.sad, du_iso, scale, proj, out);
}

int fdk_max_nu() { return kFdkMaxNu; }

// ---------------------------------------------------------------------------
// Sharpness
// ---------------------------------------------------------------------------

constexpr int kShThreads = 256;

__global__ __launch_bounds__(kShThreads) void sharpness_kernel(int nx, int ny, int nz,
                                                               const float* __restrict__ vol,
                                                               float* __restrict__ grad,
                                                               double* __restrict__ partial)
{
    __shared__ float red[kShThreads];
    const size_t n = (size_t)nx * ny * nz;
    const size_t i = (size_t)blockIdx.x * kShThreads + threadIdx.x;
    float s = 0.0f;
    if (i < n) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((size_t)nx * ny));
        const float m = vol[i];
        float g = 0.0f;
        const size_t sx = 1, sy = (size_t)nx, sz = (size_t)nx * ny;
        if (x + 1 < nx) { const float d = vol[i + sx] - m; s += d * d; g += 2.0f * d; }
        if (y + 1 < ny) { const float d = vol[i + sy] - m; s += d * d; g += 2.0f * d; }
        if (z + 1 < nz) { const float d = vol[i + sz] - m; s += d * d; g += 2.0f * d; }
        if (x > 0) g -= 2.0f * (m - vol[i - sx]);
        if (y > 0) g -= 2.0f * (m - vol[i - sy]);
        if (z > 0) g -= 2.0f * (m - vol[i - sz]);
        if (grad) grad[i] = g;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kShThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = (double)red[0];
}

// One block: fixed-order FP64 sum of the block partials, negated.
__global__ __launch_bounds__(kShThreads) void sharpness_total_kernel(int n_part,
                                                                     const double* __restrict__ partial,
                                                                     double* __restrict__ loss)
{
    __shared__ double red[kShThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < n_part; i += kShThreads) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kShThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = -red[0];
}

size_t sharpness_partials(int nx, int ny, int nz)
{
    return ((size_t)nx * ny * nz + kShThreads - 1) / kShThreads;
}

void launch_sharpness(int nx, int ny, int nz, const float* vol, float* grad, double* loss,
                      double* partial, hipStream_t st)
{
    const size_t blocks = sharpness_partials(nx, ny, nz);
    sharpness_kernel<<<(unsigned)blocks, kShThreads, 0, st>>>(nx, ny, nz, vol, grad, partial);
    sharpness_total_kernel<<<1, kShThreads, 0, st>>>((int)blocks, partial, loss);
}

// ---------------------------------------------------------------------------
// Gradient entropy
// ---------------------------------------------------------------------------

struct GeDiffs {
    float dx, dy, dz, g;
};

__device__ inline GeDiffs ge_at(const float* __restrict__ vol, int x, int y, int z, int nx, int ny,
                                int nz, float eps)
{
    const size_t i = ((size_t)z * ny + y) * nx + x;
    const float m = vol[i];
    GeDiffs d;
    d.dx = x + 1 < nx ? vol[i + 1] - m : 0.0f;
    d.dy = y + 1 < ny ? vol[i + nx] - m : 0.0f;
    d.dz = z + 1 < nz ? vol[i + (size_t)nx * ny] - m : 0.0f;
    d.g = sqrtf(d.dx * d.dx + d.dy * d.dy + d.dz * d.dz + eps);
    return d;
}

__global__ __launch_bounds__(kShThreads) void ge_sums_kernel(int nx, int ny, int nz, float eps,
                                                             const float* __restrict__ vol,
                                                             double* __restrict__ partial)
{
    __shared__ float r1[kShThreads], r2[kShThreads];
    const size_t n = (size_t)nx * ny * nz;
    const size_t i = (size_t)blockIdx.x * kShThreads + threadIdx.x;
    float s1 = 0.0f, s2 = 0.0f;
    if (i < n) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((size_t)nx * ny));
        const float g = ge_at(vol, x, y, z, nx, ny, nz, eps).g;
        s1 = g;
        s2 = g * logf(g);
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int w = kShThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = (double)r1[0];
        partial[2 * blockIdx.x + 1] = (double)r2[0];
    }
}

// scal[0] = Z, scal[1] = GE, scal[2] = log Z; *loss = GE.
__global__ __launch_bounds__(kShThreads) void ge_total_kernel(int n_part, const double* __restrict__ partial,
                                                              double* __restrict__ scal,
                                                              double* __restrict__ loss)
{
    __shared__ double r1[kShThreads], r2[kShThreads];
    double s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < n_part; i += kShThreads) {
        s1 += partial[2 * i];
        s2 += partial[2 * i + 1];
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int w = kShThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double Z = r1[0], lz = log(Z), ge = lz - r2[0] / Z;
        scal[0] = Z;
        scal[1] = ge;
        scal[2] = lz;
        loss[0] = ge;
    }
}

__global__ __launch_bounds__(kShThreads) void ge_grad_kernel(int nx, int ny, int nz, float eps,
                                                             const float* __restrict__ vol,
                                                             const double* __restrict__ scal,
                                                             float* __restrict__ grad)
{
    const size_t n = (size_t)nx * ny * nz;
    const size_t i = (size_t)blockIdx.x * kShThreads + threadIdx.x;
    if (i >= n) return;
    const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((size_t)nx * ny));
    const float invZ = (float)(1.0 / scal[0]);
    const float shift = (float)(scal[1] - scal[2]);  // GE - log Z
    // c_j = -(log g_j + GE - log Z) / (Z g_j)
    const GeDiffs d0 = ge_at(vol, x, y, z, nx, ny, nz, eps);
    const float c0 = -(logf(d0.g) + shift) * invZ / d0.g;
    float acc = -c0 * (d0.dx + d0.dy + d0.dz);
    if (x > 0) {
        const GeDiffs d = ge_at(vol, x - 1, y, z, nx, ny, nz, eps);
        acc += -(logf(d.g) + shift) * invZ / d.g * d.dx;
    }
    if (y > 0) {
        const GeDiffs d = ge_at(vol, x, y - 1, z, nx, ny, nz, eps);
        acc += -(logf(d.g) + shift) * invZ / d.g * d.dy;
    }
    if (z > 0) {
        const GeDiffs d = ge_at(vol, x, y, z - 1, nx, ny, nz, eps);
        acc += -(logf(d.g) + shift) * invZ / d.g * d.dz;
    }
    grad[i] = acc;
}

void launch_gradient_entropy(int nx, int ny, int nz, float eps, const float* vol, float* grad,
                             double* loss, double* ws, hipStream_t st)
{
    const size_t blocks = sharpness_partials(nx, ny, nz);
    double* partial = ws;                 // [blocks][2]
    double* scal = ws + 2 * blocks;       // Z, GE, log Z
    ge_sums_kernel<<<(unsigned)blocks, kShThreads, 0, st>>>(nx, ny, nz, eps, vol, partial);
    ge_total_kernel<<<1, kShThreads, 0, st>>>((int)blocks, partial, scal, loss);
    if (grad)
        ge_grad_kernel<<<(unsigned)blocks, kShThreads, 0, st>>>(nx, ny, nz, eps, vol, scal, grad);
}

size_t gradient_entropy_ws_doubles(int nx, int ny, int nz)
{
    return 2 * sharpness_partials(nx, ny, nz) + 4;
}

}  // namespace dp
