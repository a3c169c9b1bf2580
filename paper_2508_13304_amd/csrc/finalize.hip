// Final cross-block sum (FP64, fixed order: deterministic) and the chain
// rule dL/dtheta = grad_theta M . dL/dM (Sec. II-B) in generator form:
// dR/dgamma_a = [omega_a]x R.
//
// Forward (per view, from the 9 per-block channel sums of the ray kernel):
//   b = B / h (per mm),  tau = sum phi p x g  (object frame)
//   dL/dt = -R b,  dL/dgamma_a = -omega_a . (R tau)
// Back-projection (per view, from the 12 channel sums of the voxel kernel):
//   dL/dt = sum_k A_k E_k,  dL/dgamma_a = omega_a . sum_k (R Q_k) x E_k
// with Q_k the object-frame moments (I - centre) * h.
#include "dp_internal.h"

namespace dp {

constexpr int kFinThreads = 256;

template <int C>
__device__ inline void fixed_order_sum(const float* __restrict__ part, int n_part, double* out)
{
    __shared__ double sh[C][kFinThreads];
    double acc[C];
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    for (int p = threadIdx.x; p < n_part; p += kFinThreads)
        for (int c = 0; c < C; ++c) acc[c] += (double)part[(size_t)p * C + c];
    for (int c = 0; c < C; ++c) sh[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int w = kFinThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int c = 0; c < C; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        __syncthreads();
    }
    for (int c = 0; c < C; ++c) out[c] = sh[c][0];
}

__device__ inline void cross3(const double* a, const double* b, double* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ inline void matvec3(const double* R, const double* x, double* y)
{
    for (int r = 0; r < 3; ++r) y[r] = R[r * 3 + 0] * x[0] + R[r * 3 + 1] * x[1] + R[r * 3 + 2] * x[2];
}

// C = 9 gradient channels; 10 with the per-view SSD of the fused kernel in
// channel 9 (written to loss[v]); 31 with the 21 Gauss-Newton entries after
// it (written to hess[v][21]).
template <int C>
__global__ __launch_bounds__(kFinThreads) void finalize_fwd_kernel(GeoScalars s,
                                                                   const ViewGeo* __restrict__ views,
                                                                   const float* __restrict__ partials,
                                                                   int n_part,
                                                                   double* __restrict__ grad_pose,
                                                                   double* __restrict__ loss,
                                                                   double* __restrict__ hess)
{
    const int v = blockIdx.x;
    double S[C];
    fixed_order_sum<C>(partials + (size_t)v * n_part * C, n_part, S);
    if (threadIdx.x != 0) return;
    if (C > kRdChannels && loss) loss[v] = S[kRdChannels];
    if (C == kRdChannelsGN && hess)
        for (int e = 0; e < 21; ++e) hess[21 * v + e] = S[kRdChannels + 1 + e];
    const ViewGeo& g = views[v];
    const double hx = s.vx, hy = s.vy, hz = s.vz;
    const double b[3] = {S[0] / hx, S[1] / hy, S[2] / hz};
    // S[3..8] = T_xy, T_xz, T_yx, T_yz, T_zx, T_zy (index units)
    const double tau[3] = {hy / hz * S[6] - hz / hy * S[8], hz / hx * S[7] - hx / hz * S[4],
                           hx / hy * S[3] - hy / hx * S[5]};
    double Rb[3], Rt[3];
    matvec3(g.R, b, Rb);
    matvec3(g.R, tau, Rt);
    double* out = grad_pose + 6 * v;
    for (int c = 0; c < 3; ++c) out[c] = -Rb[c];
    for (int a = 0; a < 3; ++a) {
        const double* w = g.omega + 3 * a;
        out[3 + a] = -(w[0] * Rt[0] + w[1] * Rt[1] + w[2] * Rt[2]);
    }
}

__global__ __launch_bounds__(kFinThreads) void finalize_bp_kernel(GeoScalars s,
                                                                  const ViewGeo* __restrict__ views,
                                                                  const float* __restrict__ partials,
                                                                  int n_part,
                                                                  double* __restrict__ grad_pose)
{
    const int v = blockIdx.x;
    double S[kVdChannels];
    fixed_order_sum<kVdChannels>(partials + (size_t)v * n_part * kVdChannels, n_part, S);
    if (threadIdx.x != 0) return;
    const ViewGeo& g = views[v];
    double gt[3] = {0.0, 0.0, 0.0}, tau[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 3; ++k) {
        const double* E = g.E + 3 * k;
        const double A = S[k];
        const double Q[3] = {S[3 + k] * s.vx, S[6 + k] * s.vy, S[9 + k] * s.vz};
        double RQ[3], x[3];
        matvec3(g.R, Q, RQ);
        cross3(RQ, E, x);
        for (int c = 0; c < 3; ++c) {
            gt[c] += A * E[c];
            tau[c] += x[c];
        }
    }
    double* out = grad_pose + 6 * v;
    for (int c = 0; c < 3; ++c) out[c] = gt[c];
    for (int a = 0; a < 3; ++a) {
        const double* w = g.omega + 3 * a;
        out[3 + a] = w[0] * tau[0] + w[1] * tau[1] + w[2] * tau[2];
    }
}

void launch_finalize_fwd(const GeoScalars& s, int V, const ViewGeo* views, const float* partials,
                         int n_part, double* grad_pose, hipStream_t st)
{
    prof_begin(DP_K_FINALIZE, st);
    finalize_fwd_kernel<kRdChannels><<<V, kFinThreads, 0, st>>>(s, views, partials, n_part, grad_pose,
                                                               nullptr, nullptr);
    prof_end(DP_K_FINALIZE, st);
}

void launch_finalize_fwd_ssd(const GeoScalars& s, int V, const ViewGeo* views,
                             const float* partials, int n_part, double* grad_pose, double* loss,
                             double* hess, hipStream_t st)
{
    prof_begin(DP_K_FINALIZE, st);
    if (hess)
        finalize_fwd_kernel<kRdChannelsGN><<<V, kFinThreads, 0, st>>>(s, views, partials, n_part,
                                                                      grad_pose, loss, hess);
    else
        finalize_fwd_kernel<kRdChannels + 1><<<V, kFinThreads, 0, st>>>(s, views, partials, n_part,
                                                                       grad_pose, loss, nullptr);
    prof_end(DP_K_FINALIZE, st);
}

void launch_finalize_bp(const GeoScalars& s, int V, const ViewGeo* views, const float* partials,
                        int n_part, double* grad_pose, hipStream_t st)
{
    prof_begin(DP_K_FINALIZE, st);
    finalize_bp_kernel<<<V, kFinThreads, 0, st>>>(s, views, partials, n_part, grad_pose);
    prof_end(DP_K_FINALIZE, st);
}

}  // namespace dp
