// Device-side Levenberg-Marquardt update for batched rigid 2D/3D
// registration on the SSD (Sec. III-A's registration task, solved with the
// analytic pose gradient of Eq. final_for and the Gauss-Newton matrix
// 2 sum J J^T built from the same per-ray Jacobians).
//
// One thread per view, FP64 throughout.  The update reads the SSD f, the
// gradient g and the packed Gauss-Newton matrix H the single-pass SSD
// launch just evaluated at the trial poses, takes the accept/reject
// decision against the last accepted point, and writes the next trial
// poses, so an iteration is two launches with no host round trip.
//
// Parameters are scaled as z = (t / 1 mm, gamma / 1 deg): theta = D z with
// D = diag(1, 1, 1, r, r, r), r = pi / 180, so g_z = D g and H_z = D H D.
// The damped system (H_z + lam (diag H_z + 1e-12)) d = -g_z is solved by an
// unpivoted Cholesky factorisation (the matrix is symmetric positive
// definite for lam > 0 since H_z is a sum of outer products).

#include "dp_internal.h"

namespace dp {

namespace {

constexpr int kLmThreads = 64;
constexpr double kDeg = 0.017453292519943295769;  // pi / 180
constexpr double kLamMax = 1e10;
constexpr double kDown = 3.0;
constexpr double kUp = 4.0;

__device__ inline double scale_of(int k) { return k < 3 ? 1.0 : kDeg; }

// index of (r, c), r <= c, in the row-by-row upper triangle of a 6 x 6 matrix
__device__ inline int tri6(int r, int c) { return r * 6 - r * (r - 1) / 2 + (c - r); }

__global__ __launch_bounds__(kLmThreads) void lm_update_kernel(
    int n, double* __restrict__ trial, const double* __restrict__ loss,
    const double* __restrict__ grad, const double* __restrict__ hess,
    double* __restrict__ sp, double* __restrict__ sf, double* __restrict__ sg,
    double* __restrict__ sh, double* __restrict__ lam, int* __restrict__ done, double tol)
{
    const int i = blockIdx.x * kLmThreads + threadIdx.x;
    if (i >= n || done[i]) return;
    double* tp = trial + 6 * i;
    const double f = loss[i];
    const double f0 = sf[i];
    double l = lam[i];
    bool stop = false;
    if (f < f0) {  // also false for a NaN trial value: rejected
        double step = 0.0;
        for (int k = 0; k < 6; ++k) step = fmax(step, fabs(tp[k] - sp[6 * i + k]) / scale_of(k));
        const bool first = !isfinite(f0);
        for (int k = 0; k < 6; ++k) {
            sp[6 * i + k] = tp[k];
            sg[6 * i + k] = grad[6 * i + k];
        }
        for (int e = 0; e < 21; ++e) sh[21 * i + e] = hess[21 * i + e];
        sf[i] = f;
        if (!first) {
            l /= kDown;
            stop = step < tol;
        }
    } else {
        l *= kUp;
    }
    stop = stop || l > kLamMax;
    lam[i] = l;
    if (stop) {
        done[i] = 1;
        for (int k = 0; k < 6; ++k) tp[k] = sp[6 * i + k];
        return;
    }
    // damped system in the scaled parameters
    double A[6][6], b[6];
    for (int r = 0; r < 6; ++r) {
        b[r] = -sg[6 * i + r] * scale_of(r);
        for (int c = r; c < 6; ++c) {
            const double h = sh[21 * i + tri6(r, c)] * scale_of(r) * scale_of(c);
            A[r][c] = h;
            A[c][r] = h;
        }
    }
    for (int r = 0; r < 6; ++r) A[r][r] += l * (A[r][r] + 1e-12);
    // Cholesky A = L L^T in place (lower triangle)
    bool ok = true;
    for (int c = 0; c < 6; ++c) {
        double d = A[c][c];
        for (int k = 0; k < c; ++k) d -= A[c][k] * A[c][k];
        if (!(d > 0.0)) { ok = false; break; }
        d = sqrt(d);
        A[c][c] = d;
        for (int r = c + 1; r < 6; ++r) {
            double s = A[r][c];
            for (int k = 0; k < c; ++k) s -= A[r][k] * A[c][k];
            A[r][c] = s / d;
        }
    }
    if (!ok) {  // not positive definite (degenerate H): stay at the accepted pose
        done[i] = 1;
        for (int k = 0; k < 6; ++k) tp[k] = sp[6 * i + k];
        return;
    }
    double y[6], d[6];
    for (int r = 0; r < 6; ++r) {
        double s = b[r];
        for (int k = 0; k < r; ++k) s -= A[r][k] * y[k];
        y[r] = s / A[r][r];
    }
    for (int r = 5; r >= 0; --r) {
        double s = y[r];
        for (int k = r + 1; k < 6; ++k) s -= A[k][r] * d[k];
        d[r] = s / A[r][r];
    }
    for (int k = 0; k < 6; ++k) tp[k] = sp[6 * i + k] + d[k] * scale_of(k);
}

}  // namespace

void launch_lm_update(int n, double* trial, const double* loss, const double* grad,
                      const double* hess, double* state_pose, double* state_f, double* state_g,
                      double* state_h, double* lam, int* done, double tol, hipStream_t st)
{
    const int blocks = (n + kLmThreads - 1) / kLmThreads;
    lm_update_kernel<<<blocks, kLmThreads, 0, st>>>(n, trial, loss, grad, hess, state_pose,
                                                     state_f, state_g, state_h, lam, done, tol);
}

}  // namespace dp
