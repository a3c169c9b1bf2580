// Per-view setup (FP64): rigid motion M = [R | t] from theta (notation
// table, Sec. II-A), the circular-orbit detector frame, the projective
// mapping of Eq. projmatrix expressed on voxel indices, and the rotation
// generators used by the chain rule dL/dtheta = grad_theta M . dL/dM
// (Sec. II-B).  One thread per view; poses stay on the device so replays
// of a captured launch sequence see updated poses.
#include "dp_internal.h"

namespace dp {

__device__ inline void mat3_mul(const double* A, const double* B, double* C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[i * 3 + j] = A[i * 3 + 0] * B[0 * 3 + j] + A[i * 3 + 1] * B[1 * 3 + j] +
                           A[i * 3 + 2] * B[2 * 3 + j];
}

__global__ void view_setup_kernel(GeoScalars s, int V, const double* __restrict__ angles,
                                  const double* __restrict__ poses, ViewGeo* __restrict__ out)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const double beta = angles[v];
    const double cb = cos(beta), sb = sin(beta);
    const double ew[3] = {-cb, -sb, 0.0};
    const double eu[3] = {-sb, cb, 0.0};
    const double ev[3] = {0.0, 0.0, 1.0};
    const double* th = poses + 6 * v;
    const double t[3] = {th[0], th[1], th[2]};
    const double cx = cos(th[3]), sx = sin(th[3]);
    const double cy = cos(th[4]), sy = sin(th[4]);
    const double cz = cos(th[5]), sz = sin(th[5]);
    const double Rx[9] = {1, 0, 0, 0, cx, -sx, 0, sx, cx};
    const double Ry[9] = {cy, 0, sy, 0, 1, 0, -sy, 0, cy};
    const double Rz[9] = {cz, -sz, 0, sz, cz, 0, 0, 0, 1};
    double T[9], R[9];
    mat3_mul(Rz, Ry, T);
    mat3_mul(T, Rx, R);

    const double h[3] = {s.vx, s.vy, s.vz};
    const double c[3] = {0.5 * (s.nx - 1), 0.5 * (s.ny - 1), 0.5 * (s.nz - 1)};
    ViewGeo g;
    // R^T e and R^T(-t), object frame, in (padded) voxel-index units.
    double rtu[3], rtv[3], rtw[3], rtt[3];
    for (int k = 0; k < 3; ++k) {
        rtu[k] = R[0 * 3 + k] * eu[0] + R[1 * 3 + k] * eu[1] + R[2 * 3 + k] * eu[2];
        rtv[k] = R[0 * 3 + k] * ev[0] + R[1 * 3 + k] * ev[1] + R[2 * 3 + k] * ev[2];
        rtw[k] = R[0 * 3 + k] * ew[0] + R[1 * 3 + k] * ew[1] + R[2 * 3 + k] * ew[2];
        rtt[k] = -(R[0 * 3 + k] * t[0] + R[1 * 3 + k] * t[1] + R[2 * 3 + k] * t[2]);
        g.EU[k] = rtu[k] / h[k];
        g.EV[k] = rtv[k] / h[k];
        g.EW[k] = rtw[k] / h[k];
        g.OT[k] = rtt[k] / h[k] + c[k] + kPadV;
    }
    // Projective mapping on voxel indices: r = R (I - c) h + t, then
    // U = (S/du) e_u.r, V = (S/dv) e_v.r, W = e_w.r + D (depth).
    const double su = s.sdd / s.du, sv = s.sdd / s.dv;
    double u3 = 0.0, v3 = 0.0, w3 = 0.0;
    for (int k = 0; k < 3; ++k) {
        g.PU[k] = (float)(su * rtu[k] * h[k]);
        g.PV[k] = (float)(sv * rtv[k] * h[k]);
        g.PW[k] = (float)(rtw[k] * h[k]);
        u3 -= rtu[k] * c[k] * h[k];
        v3 -= rtv[k] * c[k] * h[k];
        w3 -= rtw[k] * c[k] * h[k];
    }
    const double eut = eu[0] * t[0] + eu[1] * t[1] + eu[2] * t[2];
    const double evt = ev[0] * t[0] + ev[1] * t[1] + ev[2] * t[2];
    const double ewt = ew[0] * t[0] + ew[1] * t[1] + ew[2] * t[2];
    g.PU[3] = (float)(su * (u3 + eut));
    g.PV[3] = (float)(sv * (v3 + evt));
    g.PW[3] = (float)(w3 + ewt + s.sad);
    for (int k = 0; k < 3; ++k) {
        g.PUd[k] = su * rtu[k] * h[k];
        g.PVd[k] = sv * rtv[k] * h[k];
        g.PWd[k] = rtw[k] * h[k];
    }
    g.PUd[3] = su * (u3 + eut);
    g.PVd[3] = sv * (v3 + evt);
    g.PWd[3] = w3 + ewt + s.sad;
    for (int k = 0; k < 3; ++k) {
        g.E[0 * 3 + k] = su * eu[k];
        g.E[1 * 3 + k] = sv * ev[k];
        g.E[2 * 3 + k] = ew[k];
    }
    for (int k = 0; k < 9; ++k) g.R[k] = R[k];
    // dR/dg_a = [omega_a]x R with omega_x = Rz Ry e_x, omega_y = Rz e_y, omega_z = e_z.
    g.omega[0] = cz * cy; g.omega[1] = sz * cy; g.omega[2] = -sy;
    g.omega[3] = -sz;     g.omega[4] = cz;      g.omega[5] = 0.0;
    g.omega[6] = 0.0;     g.omega[7] = 0.0;     g.omega[8] = 1.0;
    out[v] = g;
}

void launch_view_setup(const GeoScalars& s, int V, const double* angles, const double* poses,
                       ViewGeo* views, hipStream_t st)
{
    const int threads = 64;
    prof_begin(DP_K_SETUP, st);
    view_setup_kernel<<<(V + threads - 1) / threads, threads, 0, st>>>(s, V, angles, poses, views);
    prof_end(DP_K_SETUP, st);
}

}  // namespace dp
