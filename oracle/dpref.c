/*
 * dpref.c -- plain FP64 CPU oracle (see dpref.h).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.  It shares no code
 * with the GPU library.
 *
 * Every routine follows the paper (arXiv 2508.13304, "Differentiable Forward
 * and Back-Projector for Rigid Motion Estimation in X-ray Imaging") in its
 * own order and notation, without blocking or fusion:
 *   - rigid motion r = M r' = R r' + t, r' = R^T (r - t)   (notation table, Sec. II-A)
 *   - projective mapping d = p(r) = (u'/w', v'/w'), (u',v',w') = P [r;1]   (Eq. projmatrix)
 *   - forward l(d) = int mu(r'(r,M)) delta(p(r)-d) dr      (Eq. forward)
 *   - back    mu(r') = int l(d) delta(p(M r')-d) dd        (Eq. back)
 *   - forward gradient: project each entry of the per-voxel 3x4 matrix
 *     G_f = grad'mu^T grad_M r' with the same weights a^ij, weighted by dL/dl
 *     (Eqs. for_grad, final_forward, for_int, dis_forward)
 *   - back-projection gradient: G_b = grad_d l^T grad_r p grad_M r,
 *     back-projected with the same weights, weighted by dL/dmu
 *     (Eqs. back_derive, final_back, back_int, dis_back)
 *   - dL/dtheta = <dM/dtheta, dL/dM> (chain rule of Sec. II-B)
 *   - spatial gradients of mu and of l by central finite differences (Sec. II-C)
 *
 * Readings where the paper is silent (listed in the design notes):
 *   R = Rz(gz) Ry(gy) Rx(gx); rotation centre = volume centre = isocentre;
 *   circular source orbit in the z = 0 plane; samples at world-anchored arc
 *   lengths k*step (k >= 0) from the source; trilinear / bilinear
 *   interpolation on voxel / pixel centres, zero outside the grid; spatial
 *   gradients defined on grid points only (zero outside); G_f evaluated per
 *   voxel; optional FDK weight W = (D/w')^2 with its product-rule term.
 */
#include "dpref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int dpref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count for the following calls (timing only: no result depends on it
 * beyond the order of FP64 additions in the parallel sums). */
void dpref_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Pose algebra                                                             */
/* ------------------------------------------------------------------------ */

static void matmul3(const double A[9], const double B[9], double C[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
            C[i * 3 + j] = s;
        }
}

/* Elemental right-handed rotations and their derivatives d/dgamma. */
static void rot_x(double g, double M[9], double dM[9])
{
    double c = cos(g), s = sin(g);
    double m[9] = {1, 0, 0, 0, c, -s, 0, s, c};
    double d[9] = {0, 0, 0, 0, -s, -c, 0, c, -s};
    memcpy(M, m, sizeof m);
    memcpy(dM, d, sizeof d);
}
static void rot_y(double g, double M[9], double dM[9])
{
    double c = cos(g), s = sin(g);
    double m[9] = {c, 0, s, 0, 1, 0, -s, 0, c};
    double d[9] = {-s, 0, c, 0, 0, 0, -c, 0, -s};
    memcpy(M, m, sizeof m);
    memcpy(dM, d, sizeof d);
}
static void rot_z(double g, double M[9], double dM[9])
{
    double c = cos(g), s = sin(g);
    double m[9] = {c, -s, 0, s, c, 0, 0, 0, 1};
    double d[9] = {-s, -c, 0, c, -s, 0, 0, 0, 0};
    memcpy(M, m, sizeof m);
    memcpy(dM, d, sizeof d);
}

void dpref_rotation(const double gam[3], double R[9])
{
    double X[9], Y[9], Z[9], dX[9], dY[9], dZ[9], T[9];
    rot_x(gam[0], X, dX);
    rot_y(gam[1], Y, dY);
    rot_z(gam[2], Z, dZ);
    matmul3(Z, Y, T);
    matmul3(T, X, R);
}

void dpref_rotation_partials(const double gam[3], double dR[27])
{
    double X[9], Y[9], Z[9], dX[9], dY[9], dZ[9], T[9];
    rot_x(gam[0], X, dX);
    rot_y(gam[1], Y, dY);
    rot_z(gam[2], Z, dZ);
    matmul3(Z, Y, T);
    matmul3(T, dX, dR + 0);      /* dR/dgx = Rz Ry Rx' */
    matmul3(Z, dY, T);
    matmul3(T, X, dR + 9);       /* dR/dgy = Rz Ry' Rx */
    matmul3(dZ, Y, T);
    matmul3(T, X, dR + 18);      /* dR/dgz = Rz' Ry Rx */
}

/* dL/dtheta_q = sum_{i,c} (dM/dtheta_q)_{ic} (dL/dM)_{ic}, M = [R | t]. */
void dpref_contract_pose(const double pose[6], const double dLdM[12], double grad[6])
{
    double dR[27];
    dpref_rotation_partials(pose + 3, dR);
    for (int q = 0; q < 3; ++q) grad[q] = dLdM[q * 4 + 3];
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int c = 0; c < 3; ++c) s += dR[a * 9 + i * 3 + c] * dLdM[i * 4 + c];
        grad[3 + a] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Acquisition geometry (circular orbit in z = 0, flat detector)            */
/* ------------------------------------------------------------------------ */

typedef struct {
    double src[3], ew[3], eu[3], ev[3];
    double cu, cv;
} view_frame;

static view_frame make_frame(const dpref_geom* g, double beta)
{
    view_frame f;
    double c = cos(beta), s = sin(beta);
    f.src[0] = g->sad * c; f.src[1] = g->sad * s; f.src[2] = 0.0;
    f.ew[0] = -c; f.ew[1] = -s; f.ew[2] = 0.0;     /* source -> isocentre */
    f.eu[0] = -s; f.eu[1] = c;  f.eu[2] = 0.0;     /* detector columns    */
    f.ev[0] = 0.0; f.ev[1] = 0.0; f.ev[2] = 1.0;   /* detector rows       */
    f.cu = 0.5 * (g->nu - 1) + g->off_u;
    f.cv = 0.5 * (g->nv - 1) + g->off_v;
    return f;
}

/* P in pixel-index units: row 3 = [e_w, D] (depth), rows 1,2 map to (a, b). */
void dpref_projection_matrix(const dpref_geom* g, double beta, double P[12])
{
    view_frame f = make_frame(g, beta);
    double D = g->sad, S = g->sdd;
    for (int c = 0; c < 3; ++c) P[8 + c] = f.ew[c];
    P[11] = D;
    for (int c = 0; c < 4; ++c) {
        double eu = c < 3 ? f.eu[c] : 0.0, ev = c < 3 ? f.ev[c] : 0.0;
        P[0 + c] = (S / g->du) * eu + f.cu * P[8 + c];
        P[4 + c] = (S / g->dv) * ev + f.cv * P[8 + c];
    }
}

/* Unit direction of the ray from the source through pixel centre (a, b). */
static void ray_direction(const dpref_geom* g, const view_frame* f, int a, int b, double u[3])
{
    double xa = (a - f->cu) * g->du, yb = (b - f->cv) * g->dv;
    double q[3], n = 0.0;
    for (int c = 0; c < 3; ++c) {
        q[c] = g->sdd * f->ew[c] + xa * f->eu[c] + yb * f->ev[c]; /* pixel - source */
        n += q[c] * q[c];
    }
    n = sqrt(n);
    for (int c = 0; c < 3; ++c) u[c] = q[c] / n;
}

/* ------------------------------------------------------------------------ */
/* Interpolation (zero-extended)                                            */
/* ------------------------------------------------------------------------ */

static double vox(const double* v, const dpref_geom* g, long i, long j, long k)
{
    if (i < 0 || j < 0 || k < 0 || i >= g->nx || j >= g->ny || k >= g->nz) return 0.0;
    return v[((long)k * g->ny + j) * g->nx + i];
}

/* Trilinear interpolation at continuous voxel index (X, Y, Z). */
static double interp3(const double* v, const dpref_geom* g, double X, double Y, double Z)
{
    double fx = floor(X), fy = floor(Y), fz = floor(Z);
    long i0 = (long)fx, j0 = (long)fy, k0 = (long)fz;
    double wx[2] = {1.0 - (X - fx), X - fx};
    double wy[2] = {1.0 - (Y - fy), Y - fy};
    double wz[2] = {1.0 - (Z - fz), Z - fz};
    double s = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                s += wx[dx] * wy[dy] * wz[dz] * vox(v, g, i0 + dx, j0 + dy, k0 + dz);
    return s;
}

static double pix(const double* img, int nu, int nv, long a, long b)
{
    if (a < 0 || b < 0 || a >= nu || b >= nv) return 0.0;
    return img[(long)b * nu + a];
}

/* Bilinear interpolation at continuous pixel index (A, B). */
static double interp2(const double* img, int nu, int nv, double A, double B)
{
    double fa = floor(A), fb = floor(B);
    long a0 = (long)fa, b0 = (long)fb;
    double wa[2] = {1.0 - (A - fa), A - fa};
    double wb[2] = {1.0 - (B - fb), B - fb};
    double s = 0.0;
    for (int db = 0; db < 2; ++db)
        for (int da = 0; da < 2; ++da) s += wa[da] * wb[db] * pix(img, nu, nv, a0 + da, b0 + db);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Ray samples                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    double R[9];
    double t[3];
    view_frame f;
} view_pose;

static view_pose make_view(const dpref_geom* g, const double* angles, const double* poses, int v)
{
    view_pose vp;
    vp.f = make_frame(g, angles[v]);
    dpref_rotation(poses + 6 * v + 3, vp.R);
    for (int c = 0; c < 3; ++c) vp.t[c] = poses[6 * v + c];
    return vp;
}

/* Object-frame continuous voxel index of world point r: r' = R^T (r - t). */
static void world_to_index(const dpref_geom* g, const view_pose* vp, const double r[3], double X[3])
{
    double d[3] = {r[0] - vp->t[0], r[1] - vp->t[1], r[2] - vp->t[2]};
    double h[3] = {g->vx, g->vy, g->vz};
    int n[3] = {g->nx, g->ny, g->nz};
    for (int c = 0; c < 3; ++c) {
        double rp = vp->R[0 * 3 + c] * d[0] + vp->R[1 * 3 + c] * d[1] + vp->R[2 * 3 + c] * d[2];
        X[c] = rp / h[c] + 0.5 * (n[c] - 1);
    }
}

static int in_support(const dpref_geom* g, const double X[3])
{
    return X[0] > -1.0 && X[0] < g->nx && X[1] > -1.0 && X[1] < g->ny && X[2] > -1.0 &&
           X[2] < g->nz;
}

/* Range of sample numbers k that can reach the volume's support: the
 * support box (index range (-1, N) on every axis) lies inside a sphere of
 * radius rho centred on the moved volume centre t.  The range is only a
 * conservative bound; membership is decided per sample by in_support. */
static void sample_range(const dpref_geom* g, const view_pose* vp, const double u[3],
                         long* k_lo, long* k_hi)
{
    double hx = (g->nx + 1) * g->vx, hy = (g->ny + 1) * g->vy, hz = (g->nz + 1) * g->vz;
    double rho = 0.5 * sqrt(hx * hx + hy * hy + hz * hz);
    double lc = 0.0;
    for (int c = 0; c < 3; ++c) lc += (vp->t[c] - vp->f.src[c]) * u[c];
    long lo = (long)floor((lc - rho) / g->step) - 1;
    long hi = (long)ceil((lc + rho) / g->step) + 1;
    *k_lo = lo < 0 ? 0 : lo;
    *k_hi = hi;
}

static void sample_index(const dpref_geom* g, const view_pose* vp, const double u[3], long k,
                         double X[3])
{
    double r[3];
    for (int c = 0; c < 3; ++c) r[c] = vp->f.src[c] + (double)k * g->step * u[c];
    world_to_index(g, vp, r, X);
}

/* l_v[b][a] = step * sum_k mu~(X_k) over in-support samples. */
static double project_ray(const dpref_geom* g, const view_pose* vp, const double* vol, int a, int b)
{
    double u[3], X[3], s = 0.0;
    long k_lo, k_hi;
    ray_direction(g, &vp->f, a, b, u);
    sample_range(g, vp, u, &k_lo, &k_hi);
    for (long k = k_lo; k <= k_hi; ++k) {
        sample_index(g, vp, u, k, X);
        if (in_support(g, X)) s += interp3(vol, g, X[0], X[1], X[2]);
    }
    return g->step * s;
}

void dpref_project_fwd(const dpref_geom* g, int V, const double* angles, const double* poses,
                       const double* vol, double* proj)
{
    for (int v = 0; v < V; ++v) {
        view_pose vp = make_view(g, angles, poses, v);
        double* out = proj + (long)v * g->nu * g->nv;
#pragma omp parallel for schedule(dynamic, 4)
        for (int b = 0; b < g->nv; ++b)
            for (int a = 0; a < g->nu; ++a) out[(long)b * g->nu + a] = project_ray(g, &vp, vol, a, b);
    }
}

void dpref_project_fwd_rays(const dpref_geom* g, int V, const double* angles, const double* poses,
                            const double* vol, int64_t n_rays, const int64_t* ray_ids, double* out)
{
    long npix = (long)g->nu * g->nv;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < n_rays; ++r) {
        int64_t id = ray_ids[r];
        int v = (int)(id / npix);
        long rem = id % npix;
        int b = (int)(rem / g->nu), a = (int)(rem % g->nu);
        out[r] = 0.0;
        if (v < 0 || v >= V) continue;
        view_pose vp = make_view(g, angles, poses, v);
        out[r] = project_ray(g, &vp, vol, a, b);
    }
}

void dpref_count_samples_per_ray(const dpref_geom* g, int V, const double* angles,
                                 const double* poses, int64_t* counts)
{
    long npix = (long)g->nu * g->nv;
    for (int v = 0; v < V; ++v) {
        view_pose vp = make_view(g, angles, poses, v);
#pragma omp parallel for schedule(dynamic, 4)
        for (int b = 0; b < g->nv; ++b)
            for (int a = 0; a < g->nu; ++a) {
                double u[3], X[3];
                long k_lo, k_hi, n = 0;
                ray_direction(g, &vp.f, a, b, u);
                sample_range(g, &vp, u, &k_lo, &k_hi);
                for (long k = k_lo; k <= k_hi; ++k) {
                    sample_index(g, &vp, u, k, X);
                    n += in_support(g, X);
                }
                counts[(long)v * npix + (long)b * g->nu + a] = n;
            }
    }
}

int64_t dpref_count_samples(const dpref_geom* g, int V, const double* angles, const double* poses)
{
    long npix = (long)g->nu * g->nv;
    int64_t* c = (int64_t*)malloc(sizeof(int64_t) * npix * V);
    if (!c) return -1;
    dpref_count_samples_per_ray(g, V, angles, poses, c);
    int64_t s = 0;
    for (long i = 0; i < npix * V; ++i) s += c[i];
    free(c);
    return s;
}

/* Exact transpose: scatter step * phi_j(X_k) * y_ab to the 8 corners. */
void dpref_project_fwd_T(const dpref_geom* g, int V, const double* angles, const double* poses,
                         const double* proj, double* vol)
{
    long nvox = (long)g->nx * g->ny * g->nz;
    memset(vol, 0, sizeof(double) * nvox);
    for (int v = 0; v < V; ++v) {
        view_pose vp = make_view(g, angles, poses, v);
        for (int b = 0; b < g->nv; ++b)
            for (int a = 0; a < g->nu; ++a) {
                double y = proj[((long)v * g->nv + b) * g->nu + a];
                double u[3], X[3];
                long k_lo, k_hi;
                if (y == 0.0) continue;
                ray_direction(g, &vp.f, a, b, u);
                sample_range(g, &vp, u, &k_lo, &k_hi);
                for (long k = k_lo; k <= k_hi; ++k) {
                    sample_index(g, &vp, u, k, X);
                    if (!in_support(g, X)) continue;
                    double fx = floor(X[0]), fy = floor(X[1]), fz = floor(X[2]);
                    double wx[2] = {1.0 - (X[0] - fx), X[0] - fx};
                    double wy[2] = {1.0 - (X[1] - fy), X[1] - fy};
                    double wz[2] = {1.0 - (X[2] - fz), X[2] - fz};
                    for (int dz = 0; dz < 2; ++dz)
                        for (int dy = 0; dy < 2; ++dy)
                            for (int dx = 0; dx < 2; ++dx) {
                                long i = (long)fx + dx, j = (long)fy + dy, kk = (long)fz + dz;
                                if (i < 0 || j < 0 || kk < 0 || i >= g->nx || j >= g->ny || kk >= g->nz)
                                    continue;
                                vol[(kk * g->ny + j) * g->nx + i] +=
                                    g->step * wx[dx] * wy[dy] * wz[dz] * y;
                            }
                }
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Forward-projection pose gradient                                         */
/* ------------------------------------------------------------------------ */

/* Central-difference spatial gradient of mu (per mm), on grid voxels. */
static double* volume_gradient(const dpref_geom* g, const double* vol)
{
    long nvox = (long)g->nx * g->ny * g->nz;
    double* gr = (double*)malloc(sizeof(double) * 3 * nvox);
    if (!gr) return NULL;
#pragma omp parallel for
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                long id = (k * g->ny + j) * g->nx + i;
                gr[3 * id + 0] = (vox(vol, g, i + 1, j, k) - vox(vol, g, i - 1, j, k)) / (2.0 * g->vx);
                gr[3 * id + 1] = (vox(vol, g, i, j + 1, k) - vox(vol, g, i, j - 1, k)) / (2.0 * g->vy);
                gr[3 * id + 2] = (vox(vol, g, i, j, k + 1) - vox(vol, g, i, j, k - 1)) / (2.0 * g->vz);
            }
    return gr;
}

/* G_f^j = grad'mu_j^T grad_M r' at voxel j:  [ (r_j - t) g_j^T | -R g_j ],
 * with r_j - t = R p_j (p_j the object-frame voxel centre). */
static void forward_G(const dpref_geom* g, const view_pose* vp, const double* gr, long i, long j,
                      long k, double G[12])
{
    long id = (k * g->ny + j) * g->nx + i;
    double p[3] = {(i - 0.5 * (g->nx - 1)) * g->vx, (j - 0.5 * (g->ny - 1)) * g->vy,
                   (k - 0.5 * (g->nz - 1)) * g->vz};
    const double* gj = gr + 3 * id;
    double rp[3], Rg[3];
    for (int r = 0; r < 3; ++r) {
        rp[r] = vp->R[r * 3 + 0] * p[0] + vp->R[r * 3 + 1] * p[1] + vp->R[r * 3 + 2] * p[2];
        Rg[r] = vp->R[r * 3 + 0] * gj[0] + vp->R[r * 3 + 1] * gj[1] + vp->R[r * 3 + 2] * gj[2];
    }
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) G[r * 4 + c] = rp[r] * gj[c];
        G[r * 4 + 3] = -Rg[r];
    }
}

void dpref_project_fwd_grad_M(const dpref_geom* g, int V, const double* angles, const double* poses,
                              const double* vol, const double* grad_proj, double* dLdM)
{
    double* gr = volume_gradient(g, vol);
    if (!gr) return;
    for (int v = 0; v < V; ++v) {
        view_pose vp = make_view(g, angles, poses, v);
        double acc[12] = {0};
#pragma omp parallel
        {
            double loc[12] = {0};
#pragma omp for schedule(dynamic, 2)
            for (int b = 0; b < g->nv; ++b)
                for (int a = 0; a < g->nu; ++a) {
                    double w = grad_proj[((long)v * g->nv + b) * g->nu + a];
                    double u[3], X[3], G[12];
                    long k_lo, k_hi;
                    if (w == 0.0) continue;
                    ray_direction(g, &vp.f, a, b, u);
                    sample_range(g, &vp, u, &k_lo, &k_hi);
                    for (long k = k_lo; k <= k_hi; ++k) {
                        sample_index(g, &vp, u, k, X);
                        if (!in_support(g, X)) continue;
                        double fx = floor(X[0]), fy = floor(X[1]), fz = floor(X[2]);
                        double wx[2] = {1.0 - (X[0] - fx), X[0] - fx};
                        double wy[2] = {1.0 - (X[1] - fy), X[1] - fy};
                        double wz[2] = {1.0 - (X[2] - fz), X[2] - fz};
                        for (int dz = 0; dz < 2; ++dz)
                            for (int dy = 0; dy < 2; ++dy)
                                for (int dx = 0; dx < 2; ++dx) {
                                    long i = (long)fx + dx, j = (long)fy + dy, kk = (long)fz + dz;
                                    if (i < 0 || j < 0 || kk < 0 || i >= g->nx || j >= g->ny ||
                                        kk >= g->nz)
                                        continue; /* G_f is zero off the grid */
                                    double a_ij = g->step * wx[dx] * wy[dy] * wz[dz];
                                    forward_G(g, &vp, gr, i, j, kk, G);
                                    for (int e = 0; e < 12; ++e) loc[e] += w * a_ij * G[e];
                                }
                    }
                }
#pragma omp critical
            for (int e = 0; e < 12; ++e) acc[e] += loc[e];
        }
        memcpy(dLdM + 12 * v, acc, sizeof acc);
    }
    free(gr);
}

void dpref_project_fwd_grad_pose(const dpref_geom* g, int V, const double* angles,
                                 const double* poses, const double* vol, const double* grad_proj,
                                 double* grad_pose)
{
    double* dLdM = (double*)malloc(sizeof(double) * 12 * V);
    if (!dLdM) return;
    dpref_project_fwd_grad_M(g, V, angles, poses, vol, grad_proj, dLdM);
    for (int v = 0; v < V; ++v) dpref_contract_pose(poses + 6 * v, dLdM + 12 * v, grad_pose + 6 * v);
    free(dLdM);
}

/* Per-ray Jacobian J[v][b][a][6] = dl_ab/dtheta_v: the same sums as the
 * gradient with dL/dl = 1 on one ray, contracted per ray (so that
 * sum_ab w_ab J_ab = dL/dtheta for any w, and 2 sum_ab J_ab J_ab^T is the
 * Gauss-Newton matrix of the SSD). */
void dpref_project_fwd_jacobian(const dpref_geom* g, int V, const double* angles,
                                const double* poses, const double* vol, double* J)
{
    double* gr = volume_gradient(g, vol);
    if (!gr) return;
    for (int v = 0; v < V; ++v) {
        view_pose vp = make_view(g, angles, poses, v);
#pragma omp parallel for schedule(dynamic, 2)
        for (int b = 0; b < g->nv; ++b)
            for (int a = 0; a < g->nu; ++a) {
                double u[3], X[3], G[12], acc[12] = {0};
                long k_lo, k_hi;
                ray_direction(g, &vp.f, a, b, u);
                sample_range(g, &vp, u, &k_lo, &k_hi);
                for (long k = k_lo; k <= k_hi; ++k) {
                    sample_index(g, &vp, u, k, X);
                    if (!in_support(g, X)) continue;
                    double fx = floor(X[0]), fy = floor(X[1]), fz = floor(X[2]);
                    double wx[2] = {1.0 - (X[0] - fx), X[0] - fx};
                    double wy[2] = {1.0 - (X[1] - fy), X[1] - fy};
                    double wz[2] = {1.0 - (X[2] - fz), X[2] - fz};
                    for (int dz = 0; dz < 2; ++dz)
                        for (int dy = 0; dy < 2; ++dy)
                            for (int dx = 0; dx < 2; ++dx) {
                                long i = (long)fx + dx, j = (long)fy + dy, kk = (long)fz + dz;
                                if (i < 0 || j < 0 || kk < 0 || i >= g->nx || j >= g->ny ||
                                    kk >= g->nz)
                                    continue;
                                double a_ij = g->step * wx[dx] * wy[dy] * wz[dz];
                                forward_G(g, &vp, gr, i, j, kk, G);
                                for (int e = 0; e < 12; ++e) acc[e] += a_ij * G[e];
                            }
                }
                dpref_contract_pose(poses + 6 * v, acc, J + (((long)v * g->nv + b) * g->nu + a) * 6);
            }
    }
    free(gr);
}

/* Materialised route: build the 12 channel volumes G_f[m][n] for the view,
 * forward-project each with the same projector, and take the dL/dl-weighted
 * sum over the detector (the paper's "12x memory" alternative). */
void dpref_project_fwd_grad_M_materialized(const dpref_geom* g, int V, const double* angles,
                                           const double* poses, const double* vol,
                                           const double* grad_proj, double* dLdM)
{
    long nvox = (long)g->nx * g->ny * g->nz, npix = (long)g->nu * g->nv;
    double* gr = volume_gradient(g, vol);
    double* ch = (double*)malloc(sizeof(double) * nvox);
    double* pr = (double*)malloc(sizeof(double) * npix);
    if (!gr || !ch || !pr) { free(gr); free(ch); free(pr); return; }
    for (int v = 0; v < V; ++v) {
        view_pose vp = make_view(g, angles, poses, v);
        for (int e = 0; e < 12; ++e) {
            for (long k = 0; k < g->nz; ++k)
                for (long j = 0; j < g->ny; ++j)
                    for (long i = 0; i < g->nx; ++i) {
                        double G[12];
                        forward_G(g, &vp, gr, i, j, k, G);
                        ch[(k * g->ny + j) * g->nx + i] = G[e];
                    }
            dpref_project_fwd(g, 1, angles + v, poses + 6 * v, ch, pr);
            double s = 0.0;
            for (long p = 0; p < npix; ++p) s += grad_proj[(long)v * npix + p] * pr[p];
            dLdM[12 * v + e] = s;
        }
    }
    free(gr); free(ch); free(pr);
}

/* ------------------------------------------------------------------------ */
/* Voxel-driven back-projection                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    double P[12];
    double R[9], t[3];
    double D;
} bp_view;

static bp_view make_bp_view(const dpref_geom* g, const double* angles, const double* poses, int v)
{
    bp_view bv;
    dpref_projection_matrix(g, angles[v], bv.P);
    dpref_rotation(poses + 6 * v + 3, bv.R);
    for (int c = 0; c < 3; ++c) bv.t[c] = poses[6 * v + c];
    bv.D = g->sad;
    return bv;
}

static void voxel_centre(const dpref_geom* g, long i, long j, long k, double p[3])
{
    p[0] = (i - 0.5 * (g->nx - 1)) * g->vx;
    p[1] = (j - 0.5 * (g->ny - 1)) * g->vy;
    p[2] = (k - 0.5 * (g->nz - 1)) * g->vz;
}

/* World position r = M p and its projective coordinates (u', v', w'). */
static void project_point(const bp_view* bv, const double p[3], double r[3], double uvw[3])
{
    for (int c = 0; c < 3; ++c)
        r[c] = bv->R[c * 3 + 0] * p[0] + bv->R[c * 3 + 1] * p[1] + bv->R[c * 3 + 2] * p[2] + bv->t[c];
    for (int k = 0; k < 3; ++k)
        uvw[k] = bv->P[k * 4 + 0] * r[0] + bv->P[k * 4 + 1] * r[1] + bv->P[k * 4 + 2] * r[2] +
                 bv->P[k * 4 + 3];
}

static double fdk_weight(const bp_view* bv, double w, int mode)
{
    return mode == DPREF_W_FDK ? (bv->D / w) * (bv->D / w) : 1.0;
}

static double bp_voxel(const dpref_geom* g, int V, const bp_view* bvs, const double* proj,
                       int mode, long i, long j, long k)
{
    double p[3], r[3], uvw[3], s = 0.0;
    long npix = (long)g->nu * g->nv;
    voxel_centre(g, i, j, k, p);
    for (int v = 0; v < V; ++v) {
        project_point(&bvs[v], p, r, uvw);
        if (!(uvw[2] > 0.0)) continue; /* behind the source: no ray reaches it */
        double A = uvw[0] / uvw[2], B = uvw[1] / uvw[2];
        s += fdk_weight(&bvs[v], uvw[2], mode) * interp2(proj + v * npix, g->nu, g->nv, A, B);
    }
    return s;
}

static bp_view* make_bp_views(const dpref_geom* g, int V, const double* angles, const double* poses)
{
    bp_view* bvs = (bp_view*)malloc(sizeof(bp_view) * (V > 0 ? V : 1));
    if (!bvs) return NULL;
    for (int v = 0; v < V; ++v) bvs[v] = make_bp_view(g, angles, poses, v);
    return bvs;
}

void dpref_backproject(const dpref_geom* g, int V, const double* angles, const double* poses,
                       const double* proj, double* vol, int weight_mode)
{
    bp_view* bvs = make_bp_views(g, V, angles, poses);
    if (!bvs) return;
#pragma omp parallel for schedule(dynamic, 1)
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i)
                vol[(k * g->ny + j) * g->nx + i] = bp_voxel(g, V, bvs, proj, weight_mode, i, j, k);
    free(bvs);
}

void dpref_backproject_voxels(const dpref_geom* g, int V, const double* angles, const double* poses,
                              const double* proj, int weight_mode, int64_t n_vox,
                              const int64_t* vox_ids, double* out)
{
    bp_view* bvs = make_bp_views(g, V, angles, poses);
    if (!bvs) return;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t n = 0; n < n_vox; ++n) {
        int64_t id = vox_ids[n];
        long i = id % g->nx, j = (id / g->nx) % g->ny, k = id / ((long)g->nx * g->ny);
        out[n] = bp_voxel(g, V, bvs, proj, weight_mode, i, j, k);
    }
    free(bvs);
}

/* The forward operator whose transpose is the back-projector: splat
 * W * phi_ab(a, b) * mu_j onto the 4 nearest pixels. */
void dpref_vd_splat(const dpref_geom* g, int V, const double* angles, const double* poses,
                    const double* vol, double* proj, int weight_mode)
{
    long npix = (long)g->nu * g->nv;
    bp_view* bvs = make_bp_views(g, V, angles, poses);
    if (!bvs) return;
    memset(proj, 0, sizeof(double) * npix * V);
    for (int v = 0; v < V; ++v)
        for (long k = 0; k < g->nz; ++k)
            for (long j = 0; j < g->ny; ++j)
                for (long i = 0; i < g->nx; ++i) {
                    double x = vol[(k * g->ny + j) * g->nx + i];
                    double p[3], r[3], uvw[3];
                    if (x == 0.0) continue;
                    voxel_centre(g, i, j, k, p);
                    project_point(&bvs[v], p, r, uvw);
                    if (!(uvw[2] > 0.0)) continue;
                    double A = uvw[0] / uvw[2], B = uvw[1] / uvw[2];
                    double W = fdk_weight(&bvs[v], uvw[2], weight_mode);
                    double fa = floor(A), fb = floor(B);
                    double wa[2] = {1.0 - (A - fa), A - fa};
                    double wb[2] = {1.0 - (B - fb), B - fb};
                    for (int db = 0; db < 2; ++db)
                        for (int da = 0; da < 2; ++da) {
                            long aa = (long)fa + da, bb = (long)fb + db;
                            if (aa < 0 || bb < 0 || aa >= g->nu || bb >= g->nv) continue;
                            proj[v * npix + bb * g->nu + aa] += W * wa[da] * wb[db] * x;
                        }
                }
    free(bvs);
}

/* ------------------------------------------------------------------------ */
/* Back-projection pose gradient                                            */
/* ------------------------------------------------------------------------ */

/* Central differences of a detector image (per pixel), on grid pixels. */
static void image_gradient(const double* img, int nu, int nv, double* la, double* lb)
{
    for (long b = 0; b < nv; ++b)
        for (long a = 0; a < nu; ++a) {
            la[b * nu + a] = 0.5 * (pix(img, nu, nv, a + 1, b) - pix(img, nu, nv, a - 1, b));
            lb[b * nu + a] = 0.5 * (pix(img, nu, nv, a, b + 1) - pix(img, nu, nv, a, b - 1));
        }
}

void dpref_backproject_grad_M(const dpref_geom* g, int V, const double* angles, const double* poses,
                              const double* proj, const double* grad_vol, double* dLdM,
                              int weight_mode)
{
    long npix = (long)g->nu * g->nv;
    bp_view* bvs = make_bp_views(g, V, angles, poses);
    double* la = (double*)malloc(sizeof(double) * npix);
    double* lb = (double*)malloc(sizeof(double) * npix);
    if (!bvs || !la || !lb) { free(bvs); free(la); free(lb); return; }
    for (int v = 0; v < V; ++v) {
        const bp_view* bv = &bvs[v];
        const double* img = proj + v * npix;
        double acc[12] = {0};
        image_gradient(img, g->nu, g->nv, la, lb);
#pragma omp parallel
        {
            double loc[12] = {0};
#pragma omp for schedule(dynamic, 1)
            for (long k = 0; k < g->nz; ++k)
                for (long j = 0; j < g->ny; ++j)
                    for (long i = 0; i < g->nx; ++i) {
                        double e = grad_vol[(k * g->ny + j) * g->nx + i];
                        double p[3], r[3], uvw[3], gr[3];
                        if (e == 0.0) continue;
                        voxel_centre(g, i, j, k, p);
                        project_point(bv, p, r, uvw);
                        if (!(uvw[2] > 0.0)) continue;
                        double w = uvw[2], A = uvw[0] / w, B = uvw[1] / w;
                        double l = interp2(img, g->nu, g->nv, A, B);
                        double dl[2] = {interp2(la, g->nu, g->nv, A, B), interp2(lb, g->nu, g->nv, A, B)};
                        double W = fdk_weight(bv, w, weight_mode);
                        /* Jacobian of p(r): rows (P_k w' - P_3 u'_k) / w'^2 */
                        for (int c = 0; c < 3; ++c) {
                            double J0 = (bv->P[0 * 4 + c] * w - bv->P[2 * 4 + c] * uvw[0]) / (w * w);
                            double J1 = (bv->P[1 * 4 + c] * w - bv->P[2 * 4 + c] * uvw[1]) / (w * w);
                            double gW = weight_mode == DPREF_W_FDK
                                            ? -2.0 * bv->D * bv->D / (w * w * w) * bv->P[2 * 4 + c]
                                            : 0.0;
                            gr[c] = W * (J0 * dl[0] + J1 * dl[1]) + l * gW;
                        }
                        double pe[4] = {p[0], p[1], p[2], 1.0}; /* grad_M r = [p^T, 1] per row */
                        for (int rr = 0; rr < 3; ++rr)
                            for (int c = 0; c < 4; ++c) loc[rr * 4 + c] += e * gr[rr] * pe[c];
                    }
#pragma omp critical
            for (int q = 0; q < 12; ++q) acc[q] += loc[q];
        }
        memcpy(dLdM + 12 * v, acc, sizeof acc);
    }
    free(bvs); free(la); free(lb);
}

void dpref_backproject_grad_pose(const dpref_geom* g, int V, const double* angles,
                                 const double* poses, const double* proj, const double* grad_vol,
                                 double* grad_pose, int weight_mode)
{
    double* dLdM = (double*)malloc(sizeof(double) * 12 * (V > 0 ? V : 1));
    if (!dLdM) return;
    dpref_backproject_grad_M(g, V, angles, poses, proj, grad_vol, dLdM, weight_mode);
    for (int v = 0; v < V; ++v) dpref_contract_pose(poses + 6 * v, dLdM + 12 * v, grad_pose + 6 * v);
    free(dLdM);
}

/* ------------------------------------------------------------------------ */
/* Separable-footprint (SF) projector pair and its pose gradients           */
/* ------------------------------------------------------------------------ */
/* Weights a_ij of voxel j on pixel i (one view), with the voxel moved by the
 * pose (corners r = R p + t, projected by the view's P):
 *   transaxial: the four corners (x +- hx, y +- hy) of the voxel's mid-height
 *     cross-section project to column coordinates tau0 <= .. <= tau3, the
 *     breakpoints of a unit-height trapezoid T(a);
 *   axial: the top and bottom centres (z +- hz) project to rows b_lo, b_hi,
 *     a unit-height rectangle;
 *   amplitude: the chord L_j of the voxel cut by the line from the source
 *     through its centre;
 *   a_ij = L_j * int_{cell a} T * |[b_lo, b_hi] cap cell b|   (pixel cells of
 *     unit width centred on integer indices).
 * Forward: l_i = sum_j a_ij mu_j; back-projection: mu_j = sum_i a_ij l_i (the
 * exact transpose).  Gradients (Eqs. dis_forward / dis_back): the same
 * weights applied to G_f^j (per voxel) and to G_b^i (per pixel: the
 * central-difference detector gradient at the pixel, with the projection
 * Jacobian and grad_M r of the voxel). */

static double trap_cdf(double x, const double t[4])
{
    double s = 0.0;
    if (x > t[0] && t[1] > t[0]) {
        double xr = x < t[1] ? x : t[1];
        s += (xr - t[0]) * (xr - t[0]) / (2.0 * (t[1] - t[0]));
    }
    if (x > t[1]) s += (x < t[2] ? x : t[2]) - t[1];
    if (x > t[2] && t[3] > t[2]) {
        double xf = x < t[3] ? x : t[3];
        s += ((t[3] - t[2]) * (t[3] - t[2]) - (t[3] - xf) * (t[3] - xf)) / (2.0 * (t[3] - t[2]));
    }
    return s;
}

typedef struct {
    double tau[4], blo, bhi, L;
} sf_fp;

/* kind 0 (SF): trapezoid from the mid-height cross-section's corners,
 * amplitude = the central chord.  kind 1 (DD, distance-driven): a
 * unit-height rectangle between the projections of the voxel's two
 * boundaries across the view's dominant transaxial axis (x if the central
 * ray's object-frame direction has |d_x| >= |d_y|, else y), taken at the
 * voxel centre, and amplitude = the path length through the slab along the
 * dominant axis, h_dom |d| / |d_dom| for the line from the source through
 * the voxel centre.  Both use the same axial rectangle. */
static int sf_footprint_kind(const dpref_geom* g, const bp_view* bv, const double sobj[3], int kind,
                             int dom, long i, long j, long k, sf_fp* fp)
{
    double p[3], q[3], r[3], uvw[3];
    const double hx = 0.5 * g->vx, hy = 0.5 * g->vy, hz = 0.5 * g->vz;
    voxel_centre(g, i, j, k, p);
    if (kind == 0) {
        for (int c = 0; c < 4; ++c) {
            q[0] = p[0] + ((c & 1) ? hx : -hx);
            q[1] = p[1] + ((c & 2) ? hy : -hy);
            q[2] = p[2];
            project_point(bv, q, r, uvw);
            if (!(uvw[2] > 0.0)) return 0;
            fp->tau[c] = uvw[0] / uvw[2];
        }
        for (int a = 1; a < 4; ++a)  /* insertion sort of 4 values */
            for (int b = a; b > 0 && fp->tau[b - 1] > fp->tau[b]; --b) {
                double t = fp->tau[b]; fp->tau[b] = fp->tau[b - 1]; fp->tau[b - 1] = t;
            }
    } else {
        double e[2];
        for (int c = 0; c < 2; ++c) {
            q[0] = p[0]; q[1] = p[1]; q[2] = p[2];
            if (dom == 0) q[1] += c ? hy : -hy;  /* x-dominant: boundaries across y */
            else q[0] += c ? hx : -hx;           /* y-dominant: boundaries across x */
            project_point(bv, q, r, uvw);
            if (!(uvw[2] > 0.0)) return 0;
            e[c] = uvw[0] / uvw[2];
        }
        fp->tau[0] = fp->tau[1] = e[0] < e[1] ? e[0] : e[1];
        fp->tau[2] = fp->tau[3] = e[0] < e[1] ? e[1] : e[0];
    }
    double bb[2];
    for (int c = 0; c < 2; ++c) {
        q[0] = p[0]; q[1] = p[1]; q[2] = p[2] + (c ? hz : -hz);
        project_point(bv, q, r, uvw);
        if (!(uvw[2] > 0.0)) return 0;
        bb[c] = uvw[1] / uvw[2];
    }
    fp->blo = bb[0] < bb[1] ? bb[0] : bb[1];
    fp->bhi = bb[0] < bb[1] ? bb[1] : bb[0];
    double d[3] = {p[0] - sobj[0], p[1] - sobj[1], p[2] - sobj[2]};
    double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double h[3] = {hx, hy, hz};
    if (kind == 0) {
        double L = INFINITY;
        for (int c = 0; c < 3; ++c)
            if (d[c] != 0.0) {
                double s = h[c] / (fabs(d[c]) / n);
                if (s < L) L = s;
            }
        fp->L = 2.0 * L;
    } else {
        fp->L = d[dom] != 0.0 ? 2.0 * h[dom] * n / fabs(d[dom]) : 0.0;
    }
    return 1;
}

/* Dominant transaxial axis of a view: 0 (x) if the central ray (source to
 * the volume centre, object frame) has |d_x| >= |d_y|, else 1 (y). */
static int dd_dominant(const double sobj[3])
{
    return fabs(sobj[0]) >= fabs(sobj[1]) ? 0 : 1;
}

/* Pixel window of a footprint: cells overlapping (tau0, tau3) x (blo, bhi). */
static void sf_window(const dpref_geom* g, const sf_fp* fp, long* a0, long* a1, long* b0, long* b1)
{
    *a0 = (long)floor(fp->tau[0] - 0.5) + 1;
    *a1 = (long)ceil(fp->tau[3] + 0.5) - 1;
    *b0 = (long)floor(fp->blo - 0.5) + 1;
    *b1 = (long)ceil(fp->bhi + 0.5) - 1;
    if (*a0 < 0) *a0 = 0;
    if (*b0 < 0) *b0 = 0;
    if (*a1 > g->nu - 1) *a1 = g->nu - 1;
    if (*b1 > g->nv - 1) *b1 = g->nv - 1;
}

static double sf_weight(const sf_fp* fp, long a, long b)
{
    double ta = trap_cdf(a + 0.5, fp->tau) - trap_cdf(a - 0.5, fp->tau);
    double lo = b - 0.5 > fp->blo ? b - 0.5 : fp->blo;
    double hi = b + 0.5 < fp->bhi ? b + 0.5 : fp->bhi;
    double tb = hi > lo ? hi - lo : 0.0;
    return fp->L * ta * tb;
}

static void source_object_frame(const dpref_geom* g, double beta, const bp_view* bv, double s[3])
{
    view_frame f = make_frame(g, beta);
    double d[3] = {f.src[0] - bv->t[0], f.src[1] - bv->t[1], f.src[2] - bv->t[2]};
    for (int c = 0; c < 3; ++c) s[c] = bv->R[0 * 3 + c] * d[0] + bv->R[1 * 3 + c] * d[1] + bv->R[2 * 3 + c] * d[2];
}

void dpref_fp_project(const dpref_geom* g, int V, const double* angles, const double* poses,
                      const double* vol, double* proj, int kind)
{
    long npix = (long)g->nu * g->nv;
    for (int v = 0; v < V; ++v) {
        bp_view bv = make_bp_view(g, angles, poses, v);
        double sobj[3];
        source_object_frame(g, angles[v], &bv, sobj);
        const int dom = dd_dominant(sobj);
        double* img = proj + v * npix;
        for (long p = 0; p < npix; ++p) img[p] = 0.0;
#pragma omp parallel
        {
            double* loc = (double*)calloc(npix, sizeof(double));
#pragma omp for schedule(dynamic, 1)
            for (long k = 0; k < g->nz; ++k)
                for (long j = 0; j < g->ny; ++j)
                    for (long i = 0; i < g->nx; ++i) {
                        double mu = vol[(k * g->ny + j) * g->nx + i];
                        sf_fp fp;
                        long a0, a1, b0, b1;
                        if (mu == 0.0 || !sf_footprint_kind(g, &bv, sobj, kind, dom, i, j, k, &fp)) continue;
                        sf_window(g, &fp, &a0, &a1, &b0, &b1);
                        for (long b = b0; b <= b1; ++b)
                            for (long a = a0; a <= a1; ++a) loc[b * g->nu + a] += sf_weight(&fp, a, b) * mu;
                    }
#pragma omp critical
            for (long p = 0; p < npix; ++p) img[p] += loc[p];
            free(loc);
        }
    }
}

void dpref_fp_backproject(const dpref_geom* g, int V, const double* angles, const double* poses,
                          const double* proj, double* vol, int kind)
{
    long npix = (long)g->nu * g->nv;
    bp_view* bvs = make_bp_views(g, V, angles, poses);
    double* src = (double*)malloc(sizeof(double) * 3 * (V > 0 ? V : 1));
    if (!bvs || !src) { free(bvs); free(src); return; }
    for (int v = 0; v < V; ++v) source_object_frame(g, angles[v], &bvs[v], src + 3 * v);
#pragma omp parallel for schedule(dynamic, 1)
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                double s = 0.0;
                for (int v = 0; v < V; ++v) {
                    sf_fp fp;
                    long a0, a1, b0, b1;
                    if (!sf_footprint_kind(g, &bvs[v], src + 3 * v, kind, dd_dominant(src + 3 * v), i, j, k, &fp)) continue;
                    sf_window(g, &fp, &a0, &a1, &b0, &b1);
                    for (long b = b0; b <= b1; ++b)
                        for (long a = a0; a <= a1; ++a)
                            s += sf_weight(&fp, a, b) * proj[v * npix + b * g->nu + a];
                }
                vol[(k * g->ny + j) * g->nx + i] = s;
            }
    free(bvs);
    free(src);
}

void dpref_fp_project_grad_M(const dpref_geom* g, int V, const double* angles, const double* poses,
                             const double* vol, const double* grad_proj, double* dLdM, int kind)
{
    long npix = (long)g->nu * g->nv;
    double* gr = volume_gradient(g, vol);
    if (!gr) return;
    for (int v = 0; v < V; ++v) {
        bp_view bv = make_bp_view(g, angles, poses, v);
        view_pose vp = make_view(g, angles, poses, v);
        double sobj[3], acc[12] = {0};
        source_object_frame(g, angles[v], &bv, sobj);
        const int dom = dd_dominant(sobj);
        const double* w = grad_proj + v * npix;
#pragma omp parallel
        {
            double loc[12] = {0};
#pragma omp for schedule(dynamic, 1)
            for (long k = 0; k < g->nz; ++k)
                for (long j = 0; j < g->ny; ++j)
                    for (long i = 0; i < g->nx; ++i) {
                        sf_fp fp;
                        long a0, a1, b0, b1;
                        double G[12], s = 0.0;
                        if (!sf_footprint_kind(g, &bv, sobj, kind, dom, i, j, k, &fp)) continue;
                        sf_window(g, &fp, &a0, &a1, &b0, &b1);
                        for (long b = b0; b <= b1; ++b)
                            for (long a = a0; a <= a1; ++a) s += sf_weight(&fp, a, b) * w[b * g->nu + a];
                        if (s == 0.0) continue;
                        forward_G(g, &vp, gr, i, j, k, G);
                        for (int e = 0; e < 12; ++e) loc[e] += s * G[e];
                    }
#pragma omp critical
            for (int e = 0; e < 12; ++e) acc[e] += loc[e];
        }
        memcpy(dLdM + 12 * v, acc, sizeof acc);
    }
    free(gr);
}

void dpref_fp_backproject_grad_M(const dpref_geom* g, int V, const double* angles,
                                 const double* poses, const double* proj, const double* grad_vol,
                                 double* dLdM, int kind)
{
    long npix = (long)g->nu * g->nv;
    double* la = (double*)malloc(sizeof(double) * npix);
    double* lb = (double*)malloc(sizeof(double) * npix);
    if (!la || !lb) { free(la); free(lb); return; }
    for (int v = 0; v < V; ++v) {
        bp_view bv = make_bp_view(g, angles, poses, v);
        double sobj[3], acc[12] = {0};
        source_object_frame(g, angles[v], &bv, sobj);
        const int dom = dd_dominant(sobj);
        image_gradient(proj + v * npix, g->nu, g->nv, la, lb);
#pragma omp parallel
        {
            double loc[12] = {0};
#pragma omp for schedule(dynamic, 1)
            for (long k = 0; k < g->nz; ++k)
                for (long j = 0; j < g->ny; ++j)
                    for (long i = 0; i < g->nx; ++i) {
                        double e = grad_vol[(k * g->ny + j) * g->nx + i];
                        sf_fp fp;
                        long a0, a1, b0, b1;
                        double p[3], r[3], uvw[3], dl[2] = {0.0, 0.0};
                        if (e == 0.0 || !sf_footprint_kind(g, &bv, sobj, kind, dom, i, j, k, &fp)) continue;
                        sf_window(g, &fp, &a0, &a1, &b0, &b1);
                        for (long b = b0; b <= b1; ++b)
                            for (long a = a0; a <= a1; ++a) {
                                double wgt = sf_weight(&fp, a, b);
                                dl[0] += wgt * la[b * g->nu + a];
                                dl[1] += wgt * lb[b * g->nu + a];
                            }
                        voxel_centre(g, i, j, k, p);
                        project_point(&bv, p, r, uvw);
                        double w = uvw[2], pe[4] = {p[0], p[1], p[2], 1.0};
                        for (int rr = 0; rr < 3; ++rr) {
                            double J0 = (bv.P[0 * 4 + rr] * w - bv.P[2 * 4 + rr] * uvw[0]) / (w * w);
                            double J1 = (bv.P[1 * 4 + rr] * w - bv.P[2 * 4 + rr] * uvw[1]) / (w * w);
                            double gr = J0 * dl[0] + J1 * dl[1];
                            for (int c = 0; c < 4; ++c) loc[rr * 4 + c] += e * gr * pe[c];
                        }
                    }
#pragma omp critical
            for (int q = 0; q < 12; ++q) acc[q] += loc[q];
        }
        memcpy(dLdM + 12 * v, acc, sizeof acc);
    }
    free(la);
    free(lb);
}

void dpref_fp_project_grad_pose(const dpref_geom* g, int V, const double* angles,
                                const double* poses, const double* vol, const double* grad_proj,
                                double* grad_pose, int kind)
{
    double* dLdM = (double*)malloc(sizeof(double) * 12 * (V > 0 ? V : 1));
    if (!dLdM) return;
    dpref_fp_project_grad_M(g, V, angles, poses, vol, grad_proj, dLdM, kind);
    for (int v = 0; v < V; ++v) dpref_contract_pose(poses + 6 * v, dLdM + 12 * v, grad_pose + 6 * v);
    free(dLdM);
}

void dpref_fp_backproject_grad_pose(const dpref_geom* g, int V, const double* angles,
                                    const double* poses, const double* proj, const double* grad_vol,
                                    double* grad_pose, int kind)
{
    double* dLdM = (double*)malloc(sizeof(double) * 12 * (V > 0 ? V : 1));
    if (!dLdM) return;
    dpref_fp_backproject_grad_M(g, V, angles, poses, proj, grad_vol, dLdM, kind);
    for (int v = 0; v < V; ++v) dpref_contract_pose(poses + 6 * v, dLdM + 12 * v, grad_pose + 6 * v);
    free(dLdM);
}
