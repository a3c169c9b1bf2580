/*
 * dpref.h -- plain FP64 CPU oracle for the differentiable cone-beam
 * ray-driven forward projector, the voxel-driven back-projector, and the
 * analytic rigid-motion (6-DoF) gradients of both.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the GPU library.
 *
 * All buffers are HOST double arrays owned by the caller.
 *   volume  : [nz][ny][nx]  (x fastest), voxel (i,j,k) centre at
 *             ((i-(nx-1)/2) vx, (j-(ny-1)/2) vy, (k-(nz-1)/2) vz) mm
 *   images  : [V][nv][nu]   (u fastest)
 *   angles  : [V] gantry angle beta (rad)
 *   poses   : [V][6] (tx, ty, tz [mm], gx, gy, gz [rad])
 *   grads   : [V][6] dL/dtheta, same order, per mm and per rad
 */
#ifndef DPREF_H
#define DPREF_H
#include <stdint.h>

typedef struct {
    int32_t nx, ny, nz;
    double vx, vy, vz;
    int32_t nu, nv;
    double du, dv, off_u, off_v;
    double sad, sdd, step;
} dpref_geom;

enum { DPREF_W_NONE = 0, DPREF_W_FDK = 1 };

int  dpref_num_threads(void);
void dpref_set_num_threads(int n);

/* Pose algebra (notation table: theta = (t, gamma), M = [R | t]). */
void dpref_rotation(const double gam[3], double R[9]);
void dpref_rotation_partials(const double gam[3], double dR[27]);
void dpref_projection_matrix(const dpref_geom* g, double beta, double P[12]);

/* Forward projection, the continuous forward model discretised as a
 * trilinear march at world-anchored arc lengths k*step from the source. */
void dpref_project_fwd(const dpref_geom* g, int V, const double* angles,
                       const double* poses, const double* vol, double* proj);
void dpref_project_fwd_rays(const dpref_geom* g, int V, const double* angles,
                            const double* poses, const double* vol,
                            int64_t n_rays, const int64_t* ray_ids, double* out);
int64_t dpref_count_samples(const dpref_geom* g, int V, const double* angles,
                            const double* poses);
void dpref_count_samples_per_ray(const dpref_geom* g, int V, const double* angles,
                                 const double* poses, int64_t* counts);

/* Exact transpose of the forward projector (scatter), for the adjoint pin. */
void dpref_project_fwd_T(const dpref_geom* g, int V, const double* angles,
                         const double* poses, const double* proj, double* vol);

/* Forward pose gradient: dL/dM per view (12 entries, row-major 3x4) and the
 * contraction to dL/dtheta.  grad_proj = dL/dl. */
void dpref_project_fwd_grad_M(const dpref_geom* g, int V, const double* angles,
                              const double* poses, const double* vol,
                              const double* grad_proj, double* dLdM);
void dpref_project_fwd_jacobian(const dpref_geom* g, int V, const double* angles,
                                const double* poses, const double* vol, double* J);
void dpref_project_fwd_grad_pose(const dpref_geom* g, int V, const double* angles,
                                 const double* poses, const double* vol,
                                 const double* grad_proj, double* grad_pose);
/* Same gradient through materialised per-voxel G_f channel volumes, each
 * projected with the forward projector ("12x memory" route). */
void dpref_project_fwd_grad_M_materialized(const dpref_geom* g, int V,
                                           const double* angles, const double* poses,
                                           const double* vol, const double* grad_proj,
                                           double* dLdM);

/* Voxel-driven back-projection (weight_mode NONE or FDK). */
void dpref_backproject(const dpref_geom* g, int V, const double* angles,
                       const double* poses, const double* proj, double* vol,
                       int weight_mode);
void dpref_backproject_voxels(const dpref_geom* g, int V, const double* angles,
                              const double* poses, const double* proj, int weight_mode,
                              int64_t n_vox, const int64_t* vox_ids, double* out);
/* The forward operator whose exact transpose is the back-projector (splat). */
void dpref_vd_splat(const dpref_geom* g, int V, const double* angles,
                    const double* poses, const double* vol, double* proj,
                    int weight_mode);

/* Back-projection pose gradient; grad_vol = dL/dmu. */
void dpref_backproject_grad_M(const dpref_geom* g, int V, const double* angles,
                              const double* poses, const double* proj,
                              const double* grad_vol, double* dLdM, int weight_mode);
void dpref_backproject_grad_pose(const dpref_geom* g, int V, const double* angles,
                                 const double* poses, const double* proj,
                                 const double* grad_vol, double* grad_pose,
                                 int weight_mode);

/* dL/dtheta from dL/dM by explicit differentiation of M(theta). */
void dpref_contract_pose(const double pose[6], const double dLdM[12], double grad[6]);


/* Footprint projector pairs and pose gradients (oracle); kind 0 = separable
 * footprint (SF), 1 = distance-driven (DD). */
void dpref_fp_project(const dpref_geom* g, int V, const double* angles, const double* poses,
                      const double* vol, double* proj, int kind);
void dpref_fp_backproject(const dpref_geom* g, int V, const double* angles, const double* poses,
                          const double* proj, double* vol, int kind);
void dpref_fp_project_grad_M(const dpref_geom* g, int V, const double* angles, const double* poses,
                             const double* vol, const double* grad_proj, double* dLdM, int kind);
void dpref_fp_backproject_grad_M(const dpref_geom* g, int V, const double* angles,
                                 const double* poses, const double* proj, const double* grad_vol,
                                 double* dLdM, int kind);
void dpref_fp_project_grad_pose(const dpref_geom* g, int V, const double* angles,
                                const double* poses, const double* vol, const double* grad_proj,
                                double* grad_pose, int kind);
void dpref_fp_backproject_grad_pose(const dpref_geom* g, int V, const double* angles,
                                    const double* poses, const double* proj, const double* grad_vol,
                                    double* grad_pose, int kind);
#endif
