"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference for the cone-beam ray-driven
forward projector, the voxel-driven back-projector and their analytic
rigid-motion gradients (the C source is `dpref.c`; every routine cites the
paper passage it follows).  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no
code with the GPU library and imports nothing from it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dpref.c")
_LIB = os.path.join(_HERE, "libdpref.so")

W_NONE = 0
W_FDK = 1


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, IEEE semantics: no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Geom(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("vx", C.c_double), ("vy", C.c_double), ("vz", C.c_double),
                ("nu", C.c_int32), ("nv", C.c_int32),
                ("du", C.c_double), ("dv", C.c_double),
                ("off_u", C.c_double), ("off_v", C.c_double),
                ("sad", C.c_double), ("sdd", C.c_double), ("step", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _lib.dpref_count_samples.restype = C.c_int64
        _lib.dpref_num_threads.restype = C.c_int
        _lib.dpref_set_num_threads.argtypes = [C.c_int]
        _lib.dpref_set_num_threads.restype = None
    return _lib


def _g(geom) -> _Geom:
    return _Geom(int(geom.nx), int(geom.ny), int(geom.nz), float(geom.vx), float(geom.vy),
                 float(geom.vz), int(geom.nu), int(geom.nv), float(geom.du), float(geom.dv),
                 float(geom.off_u), float(geom.off_v), float(geom.sad), float(geom.sdd),
                 float(geom.step))


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _views(angles, poses):
    angles = _d(np.atleast_1d(angles))
    poses = _d(np.reshape(poses, (-1, 6)))
    assert angles.shape[0] == poses.shape[0]
    return angles, poses, int(angles.shape[0])


def num_threads() -> int:
    return int(lib().dpref_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads for the following calls (for timing; the parallel FP64
    sums may then add in another order)."""
    lib().dpref_set_num_threads(int(n))


def rotation(gamma) -> np.ndarray:
    R = np.zeros(9)
    lib().dpref_rotation(_p(_d(gamma)), _p(R))
    return R.reshape(3, 3)


def rotation_partials(gamma) -> np.ndarray:
    dR = np.zeros(27)
    lib().dpref_rotation_partials(_p(_d(gamma)), _p(dR))
    return dR.reshape(3, 3, 3)


def projection_matrix(geom, beta: float) -> np.ndarray:
    P = np.zeros(12)
    lib().dpref_projection_matrix(C.byref(_g(geom)), C.c_double(beta), _p(P))
    return P.reshape(3, 4)


def contract_pose(pose, dLdM) -> np.ndarray:
    out = np.zeros(6)
    lib().dpref_contract_pose(_p(_d(pose)), _p(_d(np.reshape(dLdM, 12))), _p(out))
    return out


def project_fwd(geom, angles, poses, vol) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    vol = _d(vol)
    out = np.zeros((V, geom.nv, geom.nu))
    lib().dpref_project_fwd(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(vol), _p(out))
    return out


def project_fwd_rays(geom, angles, poses, vol, ray_ids) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    vol = _d(vol)
    ids = np.ascontiguousarray(ray_ids, dtype=np.int64)
    out = np.zeros(ids.shape[0])
    lib().dpref_project_fwd_rays(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(vol),
                                 C.c_int64(ids.shape[0]), _p(ids), _p(out))
    return out


def count_samples(geom, angles, poses) -> int:
    angles, poses, V = _views(angles, poses)
    return int(lib().dpref_count_samples(C.byref(_g(geom)), V, _p(angles), _p(poses)))


def count_samples_per_ray(geom, angles, poses) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((V, geom.nv, geom.nu), dtype=np.int64)
    lib().dpref_count_samples_per_ray(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(out))
    return out


def project_fwd_T(geom, angles, poses, proj) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    proj = _d(proj)
    out = np.zeros((geom.nz, geom.ny, geom.nx))
    lib().dpref_project_fwd_T(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(proj), _p(out))
    return out


def project_fwd_grad_M(geom, angles, poses, vol, grad_proj) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((V, 3, 4))
    lib().dpref_project_fwd_grad_M(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(_d(vol)),
                                   _p(_d(grad_proj)), _p(out))
    return out


def project_fwd_grad_M_materialized(geom, angles, poses, vol, grad_proj) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((V, 3, 4))
    lib().dpref_project_fwd_grad_M_materialized(C.byref(_g(geom)), V, _p(angles), _p(poses),
                                                _p(_d(vol)), _p(_d(grad_proj)), _p(out))
    return out


def project_fwd_grad_pose(geom, angles, poses, vol, grad_proj) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((V, 6))
    lib().dpref_project_fwd_grad_pose(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(_d(vol)),
                                      _p(_d(grad_proj)), _p(out))
    return out


def project_fwd_jacobian(geom, angles, poses, vol) -> np.ndarray:
    """Per-ray pose Jacobian [V][nv][nu][6] of the forward projection (the
    gradient's per-ray sums before weighting by dL/dl)."""
    angles, poses, V = _views(angles, poses)
    out = np.zeros((V, geom.nv, geom.nu, 6))
    lib().dpref_project_fwd_jacobian(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(_d(vol)),
                                     _p(out))
    return out


def gauss_newton_ssd(geom, angles, poses, vol) -> np.ndarray:
    """Gauss-Newton matrix of the per-view SSD, 2 sum_rays J J^T, [V][6][6]."""
    J = project_fwd_jacobian(geom, angles, poses, vol)
    J = J.reshape(J.shape[0], -1, 6)
    return 2.0 * np.einsum("vpi,vpj->vij", J, J)


def backproject(geom, angles, poses, proj, weight_mode=W_NONE) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((geom.nz, geom.ny, geom.nx))
    lib().dpref_backproject(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(_d(proj)), _p(out),
                            int(weight_mode))
    return out


def backproject_voxels(geom, angles, poses, proj, vox_ids, weight_mode=W_NONE) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    ids = np.ascontiguousarray(vox_ids, dtype=np.int64)
    out = np.zeros(ids.shape[0])
    lib().dpref_backproject_voxels(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(_d(proj)),
                                   int(weight_mode), C.c_int64(ids.shape[0]), _p(ids), _p(out))
    return out


def vd_splat(geom, angles, poses, vol, weight_mode=W_NONE) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((V, geom.nv, geom.nu))
    lib().dpref_vd_splat(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(_d(vol)), _p(out),
                         int(weight_mode))
    return out


def backproject_grad_M(geom, angles, poses, proj, grad_vol, weight_mode=W_NONE) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((V, 3, 4))
    lib().dpref_backproject_grad_M(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(_d(proj)),
                                   _p(_d(grad_vol)), _p(out), int(weight_mode))
    return out


def backproject_grad_pose(geom, angles, poses, proj, grad_vol, weight_mode=W_NONE) -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((V, 6))
    lib().dpref_backproject_grad_pose(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(_d(proj)),
                                      _p(_d(grad_vol)), _p(out), int(weight_mode))
    return out


# ---------------------------------------------------------------------------
# Footprint projector pairs: separable footprint (kind "sf") and
# distance-driven (kind "dd")
# ---------------------------------------------------------------------------

FP_KINDS = {"sf": 0, "dd": 1}


def fp_project(geom, angles, poses, vol, kind="sf") -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((V, geom.nv, geom.nu))
    lib().dpref_fp_project(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(_d(vol)), _p(out),
                           FP_KINDS[kind])
    return out


def fp_backproject(geom, angles, poses, proj, kind="sf") -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((geom.nz, geom.ny, geom.nx))
    lib().dpref_fp_backproject(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(_d(proj)), _p(out),
                               FP_KINDS[kind])
    return out


def fp_project_grad_pose(geom, angles, poses, vol, grad_proj, kind="sf") -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((V, 6))
    lib().dpref_fp_project_grad_pose(C.byref(_g(geom)), V, _p(angles), _p(poses), _p(_d(vol)),
                                     _p(_d(grad_proj)), _p(out), FP_KINDS[kind])
    return out


def fp_backproject_grad_pose(geom, angles, poses, proj, grad_vol, kind="sf") -> np.ndarray:
    angles, poses, V = _views(angles, poses)
    out = np.zeros((V, 6))
    lib().dpref_fp_backproject_grad_pose(C.byref(_g(geom)), V, _p(angles), _p(poses),
                                         _p(_d(proj)), _p(_d(grad_vol)), _p(out), FP_KINDS[kind])
    return out


def sf_project(geom, angles, poses, vol):
    return fp_project(geom, angles, poses, vol, "sf")


def sf_backproject(geom, angles, poses, proj):
    return fp_backproject(geom, angles, poses, proj, "sf")


def sf_project_grad_pose(geom, angles, poses, vol, grad_proj):
    return fp_project_grad_pose(geom, angles, poses, vol, grad_proj, "sf")


def sf_backproject_grad_pose(geom, angles, poses, proj, grad_vol):
    return fp_backproject_grad_pose(geom, angles, poses, proj, grad_vol, "sf")
