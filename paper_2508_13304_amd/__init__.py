"""MI355X (gfx950) differentiable cone-beam projector: Python binding.

Thin ctypes wrapper over the C ABI of `libdiffproj.so` (include/diffproj.h).
It only marshals arguments -- every step of the projector runs in the HIP
kernels of the library -- and uses torch for device memory and the current
stream.  There is no CPU fallback: if the library is missing, `load()`
raises.

Entry points (same names as the C ABI, without the `dp_` prefix):
  project_fwd, project_fwd_grad_pose, backproject, backproject_grad_pose,
  workspace_bytes, plus the event-based per-kernel profiler.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdiffproj.so")

W_NONE = 0
W_FDK = 1
OP_FWD, OP_FWD_GRAD, OP_BP, OP_BP_GRAD = 0, 1, 2, 3
KERNELS = ("setup", "vol_prep", "rd_fwd", "rd_grad", "det_prep", "vd_bp", "vd_grad", "finalize")

EXPORTS = ("dp_workspace_bytes", "dp_project_fwd", "dp_project_fwd_grad_pose", "dp_backproject",
           "dp_backproject_grad_pose", "dp_last_error", "dp_version", "dp_profile_enable",
           "dp_profile_collect", "dp_profile_read")


class DPGeom(C.Structure):
    """Mirror of `dp_geom`."""
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("vx", C.c_double), ("vy", C.c_double), ("vz", C.c_double),
                ("nu", C.c_int32), ("nv", C.c_int32),
                ("du", C.c_double), ("dv", C.c_double),
                ("off_u", C.c_double), ("off_v", C.c_double),
                ("sad", C.c_double), ("sdd", C.c_double), ("step", C.c_double)]


_lib = None


def load(path: str | None = None):
    """Load the built HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} is missing (run __graft_entry__.build())")
    lib = C.CDLL(p)
    vp, sz, i32 = C.c_void_p, C.c_size_t, C.c_int32
    g = C.POINTER(DPGeom)
    lib.dp_workspace_bytes.argtypes = [g, i32, i32]
    lib.dp_workspace_bytes.restype = sz
    lib.dp_project_fwd.argtypes = [g, i32, vp, vp, vp, vp, vp, sz, vp]
    lib.dp_project_fwd_grad_pose.argtypes = [g, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.dp_backproject.argtypes = [g, i32, vp, vp, vp, vp, i32, vp, sz, vp]
    lib.dp_backproject_grad_pose.argtypes = [g, i32, vp, vp, vp, vp, vp, i32, vp, sz, vp]
    for f in ("dp_project_fwd", "dp_project_fwd_grad_pose", "dp_backproject",
              "dp_backproject_grad_pose", "dp_profile_enable", "dp_profile_collect",
              "dp_profile_read"):
        getattr(lib, f).restype = C.c_int
    lib.dp_last_error.restype = C.c_char_p
    lib.dp_version.restype = i32
    lib.dp_profile_enable.argtypes = [i32]
    lib.dp_profile_read.argtypes = [i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    _lib = lib
    return lib


def geom_struct(geom) -> DPGeom:
    """Any object with the dp_geom field names (e.g. synth.Geom) -> DPGeom."""
    return DPGeom(*(getattr(geom, f) for f, _ in DPGeom._fields_))


def _check(rc: int, what: str):
    if rc != 0:
        msg = load().dp_last_error().decode()
        raise RuntimeError(f"{what} failed ({rc}): {msg}")


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def workspace_bytes(geom, n_views: int, op: int) -> int:
    return int(load().dp_workspace_bytes(C.byref(geom_struct(geom)), int(n_views), int(op)))


def _workspace(geom, n_views, op, ws, device):
    import torch
    need = workspace_bytes(geom, n_views, op)
    if need == 0:
        raise ValueError("invalid geometry / view count")
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
    if ws.numel() < need:
        raise ValueError(f"workspace needs {need} bytes")
    return ws


def _views(angles, poses):
    import torch
    V = int(angles.shape[0])
    _dev(angles, torch.float64, "angles", (V,))
    _dev(poses, torch.float64, "poses", (V, 6))
    return V


def project_fwd(geom, angles, poses, vol, out=None, ws=None, stream=None):
    """DRRs [V][nv][nu] f32 of vol [nz][ny][nx] f32 at gantry angles [V] and poses [V][6] (f64)."""
    import torch
    V = _views(angles, poses)
    if out is None:
        out = torch.empty((V, geom.nv, geom.nu), dtype=torch.float32, device=vol.device)
    ws = _workspace(geom, V, OP_FWD, ws, vol.device)
    rc = load().dp_project_fwd(C.byref(geom_struct(geom)), V, _dev(angles, torch.float64, "angles"),
                               _dev(poses, torch.float64, "poses"),
                               _dev(vol, torch.float32, "vol", (geom.nz, geom.ny, geom.nx)),
                               _dev(out, torch.float32, "out", (V, geom.nv, geom.nu)),
                               C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "dp_project_fwd")
    return out


def project_fwd_grad_pose(geom, angles, poses, vol, grad_proj, out=None, ws=None, stream=None):
    """dL/dtheta [V][6] f64 given dL/dl [V][nv][nu] f32."""
    import torch
    V = _views(angles, poses)
    if out is None:
        out = torch.empty((V, 6), dtype=torch.float64, device=vol.device)
    ws = _workspace(geom, V, OP_FWD_GRAD, ws, vol.device)
    rc = load().dp_project_fwd_grad_pose(
        C.byref(geom_struct(geom)), V, _dev(angles, torch.float64, "angles"),
        _dev(poses, torch.float64, "poses"),
        _dev(vol, torch.float32, "vol", (geom.nz, geom.ny, geom.nx)),
        _dev(grad_proj, torch.float32, "grad_proj", (V, geom.nv, geom.nu)),
        _dev(out, torch.float64, "out", (V, 6)), C.c_void_p(ws.data_ptr()), ws.numel(),
        _stream(stream))
    _check(rc, "dp_project_fwd_grad_pose")
    return out


def backproject(geom, angles, poses, proj, weight_mode=W_NONE, out=None, ws=None, stream=None):
    """Volume [nz][ny][nx] f32 back-projected from proj [V][nv][nu] f32."""
    import torch
    V = _views(angles, poses)
    if out is None:
        out = torch.empty((geom.nz, geom.ny, geom.nx), dtype=torch.float32, device=proj.device)
    ws = _workspace(geom, V, OP_BP, ws, proj.device)
    rc = load().dp_backproject(C.byref(geom_struct(geom)), V, _dev(angles, torch.float64, "angles"),
                               _dev(poses, torch.float64, "poses"),
                               _dev(proj, torch.float32, "proj", (V, geom.nv, geom.nu)),
                               _dev(out, torch.float32, "out", (geom.nz, geom.ny, geom.nx)),
                               int(weight_mode), C.c_void_p(ws.data_ptr()), ws.numel(),
                               _stream(stream))
    _check(rc, "dp_backproject")
    return out


def backproject_grad_pose(geom, angles, poses, proj, grad_vol, weight_mode=W_NONE, out=None,
                          ws=None, stream=None):
    """dL/dtheta [V][6] f64 given dL/dmu [nz][ny][nx] f32."""
    import torch
    V = _views(angles, poses)
    if out is None:
        out = torch.empty((V, 6), dtype=torch.float64, device=proj.device)
    ws = _workspace(geom, V, OP_BP_GRAD, ws, proj.device)
    rc = load().dp_backproject_grad_pose(
        C.byref(geom_struct(geom)), V, _dev(angles, torch.float64, "angles"),
        _dev(poses, torch.float64, "poses"),
        _dev(proj, torch.float32, "proj", (V, geom.nv, geom.nu)),
        _dev(grad_vol, torch.float32, "grad_vol", (geom.nz, geom.ny, geom.nx)),
        _dev(out, torch.float64, "out", (V, 6)), int(weight_mode), C.c_void_p(ws.data_ptr()),
        ws.numel(), _stream(stream))
    _check(rc, "dp_backproject_grad_pose")
    return out


# --------------------------------------------------------------------------
# Event-based per-kernel timing (HIP events on the launch stream)
# --------------------------------------------------------------------------

def profile_enable(on: bool = True):
    _check(load().dp_profile_enable(1 if on else 0), "dp_profile_enable")


def profile_collect() -> dict:
    """Wait for recorded events; return {kernel: (total_ms, launches)} and reset."""
    lib = load()
    _check(lib.dp_profile_collect(), "dp_profile_collect")
    out = {}
    for k, name in enumerate(KERNELS):
        ms, n = C.c_double(), C.c_int64()
        _check(lib.dp_profile_read(k, C.byref(ms), C.byref(n)), "dp_profile_read")
        if n.value:
            out[name] = (ms.value, n.value)
    return out
