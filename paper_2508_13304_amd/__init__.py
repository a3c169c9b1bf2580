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
OP_FWD, OP_FWD_GRAD, OP_BP, OP_BP_GRAD, OP_FWD_SSD = 0, 1, 2, 3, 4
OP_FP_FWD, OP_FP_FWD_GRAD, OP_FP_BP, OP_FP_BP_GRAD = 5, 6, 7, 8
FP_KINDS = {"sf": 0, "dd": 1}  # separable footprint, distance-driven
KERNELS = ("setup", "vol_prep", "rd_fwd", "rd_grad", "det_prep", "vd_bp", "vd_grad", "finalize",
           "fdk_filter", "sharpness", "rd_fused", "footprint")

EXPORTS = ("dp_workspace_bytes", "dp_project_fwd", "dp_project_fwd_grad_pose", "dp_backproject",
           "dp_backproject_grad_pose", "dp_last_error", "dp_version", "dp_profile_enable",
           "dp_profile_collect", "dp_profile_read", "dp_batch_workspace_bytes",
           "dp_project_fwd_batch", "dp_project_fwd_grad_pose_batch", "dp_autotune",
           "dp_set_variant", "dp_get_variant", "dp_project_fwd_ssd_grad_pose",
           "dp_project_fwd_ssd_gauss_newton", "dp_fp_project", "dp_fp_backproject",
           "dp_fp_project_grad_pose", "dp_fp_backproject_grad_pose", "dp_fdk_filter", "dp_sharpness",
           "dp_sharpness_workspace_bytes", "dp_gradient_entropy",
           "dp_gradient_entropy_workspace_bytes", "dp_gemm_bf16", "dp_im2col3x3_bf16", "dp_col2im3x3",
           "dp_bias_act_bf16", "dp_act_bwd_bf16", "dp_colsum_bf16", "dp_gemm_bf16_ws_bytes",
           "dp_gemm_bf16_ws", "dp_gemm_bias_act_bf16", "dp_im2col3x3_ld_bf16",
           "dp_col2im3x3_act_bf16", "dp_adam_f32",
           "dp_project_fwd_ssd_gauss_newton_batch", "dp_lm_update", "dp_read_probe",
           "dp_bp_grad_flags_offset", "dp_lds_probe", "dp_project_fwd_ssd_grad_pose_noalloc",
           "dp_conv3x3_fwd_bf16", "dp_conv3x3_wgrad_ws_bytes", "dp_conv3x3_wgrad_bf16",
           "dp_conv3x3_dgrad_act_bf16")
MAX_BATCH = 16
N_VARIANTS = 9  # ray-driven kernel variants: 3 * tile shape (16x16, 32x8, 8x32) + chunk class


class DPGeom(C.Structure):
    """Mirror of `dp_geom`."""
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("vx", C.c_double), ("vy", C.c_double), ("vz", C.c_double),
                ("nu", C.c_int32), ("nv", C.c_int32),
                ("du", C.c_double), ("dv", C.c_double),
                ("off_u", C.c_double), ("off_v", C.c_double),
                ("sad", C.c_double), ("sdd", C.c_double), ("step", C.c_double)]


class DPProblem(C.Structure):
    """Mirror of `dp_problem`."""
    _fields_ = [("geom", DPGeom), ("n_views", C.c_int32), ("angles", C.c_void_p),
                ("poses", C.c_void_p), ("vol", C.c_void_p), ("proj", C.c_void_p),
                ("grad_proj", C.c_void_p), ("grad_pose", C.c_void_p), ("loss", C.c_void_p),
                ("hess", C.c_void_p)]


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
    lib.dp_bp_grad_flags_offset.argtypes = [g, i32]
    lib.dp_bp_grad_flags_offset.restype = sz
    lib.dp_project_fwd.argtypes = [g, i32, vp, vp, vp, vp, vp, sz, vp]
    lib.dp_project_fwd_grad_pose.argtypes = [g, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.dp_project_fwd_ssd_grad_pose.argtypes = [g, i32, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.dp_project_fwd_ssd_grad_pose.restype = C.c_int
    lib.dp_project_fwd_ssd_gauss_newton.argtypes = [g, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.dp_project_fwd_ssd_gauss_newton.restype = C.c_int
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
    P = C.POINTER(DPProblem)
    lib.dp_batch_workspace_bytes.argtypes = [P, i32, i32]
    lib.dp_batch_workspace_bytes.restype = sz
    lib.dp_project_fwd_batch.argtypes = [P, i32, vp, sz, i32, vp]
    lib.dp_project_fwd_grad_pose_batch.argtypes = [P, i32, vp, sz, i32, vp]
    lib.dp_project_fwd_batch.restype = C.c_int
    lib.dp_project_fwd_grad_pose_batch.restype = C.c_int
    lib.dp_project_fwd_ssd_gauss_newton_batch.argtypes = [P, i32, vp, sz, i32, vp]
    lib.dp_project_fwd_ssd_gauss_newton_batch.restype = C.c_int
    lib.dp_lm_update.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_double, vp]
    lib.dp_lm_update.restype = C.c_int
    lib.dp_read_probe.argtypes = [vp, C.c_int64, i32, i32, i32, vp, vp]
    lib.dp_read_probe.restype = C.c_int
    lib.dp_lds_probe.argtypes = [i32, i32, vp, vp]
    lib.dp_lds_probe.restype = C.c_int
    lib.dp_project_fwd_ssd_grad_pose_noalloc.argtypes = [g, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.dp_project_fwd_ssd_grad_pose_noalloc.restype = C.c_int
    lib.dp_autotune.argtypes = [i32, g, i32, vp, vp, vp, vp, vp, vp, sz, vp, i32,
                                C.POINTER(i32), C.POINTER(C.c_float)]
    lib.dp_autotune.restype = C.c_int
    lib.dp_set_variant.argtypes = [i32, i32]
    lib.dp_set_variant.restype = C.c_int
    lib.dp_get_variant.argtypes = [g, i32, i32]
    lib.dp_get_variant.restype = i32
    for f in ("dp_fp_project", "dp_fp_backproject"):
        getattr(lib, f).argtypes = [g, i32, vp, vp, vp, vp, i32, vp, sz, vp]
        getattr(lib, f).restype = C.c_int
    for f in ("dp_fp_project_grad_pose", "dp_fp_backproject_grad_pose"):
        getattr(lib, f).argtypes = [g, i32, vp, vp, vp, vp, vp, i32, vp, sz, vp]
        getattr(lib, f).restype = C.c_int
    lib.dp_fdk_filter.argtypes = [g, i32, vp, vp, C.c_double, vp]
    lib.dp_fdk_filter.restype = C.c_int
    lib.dp_sharpness_workspace_bytes.argtypes = [i32, i32, i32]
    lib.dp_sharpness_workspace_bytes.restype = sz
    lib.dp_sharpness.argtypes = [i32, i32, i32, vp, vp, vp, vp, sz, vp]
    lib.dp_sharpness.restype = C.c_int
    lib.dp_gradient_entropy_workspace_bytes.argtypes = [i32, i32, i32]
    lib.dp_gradient_entropy_workspace_bytes.restype = sz
    lib.dp_gradient_entropy.argtypes = [i32, i32, i32, vp, C.c_float, vp, vp, vp, sz, vp]
    lib.dp_gradient_entropy.restype = C.c_int
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


def project_fwd_ssd_grad_pose(geom, angles, poses, vol, target, proj=None, loss=None, grad=None,
                              ws=None, stream=None):
    """One pass: DRRs l [V][nv][nu] f32, per-view SSD L_v = sum (l - y)^2 [V]
    f64 and its pose gradient [V][6] f64, for targets y [V][nv][nu] f32."""
    import torch
    V = _views(angles, poses)
    dev = vol.device
    if proj is None:
        proj = torch.empty((V, geom.nv, geom.nu), dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(V, dtype=torch.float64, device=dev)
    if grad is None:
        grad = torch.empty((V, 6), dtype=torch.float64, device=dev)
    ws = _workspace(geom, V, OP_FWD_SSD, ws, dev)
    rc = load().dp_project_fwd_ssd_grad_pose(
        C.byref(geom_struct(geom)), V, _dev(angles, torch.float64, "angles"),
        _dev(poses, torch.float64, "poses"),
        _dev(vol, torch.float32, "vol", (geom.nz, geom.ny, geom.nx)),
        _dev(target, torch.float32, "target", (V, geom.nv, geom.nu)),
        _dev(proj, torch.float32, "proj", (V, geom.nv, geom.nu)),
        _dev(loss, torch.float64, "loss", (V,)), _dev(grad, torch.float64, "grad", (V, 6)),
        C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "dp_project_fwd_ssd_grad_pose")
    return proj, loss, grad


def project_fwd_ssd_gauss_newton(geom, angles, poses, vol, target, proj=None, loss=None,
                                 grad=None, hess=None, ws=None, stream=None, packed=False):
    """One pass: DRRs, per-view SSD, its pose gradient and the Gauss-Newton
    matrix 2 sum J J^T as a symmetric [V][6][6] f64 tensor (packed=True:
    the [V][21] upper triangle as the kernel writes it)."""
    import torch
    V = _views(angles, poses)
    dev = vol.device
    if proj is None:
        proj = torch.empty((V, geom.nv, geom.nu), dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(V, dtype=torch.float64, device=dev)
    if grad is None:
        grad = torch.empty((V, 6), dtype=torch.float64, device=dev)
    if hess is None:
        hess = torch.empty((V, 21), dtype=torch.float64, device=dev)
    ws = _workspace(geom, V, OP_FWD_SSD, ws, dev)
    rc = load().dp_project_fwd_ssd_gauss_newton(
        C.byref(geom_struct(geom)), V, _dev(angles, torch.float64, "angles"),
        _dev(poses, torch.float64, "poses"),
        _dev(vol, torch.float32, "vol", (geom.nz, geom.ny, geom.nx)),
        _dev(target, torch.float32, "target", (V, geom.nv, geom.nu)),
        _dev(proj, torch.float32, "proj", (V, geom.nv, geom.nu)),
        _dev(loss, torch.float64, "loss", (V,)), _dev(grad, torch.float64, "grad", (V, 6)),
        _dev(hess, torch.float64, "hess", (V, 21)),
        C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "dp_project_fwd_ssd_gauss_newton")
    return proj, loss, grad, (hess if packed else unpack_sym6(hess))


def unpack_sym6(h21):
    """[..., 21] upper triangle (row by row) -> symmetric [..., 6, 6]."""
    import torch
    iu = torch.triu_indices(6, 6, device=h21.device)
    H = torch.zeros(h21.shape[:-1] + (6, 6), dtype=h21.dtype, device=h21.device)
    H[..., iu[0], iu[1]] = h21
    H[..., iu[1], iu[0]] = h21
    return H


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


def project_fwd_ssd_grad_pose_noalloc(geom, angles, poses, vol, target, proj=None, loss=None,
                                      grad=None, stream=None):
    """As project_fwd_ssd_grad_pose, through the entry point that allocates
    nothing (its workspace is the library's fixed device array).  Outputs are
    allocated here only when not given."""
    import torch
    V = _views(angles, poses)
    dev = vol.device
    if proj is None:
        proj = torch.empty((V, geom.nv, geom.nu), dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(V, dtype=torch.float64, device=dev)
    if grad is None:
        grad = torch.empty((V, 6), dtype=torch.float64, device=dev)
    rc = load().dp_project_fwd_ssd_grad_pose_noalloc(
        C.byref(geom_struct(geom)), V, _dev(angles, torch.float64, "angles"),
        _dev(poses, torch.float64, "poses"),
        _dev(vol, torch.float32, "vol", (geom.nz, geom.ny, geom.nx)),
        _dev(target, torch.float32, "target", (V, geom.nv, geom.nu)),
        _dev(proj, torch.float32, "proj", (V, geom.nv, geom.nu)),
        _dev(loss, torch.float64, "loss", (V,)), _dev(grad, torch.float64, "grad", (V, 6)),
        _stream(stream))
    _check(rc, "dp_project_fwd_ssd_grad_pose_noalloc")
    return proj, loss, grad


def bp_grad_flags(geom, n_views: int, ws):
    """The per-view "projected voxel by voxel in FP64" flags [V] int32 that
    the last backproject_grad_pose call left in its workspace `ws`."""
    import torch
    off = int(load().dp_bp_grad_flags_offset(C.byref(geom_struct(geom)), int(n_views)))
    if off == C.c_size_t(-1).value:
        raise ValueError("invalid geometry / view count")
    return ws[off:off + 4 * n_views].view(torch.int32)


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
# Uneven batches and kernel variants
# --------------------------------------------------------------------------

def _problems(problems, op):
    """problems: list of dicts with geom, angles, poses, vol and proj (forward),
    grad_proj + grad_pose (gradient), or target + proj + grad_pose + hess and
    optionally loss (single-pass SSD), all CUDA tensors."""
    import torch
    arr = (DPProblem * len(problems))()
    for i, q in enumerate(problems):
        g = q["geom"]
        V = _views(q["angles"], q["poses"])
        arr[i].geom = geom_struct(g)
        arr[i].n_views = V
        arr[i].angles = q["angles"].data_ptr()
        arr[i].poses = q["poses"].data_ptr()
        arr[i].vol = _dev(q["vol"], torch.float32, "vol", (g.nz, g.ny, g.nx)).value
        if op == OP_FWD:
            arr[i].proj = _dev(q["proj"], torch.float32, "proj", (V, g.nv, g.nu)).value
        elif op == OP_FWD_SSD:
            arr[i].proj = _dev(q["proj"], torch.float32, "proj", (V, g.nv, g.nu)).value
            arr[i].grad_proj = _dev(q["target"], torch.float32, "target", (V, g.nv, g.nu)).value
            arr[i].grad_pose = _dev(q["grad_pose"], torch.float64, "grad_pose", (V, 6)).value
            arr[i].hess = _dev(q["hess"], torch.float64, "hess", (V, 21)).value
            if q.get("loss") is not None:
                arr[i].loss = _dev(q["loss"], torch.float64, "loss", (V,)).value
        else:
            arr[i].grad_proj = _dev(q["grad_proj"], torch.float32, "grad_proj", (V, g.nv, g.nu)).value
            arr[i].grad_pose = _dev(q["grad_pose"], torch.float64, "grad_pose", (V, 6)).value
    return arr


def batch_workspace_bytes(problems, op) -> int:
    """Workspace for the batched entries over `problems`: batches of more than
    16 problems run as consecutive launches of 16 on one stream, which reuse
    one workspace, so this is the largest chunk's requirement (0 if invalid)."""
    lib = load()
    need = 0
    for s0 in range(0, len(problems), MAX_BATCH):
        chunk = problems[s0:s0 + MAX_BATCH]
        n = int(lib.dp_batch_workspace_bytes(_problems(chunk, op), len(chunk), op))
        if n == 0:
            return 0
        need = max(need, n)
    return need


def _run_batch(problems, op, ws, variant, stream):
    import torch
    lib = load()
    for s0 in range(0, len(problems), MAX_BATCH):
        chunk = problems[s0:s0 + MAX_BATCH]
        arr = _problems(chunk, op)
        need = int(lib.dp_batch_workspace_bytes(arr, len(chunk), op))
        if need == 0:
            raise ValueError("invalid batch")
        w = ws if ws is not None and ws.numel() >= need else torch.empty(
            need, dtype=torch.uint8, device=chunk[0]["vol"].device)
        f = {OP_FWD: lib.dp_project_fwd_batch, OP_FWD_GRAD: lib.dp_project_fwd_grad_pose_batch,
             OP_FWD_SSD: lib.dp_project_fwd_ssd_gauss_newton_batch}[op]
        _check(f(arr, len(chunk), C.c_void_p(w.data_ptr()), w.numel(), int(variant),
                 _stream(stream)), f.__name__)


def project_fwd_batch(problems, ws=None, variant=-1, stream=None):
    """Forward-project an uneven batch of problems (one launch per 16 problems);
    each problem dict supplies geom, angles, poses, vol and an output `proj`."""
    _run_batch(problems, OP_FWD, ws, variant, stream)


def project_fwd_grad_pose_batch(problems, ws=None, variant=-1, stream=None):
    """Pose gradients of an uneven batch; each problem supplies grad_proj and grad_pose."""
    _run_batch(problems, OP_FWD_GRAD, ws, variant, stream)


def project_fwd_ssd_gauss_newton_batch(problems, ws=None, variant=-1, stream=None):
    """Single-pass SSD, pose gradient and Gauss-Newton matrix of an uneven
    batch (one ray launch per 16 problems); each problem supplies geom,
    angles, poses, vol, target and the outputs proj, grad_pose, hess [V][21]
    and optionally loss [V]."""
    _run_batch(problems, OP_FWD_SSD, ws, variant, stream)


def lm_update(trial, loss, grad, hess, state, tol=1e-4, stream=None):
    """One device-side Levenberg-Marquardt update for every view (library
    kernel): trial [n][6] (in: evaluated poses, out: next trial poses), loss
    [n], grad [n][6], hess [n][21] evaluated there; state: dict of device
    tensors pose [n][6], f [n] (+inf before the first update), g [n][6],
    h [n][21], lam [n] (f64) and done [n] (int32)."""
    import torch
    n = trial.shape[0]
    f64 = torch.float64
    args = [_dev(trial, f64, "trial", (n, 6)), _dev(loss, f64, "loss", (n,)),
            _dev(grad, f64, "grad", (n, 6)), _dev(hess, f64, "hess", (n, 21)),
            _dev(state["pose"], f64, "pose", (n, 6)), _dev(state["f"], f64, "f", (n,)),
            _dev(state["g"], f64, "g", (n, 6)), _dev(state["h"], f64, "h", (n, 21)),
            _dev(state["lam"], f64, "lam", (n,)),
            _dev(state["done"], torch.int32, "done", (n,))]
    _check(load().dp_lm_update(n, *args, float(tol), _stream(stream)), "dp_lm_update")


def read_probe(buf, reps, shared, n_blocks, out=None, stream=None):
    """Streaming-read probe (measurement only): n_blocks blocks of 256 threads
    read the float32 device tensor `buf` (numel a multiple of 4).  shared=True:
    every block reads all of it `reps` times (L2-resident footprint);
    shared=False: the blocks split it (HBM streaming).  Returns the per-thread
    sums, float32 [n_blocks * 256]."""
    import torch
    if not isinstance(buf, torch.Tensor) or not buf.is_cuda or buf.dtype != torch.float32 \
            or not buf.is_contiguous() or buf.numel() % 4:
        raise ValueError("buf must be a contiguous float32 CUDA tensor with numel % 4 == 0")
    if out is None:
        out = torch.empty(n_blocks * 256, dtype=torch.float32, device=buf.device)
    out_p = _dev(out, torch.float32, "out", (n_blocks * 256,))
    _check(load().dp_read_probe(C.c_void_p(buf.data_ptr()), buf.numel() // 4, int(reps),
                                1 if shared else 0, int(n_blocks), out_p, _stream(stream)),
           "dp_read_probe")
    return out


def lds_probe(reps, n_blocks, out=None, stream=None):
    """LDS read probe (measurement only): n_blocks blocks of 256 threads each
    read reps * 8 16-byte vectors per thread from 32 KiB of LDS.  Returns the
    per-thread sums, float32 [n_blocks * 256]."""
    import torch
    if out is None:
        out = torch.empty(n_blocks * 256, dtype=torch.float32, device="cuda:0")
    out_p = _dev(out, torch.float32, "out", (n_blocks * 256,))
    _check(load().dp_lds_probe(int(reps), int(n_blocks), out_p, _stream(stream)), "dp_lds_probe")
    return out


def autotune(op, geom, angles, poses, vol, out, grad_proj=None, ws=None, reps=3, stream=None):
    """Time every kernel variant of `op` on these inputs, cache the fastest for
    this shape class and return (best, [ms per variant]).  `out` is proj (FWD,
    FWD_SSD) or grad_pose (FWD_GRAD); `grad_proj` is dL/dl (FWD_GRAD) or the
    target images (FWD_SSD)."""
    import torch
    V = _views(angles, poses)
    ws = _workspace(geom, V, op, ws, vol.device)
    best = C.c_int32()
    ms = (C.c_float * N_VARIANTS)()
    gp = C.c_void_p(grad_proj.data_ptr()) if grad_proj is not None else None
    rc = load().dp_autotune(int(op), C.byref(geom_struct(geom)), V,
                            C.c_void_p(angles.data_ptr()), C.c_void_p(poses.data_ptr()),
                            _dev(vol, torch.float32, "vol"), gp, C.c_void_p(out.data_ptr()),
                            C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream), int(reps),
                            C.byref(best), ms)
    _check(rc, "dp_autotune")
    return best.value, list(ms)


def fp_project(geom, angles, poses, vol, kind="sf", out=None, ws=None, stream=None):
    """Footprint-projector DRRs [V][nv][nu] f32; kind "sf" (separable
    footprint) or "dd" (distance-driven).  FP32 atomic accumulation."""
    import torch
    V = _views(angles, poses)
    if out is None:
        out = torch.empty((V, geom.nv, geom.nu), dtype=torch.float32, device=vol.device)
    ws = _workspace(geom, V, OP_FP_FWD, ws, vol.device)
    rc = load().dp_fp_project(C.byref(geom_struct(geom)), V, _dev(angles, torch.float64, "angles"),
                              _dev(poses, torch.float64, "poses"),
                              _dev(vol, torch.float32, "vol", (geom.nz, geom.ny, geom.nx)),
                              _dev(out, torch.float32, "out", (V, geom.nv, geom.nu)), FP_KINDS[kind],
                              C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "dp_fp_project")
    return out


def fp_backproject(geom, angles, poses, proj, kind="sf", out=None, ws=None, stream=None):
    """Footprint back-projection [nz][ny][nx] f32 (the transpose of fp_project)."""
    import torch
    V = _views(angles, poses)
    if out is None:
        out = torch.empty((geom.nz, geom.ny, geom.nx), dtype=torch.float32, device=proj.device)
    ws = _workspace(geom, V, OP_FP_BP, ws, proj.device)
    rc = load().dp_fp_backproject(C.byref(geom_struct(geom)), V, _dev(angles, torch.float64, "angles"),
                                  _dev(poses, torch.float64, "poses"),
                                  _dev(proj, torch.float32, "proj", (V, geom.nv, geom.nu)),
                                  _dev(out, torch.float32, "out", (geom.nz, geom.ny, geom.nx)),
                                  FP_KINDS[kind], C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "dp_fp_backproject")
    return out


def fp_project_grad_pose(geom, angles, poses, vol, grad_proj, kind="sf", out=None, ws=None,
                         stream=None):
    import torch
    V = _views(angles, poses)
    if out is None:
        out = torch.empty((V, 6), dtype=torch.float64, device=vol.device)
    ws = _workspace(geom, V, OP_FP_FWD_GRAD, ws, vol.device)
    rc = load().dp_fp_project_grad_pose(
        C.byref(geom_struct(geom)), V, _dev(angles, torch.float64, "angles"),
        _dev(poses, torch.float64, "poses"), _dev(vol, torch.float32, "vol", (geom.nz, geom.ny, geom.nx)),
        _dev(grad_proj, torch.float32, "grad_proj", (V, geom.nv, geom.nu)),
        _dev(out, torch.float64, "out", (V, 6)), FP_KINDS[kind], C.c_void_p(ws.data_ptr()), ws.numel(),
        _stream(stream))
    _check(rc, "dp_fp_project_grad_pose")
    return out


def fp_backproject_grad_pose(geom, angles, poses, proj, grad_vol, kind="sf", out=None, ws=None,
                             stream=None):
    import torch
    V = _views(angles, poses)
    if out is None:
        out = torch.empty((V, 6), dtype=torch.float64, device=proj.device)
    ws = _workspace(geom, V, OP_FP_BP_GRAD, ws, proj.device)
    rc = load().dp_fp_backproject_grad_pose(
        C.byref(geom_struct(geom)), V, _dev(angles, torch.float64, "angles"),
        _dev(poses, torch.float64, "poses"), _dev(proj, torch.float32, "proj", (V, geom.nv, geom.nu)),
        _dev(grad_vol, torch.float32, "grad_vol", (geom.nz, geom.ny, geom.nx)),
        _dev(out, torch.float64, "out", (V, 6)), FP_KINDS[kind], C.c_void_p(ws.data_ptr()), ws.numel(),
        _stream(stream))
    _check(rc, "dp_fp_backproject_grad_pose")
    return out


def fdk_filter(geom, proj, scale, out=None, stream=None):
    """FDK pre-filtered projections (cosine weight, ramp along u, times scale);
    scale = pi / V for V views over a full circle."""
    import torch
    V = proj.shape[0]
    if out is None:
        out = torch.empty_like(proj)
    rc = load().dp_fdk_filter(C.byref(geom_struct(geom)), V,
                              _dev(proj, torch.float32, "proj", (V, geom.nv, geom.nu)),
                              _dev(out, torch.float32, "out", (V, geom.nv, geom.nu)),
                              float(scale), _stream(stream))
    _check(rc, "dp_fdk_filter")
    return out


def sharpness(vol, grad=True, ws=None, stream=None):
    """(S, dS/dvol): S a 0-d FP64 device tensor, dS/dvol FP32 like vol (or None)."""
    import torch
    nz, ny, nx = vol.shape
    need = load().dp_sharpness_workspace_bytes(nx, ny, nz)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=vol.device)
    loss = torch.empty((), dtype=torch.float64, device=vol.device)
    g = torch.empty_like(vol) if grad else None
    rc = load().dp_sharpness(nx, ny, nz, _dev(vol, torch.float32, "vol"), C.c_void_p(loss.data_ptr()),
                             C.c_void_p(g.data_ptr()) if grad else None,
                             C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "dp_sharpness")
    return loss, g


def gradient_entropy(vol, grad=True, eps=1e-12, ws=None, stream=None):
    """(GE, dGE/dvol): GE a 0-d FP64 device tensor, dGE/dvol FP32 like vol (or None)."""
    import torch
    nz, ny, nx = vol.shape
    need = load().dp_gradient_entropy_workspace_bytes(nx, ny, nz)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=vol.device)
    loss = torch.empty((), dtype=torch.float64, device=vol.device)
    g = torch.empty_like(vol) if grad else None
    rc = load().dp_gradient_entropy(nx, ny, nz, _dev(vol, torch.float32, "vol"), float(eps),
                                    C.c_void_p(loss.data_ptr()),
                                    C.c_void_p(g.data_ptr()) if grad else None,
                                    C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "dp_gradient_entropy")
    return loss, g


def set_variant(op, variant):
    _check(load().dp_set_variant(int(op), int(variant)), "dp_set_variant")


def get_variant(geom, n_views, op) -> int:
    return int(load().dp_get_variant(C.byref(geom_struct(geom)), int(n_views), int(op)))


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
