"""GPU parity of the footprint projector pairs (separable footprint and
distance-driven) and their pose gradients against the FP64 oracle (same bars
as the ray/voxel pair: projections and volumes max|gpu - ref| <= 1e-5
max|ref|; pose gradients per view and triplet <= 1e-4)."""
import math

import numpy as np
import pytest
import torch

import synth
from synth import Geom
from test_gpu_parity import check_grads, check_values, f32, f64, say

pytestmark = pytest.mark.gpu


def _case(seed, g, V, t_mm=6.0, r_deg=8.0, smooth=True):
    rng = synth.rng_for(seed)
    if smooth:
        n = max(g.nx, g.ny, g.nz)
        vol = synth.ellipsoid_phantom(n, min(g.vx, g.vy, g.vz), 8, rng)[:g.nz, :g.ny, :g.nx].copy()
    else:
        vol = rng.uniform(0, 0.05, g.vol_shape).astype(np.float32)
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, t_mm, r_deg, rng)
    return rng, vol, angles, poses


CASES = {
    "ragged": (Geom(37, 29, 23, 1.3, 1.1, 1.7, 45, 27, 1.9, 2.3, off_u=1.25, off_v=-0.75), 4),
    "fine-detector": (Geom(24, 24, 24, 2.0, 2.0, 2.0, 80, 72, 1.0, 1.0), 3),
    "tiny": (Geom(3, 2, 4, 1.0, 1.5, 0.8, 5, 4, 1.0, 1.0), 2),
    # source inside the volume: voxels at or behind the source plane are
    # skipped, columns anchored within 1 mm of it take the per-voxel FP64
    # footprint, and voxels just in front of it have footprints far wider
    # than the detector
    "source-inside": (Geom(24, 24, 24, 2.0, 2.0, 2.0, 40, 36, 2.0, 2.0, sad=20.0, sdd=40.0), 3),
    # the same with large rotations: voxel columns cross the source plane
    "source-inside-tilted": (Geom(24, 24, 24, 2.0, 2.0, 2.0, 40, 36, 2.0, 2.0, sad=20.0, sdd=40.0), 3),
}
TILT_DEG = {"source-inside-tilted": 40.0}


@pytest.mark.parametrize("kind", ["sf", "dd"])
@pytest.mark.parametrize("name", list(CASES))
def test_footprint_pair_and_gradients_match_oracle(dp, oracle, name, kind):
    g, V = CASES[name]
    rng, vol, angles, poses = _case(700 + len(name), g, V, r_deg=TILT_DEG.get(name, 8.0),
                                    smooth=name != "tiny")
    say(f"{kind} case {name}: vol {vol.shape} det {g.nv}x{g.nu} V={V}")
    a, p = f64(angles), f64(poses)
    l = dp.fp_project(g, a, p, f32(vol), kind).cpu().numpy()
    l_ref = oracle.fp_project(g, angles, poses, vol, kind)
    check_values(f"{name} {kind} project", l, l_ref)
    img = rng.standard_normal((V, g.nv, g.nu)).astype(np.float32)
    b = dp.fp_backproject(g, a, p, f32(img), kind).cpu().numpy()
    b_ref = oracle.fp_backproject(g, angles, poses, img, kind)
    check_values(f"{name} {kind} backproject", b, b_ref)
    w = rng.standard_normal((V, g.nv, g.nu)).astype(np.float32)
    gp = dp.fp_project_grad_pose(g, a, p, f32(vol), f32(w), kind).cpu().numpy()
    check_grads(f"{name} {kind} project_grad_pose", gp,
                oracle.fp_project_grad_pose(g, angles, poses, vol, w, kind))
    proj = synth.smooth_images(V, g.nv, g.nu, rng, n_blobs=3).astype(np.float32)
    e = rng.standard_normal(g.vol_shape).astype(np.float32)
    gb = dp.fp_backproject_grad_pose(g, a, p, f32(proj), f32(e), kind).cpu().numpy()
    check_grads(f"{name} {kind} backproject_grad_pose", gb,
                oracle.fp_backproject_grad_pose(g, angles, poses, proj, e, kind))


@pytest.mark.parametrize("kind", ["sf", "dd"])
def test_footprint_pair_is_adjoint_on_the_gpu(dp, kind):
    g, V = CASES["ragged"]
    rng, vol, angles, poses = _case(710, g, V, smooth=False)
    a, p = f64(angles), f64(poses)
    x = torch.tensor(rng.standard_normal(g.vol_shape), dtype=torch.float32, device="cuda:0")
    y = torch.tensor(rng.standard_normal((V, g.nv, g.nu)), dtype=torch.float32, device="cuda:0")
    lhs = float((dp.fp_project(g, a, p, x, kind).double() * y.double()).sum())
    rhs = float((x.double() * dp.fp_backproject(g, a, p, y, kind).double()).sum())
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("kind", ["sf", "dd"])
def test_footprint_projection_at_scale(dp, oracle, kind):
    """A 128^3 volume and 256^2 detector, 4 views: the full projection
    against the oracle."""
    g = Geom(128, 128, 128, 1.5, 1.5, 1.5, 256, 256, 1.2, 1.2)
    rng, vol, angles, poses = _case(720, g, 4)
    l = dp.fp_project(g, f64(angles), f64(poses), f32(vol), kind).cpu().numpy()
    check_values(f"128^3 {kind} project", l, oracle.fp_project(g, angles, poses, vol, kind))


def test_unknown_footprint_kind_is_rejected(dp):
    import ctypes as C
    g = CASES["tiny"][0]
    lib = dp.load()
    p = C.c_void_p(1 << 20)
    ws = C.c_void_p(1 << 24)
    rc = lib.dp_fp_project(C.byref(dp.geom_struct(g)), 1, p, p, p, p, 7, ws,
                           dp.workspace_bytes(g, 1, dp.OP_FP_FWD), None)
    assert rc == -1 and b"kind" in lib.dp_last_error()
