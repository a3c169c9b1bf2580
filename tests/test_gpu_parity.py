"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: projections and back-projected volumes max|gpu - ref| <=
1e-5 max|ref|; pose gradients per view ||gpu - ref|| <= 1e-4 ||ref||,
separately for the translation and the rotation triplet (views whose
reference norm is below 1e-6 of the largest view are compared against
that largest norm).  Inputs are seeded and identical on both sides.
"""
import math
import sys

import numpy as np
import pytest
import torch

import synth
from synth import Geom

pytestmark = pytest.mark.gpu

PROJ_TOL = 1e-5
GRAD_TOL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dt):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")


def f64(a):
    return dev(a, torch.float64)


def f32(a):
    return dev(a, torch.float32)


def check_values(name, got, ref, tol=PROJ_TOL):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / (scale if scale > 0 else 1.0)
    say(f"{name}: max rel err {err:.3e} (scale {scale:.3e})")
    if scale == 0:
        assert np.abs(got).max() == 0.0
    assert err <= tol, (name, err)


def check_grads(name, got, ref, tol=GRAD_TOL):
    got, ref = np.asarray(got).reshape(-1, 6), np.asarray(ref).reshape(-1, 6)
    worst = 0.0
    for sl in (slice(0, 3), slice(3, 6)):
        nr = np.linalg.norm(ref[:, sl], axis=1)
        floor = 1e-6 * nr.max()
        denom = np.where(nr < floor, nr.max(), nr)
        denom = np.where(denom > 0, denom, 1.0)
        e = np.linalg.norm(got[:, sl] - ref[:, sl], axis=1) / denom
        worst = max(worst, float(e.max()))
    say(f"{name}: worst per-view rel err {worst:.3e}")
    assert worst <= tol, (name, worst)


# ---------------------------------------------------------------------------
# Forward projector + pose gradient
# ---------------------------------------------------------------------------

def _fwd_case(dp, oracle, g, vol, angles, poses, w=None, name="fwd"):
    say(f"case {name}: vol {vol.shape} det {g.nv}x{g.nu} V={len(angles)}")
    l_gpu = dp.project_fwd(g, f64(angles), f64(poses), f32(vol)).cpu().numpy()
    l_ref = oracle.project_fwd(g, angles, poses, vol)
    check_values(f"{name} project_fwd", l_gpu, l_ref)
    if w is None:
        w = np.random.default_rng(7).standard_normal(l_ref.shape).astype(np.float32)
    g_gpu = dp.project_fwd_grad_pose(g, f64(angles), f64(poses), f32(vol), f32(w)).cpu().numpy()
    g_ref = oracle.project_fwd_grad_pose(g, angles, poses, vol, w)
    check_grads(f"{name} project_fwd_grad_pose", g_gpu, g_ref)
    return l_gpu, g_gpu


def test_config1_forward_and_ssd_gradient(dp, oracle):
    """Config 1: 64^3 at 1 mm, one 128x128 view, SSD to a target DRR at a second pose."""
    c = synth.config1_inputs()
    g = c["geom"]
    y = oracle.project_fwd(g, c["angles"], c["target_pose"], c["vol"])
    l_ref = oracle.project_fwd(g, c["angles"], c["poses"], c["vol"])
    w = (2.0 * (l_ref - y)).astype(np.float32)
    _fwd_case(dp, oracle, g, c["vol"], c["angles"], c["poses"], w, "config1")


def test_ragged_anisotropic_multiview(dp, oracle):
    rng = synth.rng_for(200)
    g = Geom(37, 29, 23, 1.3, 1.1, 1.7, 45, 27, 1.9, 2.3, off_u=1.25, off_v=-0.75)
    vol = rng.uniform(0, 0.05, g.vol_shape).astype(np.float32)
    V = 5
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 8.0, 15.0, rng)
    _fwd_case(dp, oracle, g, vol, angles, poses, name="ragged")


def test_forward_source_inside_volume(dp, oracle):
    """Source inside the volume: every ray starts inside it (the march begins
    at the source) and the chunk boxes start at the source."""
    rng = synth.rng_for(206)
    g = Geom(24, 24, 24, 2.0, 2.0, 2.0, 40, 36, 2.0, 2.0, sad=20.0, sdd=40.0)
    vol = rng.uniform(0, 0.05, g.vol_shape).astype(np.float32)
    V = 3
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 2.0, 20.0, rng)
    _fwd_case(dp, oracle, g, vol, angles, poses, name="source-inside")


def test_edges_boundary_content_and_large_rotations(dp, oracle):
    """Content on the volume faces (zero-extension and gradient masking),
    quarter-turn and large rotations, rays grazing the volume."""
    rng = synth.rng_for(201)
    g = Geom(20, 20, 20, 2.0, 2.0, 2.0, 40, 36, 2.5, 2.5)
    vol = rng.uniform(0.0, 1.0, g.vol_shape).astype(np.float32)
    angles = np.array([0.0, 0.5 * math.pi, 1.0, 4.0])
    poses = np.array([[0, 0, 0, 0.5 * math.pi, 0, 0],
                      [3.0, -4.0, 2.0, 0.0, 0.5 * math.pi, 0.5 * math.pi],
                      [25.0, -20.0, 10.0, 0.7, -1.2, 2.5],
                      [0.0, 0.0, 0.0, -2.0, 0.3, -3.0]])
    _fwd_case(dp, oracle, g, vol, angles, poses, name="edges")


def test_rays_missing_the_volume_give_zero(dp, oracle):
    g = Geom(8, 8, 8, 1.0, 1.0, 1.0, 17, 13, 1.0, 1.0)
    vol = np.ones(g.vol_shape, np.float32)
    poses = np.array([[0.0, 300.0, 0.0, 0, 0, 0]])  # moved out of the field of view
    l_gpu = dp.project_fwd(g, f64([0.0]), f64(poses), f32(vol)).cpu().numpy()
    assert np.all(l_gpu == 0.0)
    w = np.ones((1, 13, 17), np.float32)
    gg = dp.project_fwd_grad_pose(g, f64([0.0]), f64(poses), f32(vol), f32(w)).cpu().numpy()
    assert np.all(gg == 0.0)


def test_tiny_sizes(dp, oracle):
    rng = synth.rng_for(202)
    g = Geom(1, 1, 1, 3.0, 3.0, 3.0, 1, 1, 2.0, 2.0)
    vol = np.array([[[0.7]]], np.float32)
    _fwd_case(dp, oracle, g, vol, np.array([0.2]), np.array([[0.3, -0.2, 0.1, 0.01, 0.02, -0.03]]),
              w=np.ones((1, 1, 1), np.float32), name="1x1x1")
    g = Geom(3, 2, 4, 1.0, 1.5, 0.8, 3, 2, 1.0, 1.0)
    vol = rng.uniform(0, 1, g.vol_shape).astype(np.float32)
    _fwd_case(dp, oracle, g, vol, np.array([1.0, 2.0]), synth.random_poses(2, 0.5, 5, rng), name="tiny")


def test_config2_full_size_sampled(dp, oracle):
    """Config 2 at full size (256^3, 64 poses, 512x512) in the launch shape
    the benchmark times: sampled rays against the oracle one by one, and
    the gradient for a dL/dl that is non-zero on a random ray subset."""
    c = synth.config2_inputs()
    g, vol, angles, poses = c["geom"], c["vol"], c["angles"], c["poses"]
    V = len(angles)
    l_gpu = dp.project_fwd(g, f64(angles), f64(poses), f32(vol)).cpu().numpy()
    rng = np.random.default_rng(11)
    npix = g.nu * g.nv
    ids = rng.choice(V * npix, 4000, replace=False)
    ref = oracle.project_fwd_rays(g, angles, poses, vol, ids)
    got = l_gpu.reshape(-1)[ids]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"config2 sampled project_fwd: max rel err {err:.3e}")
    assert err <= PROJ_TOL
    w = np.zeros((V, g.nv, g.nu), np.float32)
    for v in range(V):
        sel = rng.choice(npix, 64, replace=False)
        w[v].reshape(-1)[sel] = rng.standard_normal(64).astype(np.float32)
    g_gpu = dp.project_fwd_grad_pose(g, f64(angles), f64(poses), f32(vol), f32(w)).cpu().numpy()
    g_ref = oracle.project_fwd_grad_pose(g, angles, poses, vol, w)
    check_grads("config2 sparse-w project_fwd_grad_pose", g_gpu, g_ref)


# ---------------------------------------------------------------------------
# Back-projector + pose gradient
# ---------------------------------------------------------------------------

def _bp_case(dp, oracle, g, proj, angles, poses, mode, e=None, name="bp"):
    """Back-projection and its pose gradient against the oracle; returns the
    per-view flags of columns projected voxel by voxel in FP64."""
    say(f"case {name}: vol {g.vol_shape} det {g.nv}x{g.nu} V={len(angles)} mode={mode}")
    b_gpu = dp.backproject(g, f64(angles), f64(poses), f32(proj), mode).cpu().numpy()
    b_ref = oracle.backproject(g, angles, poses, proj, mode)
    check_values(f"{name} backproject", b_gpu, b_ref)
    if e is None:
        e = np.random.default_rng(8).standard_normal(g.vol_shape).astype(np.float32)
    V = len(angles)
    ws = torch.empty(dp.workspace_bytes(g, V, dp.OP_BP_GRAD), dtype=torch.uint8, device="cuda:0")
    g_gpu = dp.backproject_grad_pose(g, f64(angles), f64(poses), f32(proj), f32(e), mode,
                                     ws=ws).cpu().numpy()
    g_ref = oracle.backproject_grad_pose(g, angles, poses, proj, e, mode)
    check_grads(f"{name} backproject_grad_pose", g_gpu, g_ref)
    return dp.bp_grad_flags(g, V, ws).cpu().numpy()


@pytest.mark.parametrize("mode", [0, 1])
def test_backproject_ragged(dp, oracle, mode):
    rng = synth.rng_for(203)
    g = Geom(70, 9, 37, 1.5, 1.2, 1.1, 61, 47, 1.6, 1.4, off_u=-2.5, off_v=1.5)
    V = 7
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 6.0, 8.0, rng)
    proj = synth.smooth_images(V, g.nv, g.nu, rng, signed=True)
    _bp_case(dp, oracle, g, proj, angles, poses, mode, name=f"bp-ragged-{mode}")


def _stage_split(oracle, g, angles, poses, K=32, B=16, cap=640, pad=2):
    """(staged, gathered): how many (view, gradient block) pairs have a
    detector rectangle that fits the back-projection gradient's LDS stage
    (cap padded pixels) under its rule: the window-clamped projections of the
    block region's 8 corner voxels, a 1e-3 pixel margin, every corner at
    least 1 mm in front of the source.  Host arithmetic on the oracle's
    projection matrices; it shows which paths a geometry exercises."""
    NU, NV = g.nu + 2 * pad, g.nv + 2 * pad
    staged = gathered = 0
    size = np.array([g.nx, g.ny, g.nz])
    h = np.array([g.vx, g.vy, g.vz])
    for beta, pose in zip(angles, poses):
        P = oracle.projection_matrix(g, beta)
        R = oracle.rotation(pose[3:])
        for bz in range(-(-g.nz // K)):
            for by in range(-(-g.ny // B)):
                for bx in range(-(-g.nx // B)):
                    c = np.stack(np.meshgrid([bx * B, bx * B + B - 1], [by * B, by * B + B - 1],
                                             [bz * K, bz * K + K - 1], indexing="ij"), -1)
                    p = (c.reshape(-1, 3) - 0.5 * (size - 1)) * h
                    uvw = (p @ R.T + pose[:3]) @ P[:, :3].T + P[:, 3]
                    if not (uvw[:, 2] >= 1.0).all():
                        gathered += 1
                        continue
                    a = np.clip(uvw[:, 0] / uvw[:, 2] + pad, pad - 1.5, g.nu + pad + 0.5)
                    b = np.clip(uvw[:, 1] / uvw[:, 2] + pad, pad - 1.5, g.nv + pad + 0.5)
                    w = min(NU - 1, math.floor(a.max() + 1e-3) + 1) - max(0, math.floor(a.min() - 1e-3)) + 1
                    ht = min(NV - 1, math.floor(b.max() + 1e-3) + 1) - max(0, math.floor(b.min() - 1e-3)) + 1
                    if w * ht <= cap:
                        staged += 1
                    else:
                        gathered += 1
    return staged, gathered


@pytest.mark.parametrize("mode", [0, 1])
def test_backproject_gradient_staged_and_gathered_blocks(dp, oracle, mode):
    """The back-projection gradient stages each block's detector rectangle in
    LDS when it fits and gathers its taps from global memory otherwise;
    with 1.2 x 2.0 mm pixels over 1 mm voxels both happen around the circle
    (counted on the host), and the sums match the oracle either way."""
    rng = synth.rng_for(216)
    g = Geom(64, 48, 40, 1.0, 1.0, 1.0, 96, 40, 1.2, 2.0, off_u=0.5)
    V = 8
    angles = synth.circular_angles(V)
    poses = synth.random_poses(V, 3.0, 4.0, rng)
    staged, gathered = _stage_split(oracle, g, angles, poses)
    say(f"gradient blocks: {staged} staged, {gathered} gathered")
    assert staged > 0 and gathered > 0
    proj = synth.smooth_images(V, g.nv, g.nu, rng, signed=True)
    _bp_case(dp, oracle, g, proj, angles, poses, mode, name=f"bp-stage-{mode}")


@pytest.mark.parametrize("mode", [0, 1])
def test_backproject_volume_larger_than_field_of_view(dp, oracle, mode):
    """Voxels projecting outside the detector (zero extension of l and dl)."""
    rng = synth.rng_for(204)
    g = Geom(48, 40, 33, 3.0, 3.0, 3.0, 30, 20, 2.0, 2.0)
    V = 4
    angles = synth.circular_angles(V)
    poses = synth.random_poses(V, 10.0, 20.0, rng)
    proj = rng.standard_normal((V, g.nv, g.nu)).astype(np.float32)
    _bp_case(dp, oracle, g, proj, angles, poses, mode, name=f"bp-fov-{mode}")


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tilt_deg", [3.0, 40.0])
def test_backproject_source_inside_volume(dp, oracle, mode, tilt_deg):
    """Source inside the volume: voxels at or behind it get no ray.  With small
    rotations whole voxel columns lie within 1 mm of the source plane (no
    usable anchor); with large ones columns cross that plane (voxels on both
    sides of the source in one column)."""
    rng = synth.rng_for(205)
    g = Geom(24, 24, 24, 2.0, 2.0, 2.0, 40, 36, 2.0, 2.0, sad=20.0, sdd=40.0)
    V = 3
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 2.0, tilt_deg, rng)
    proj = synth.smooth_images(V, g.nv, g.nu, rng, signed=True)
    flags = _bp_case(dp, oracle, g, proj, angles, poses, mode,
                     name=f"bp-source-inside-{mode}-tilt{tilt_deg:g}")
    say(f"FP64 per-voxel views: {flags.tolist()}")
    if tilt_deg == 3.0:
        # whole columns within 1 mm of the source plane: the FP64 pass ran
        assert flags.any()


@pytest.mark.parametrize("mode", [0, 1])
def test_backproject_source_inside_volume_config_detector(dp, oracle, mode):
    """Source inside the volume with a config-scale detector (SDD 1500 mm,
    0.776 mm pixels, S / du ~ 1900): columns passing close to the source
    plane have middle voxels projecting tens of thousands of pixels off the
    detector while their other voxels land on it; those columns go to the
    FP64 per-voxel pass (anchor limit of a few detector widths)."""
    rng = synth.rng_for(207)
    g = Geom(24, 24, 24, 2.0, 2.0, 2.0, 96, 80, 0.776, 0.776, sad=20.0, sdd=1500.0)
    V = 3
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 2.0, 3.0, rng)
    proj = synth.smooth_images(V, g.nv, g.nu, rng, signed=True)
    flags = _bp_case(dp, oracle, g, proj, angles, poses, mode, name=f"bp-source-inside-c3det-{mode}")
    say(f"FP64 per-voxel views: {flags.tolist()}")
    assert flags.any()


def test_backproject_tiny(dp, oracle):
    g = Geom(1, 1, 1, 1.0, 1.0, 1.0, 2, 1, 1.0, 1.0)
    proj = np.array([[[0.5, 1.5]]], np.float32)
    _bp_case(dp, oracle, g, proj, np.array([0.0]), np.zeros((1, 6)), 1,
             e=np.ones((1, 1, 1), np.float32), name="bp-tiny")


def test_config3_full_size_sampled(dp, oracle):
    """Config 3 sizes (512^3 recon, 360 views of 512x384, FDK weight, per-view
    sinusoidal motion) in the benchmark's launch shape: sampled voxels one by
    one, and the gradient for a dL/dmu that is non-zero on a voxel subset."""
    g = synth.geom_c3_recon()
    m = synth.config3_motion()
    angles, poses = m["angles"], m["poses"]
    V = len(angles)
    rng = np.random.default_rng(12)
    proj = synth.smooth_images(V, g.nv, g.nu, rng, n_blobs=4, signed=True)
    b_gpu = dp.backproject(g, f64(angles), f64(poses), f32(proj), 1).cpu().numpy()
    nvox = g.nx * g.ny * g.nz
    ids = rng.choice(nvox, 3000, replace=False)
    ref = oracle.backproject_voxels(g, angles, poses, proj, ids, 1)
    got = b_gpu.reshape(-1)[ids]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"config3 sampled backproject: max rel err {err:.3e}")
    assert err <= PROJ_TOL
    del b_gpu
    e = np.zeros(g.vol_shape, np.float32)
    sel = rng.choice(nvox, 3000, replace=False)
    e.reshape(-1)[sel] = rng.standard_normal(3000).astype(np.float32)
    g_gpu = dp.backproject_grad_pose(g, f64(angles), f64(poses), f32(proj), f32(e), 1).cpu().numpy()
    g_ref = oracle.backproject_grad_pose(g, angles, poses, proj, e, 1)
    check_grads("config3 sparse-e backproject_grad_pose", g_gpu, g_ref)


# ---------------------------------------------------------------------------
# Determinism and API behaviour on the device
# ---------------------------------------------------------------------------

def test_bitwise_repeatable(dp, oracle):
    rng = synth.rng_for(205)
    g = Geom(40, 40, 40, 1.0, 1.0, 1.0, 64, 48, 1.5, 1.5)
    vol = synth.ellipsoid_phantom(40, 1.0, 6, rng)
    V = 3
    angles, poses = rng.uniform(0, 6, V), synth.random_poses(V, 5, 5, rng)
    w = rng.standard_normal((V, g.nv, g.nu)).astype(np.float32)
    proj = synth.smooth_images(V, g.nv, g.nu, rng, signed=True)
    e = rng.standard_normal(g.vol_shape).astype(np.float32)
    outs = []
    for _ in range(2):
        outs.append((dp.project_fwd(g, f64(angles), f64(poses), f32(vol)).cpu().numpy(),
                     dp.project_fwd_grad_pose(g, f64(angles), f64(poses), f32(vol), f32(w)).cpu().numpy(),
                     dp.backproject(g, f64(angles), f64(poses), f32(proj), 1).cpu().numpy(),
                     dp.backproject_grad_pose(g, f64(angles), f64(poses), f32(proj), f32(e), 1).cpu().numpy()))
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


def test_non_default_stream_and_outputs_overwritten(dp, oracle):
    rng = synth.rng_for(206)
    g = Geom(16, 16, 16, 2.0, 2.0, 2.0, 24, 24, 3.0, 3.0)
    vol = rng.uniform(0, 1, g.vol_shape).astype(np.float32)
    angles, poses = np.array([0.4]), synth.random_poses(1, 3, 3, rng)
    s = torch.cuda.Stream()
    out = torch.full((1, 24, 24), 123.0, device="cuda:0")
    with torch.cuda.stream(s):
        dp.project_fwd(g, f64(angles), f64(poses), f32(vol), out=out, stream=s)
    s.synchronize()
    ref = oracle.project_fwd(g, angles, poses, vol)
    check_values("stream project_fwd", out.cpu().numpy(), ref)


def test_config3_dense_sharpness_gradient(dp, oracle):
    """Config 3 sizes and launch (512^3 recon, all 360 views of 512x384, FDK
    weight, sinusoidal motion) with a dense dL/dmu: the gradient of the
    image-sharpness loss (negative sum of squared forward differences, the
    oracle's own) of a 512^3 ellipsoid volume with noise, non-zero on every
    voxel.  The pose gradient of each view depends only on that view's image
    and dL/dmu, so the oracle evaluates 12 of the 360 views (every 30th) and
    the GPU's values for those views are compared (<= 1e-4)."""
    from oracle import fdk
    g = synth.geom_c3_recon()
    m = synth.config3_motion()
    angles, poses = m["angles"], m["poses"]
    V = len(angles)
    rng = np.random.default_rng(19)
    proj = synth.smooth_images(V, g.nv, g.nu, rng, n_blobs=4, signed=True)
    vol = synth.ellipsoid_phantom(g.nx, g.vx, 20, rng).astype(np.float64)
    vol += rng.normal(0.0, 1e-3, vol.shape)
    e = fdk.sharpness_grad(vol).astype(np.float32)
    del vol
    assert np.count_nonzero(e) > 0.99 * e.size
    say(f"config3 dense-e: |e| max {np.abs(e).max():.3e}")
    g_gpu = dp.backproject_grad_pose(g, f64(angles), f64(poses), f32(proj), f32(e), 1).cpu().numpy()
    sub = np.arange(0, V, 30)
    g_ref = oracle.backproject_grad_pose(g, angles[sub], poses[sub], proj[sub], e, 1)
    check_grads("config3 dense-e backproject_grad_pose", g_gpu[sub], g_ref)
