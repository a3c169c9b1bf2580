"""GPU parity of the fused forward + SSD + pose-gradient entry
(dp_project_fwd_ssd_grad_pose) against the FP64 oracle: projections
max|gpu - ref| <= 1e-5 max|ref|; per-view SSD within 1e-5 relative; pose
gradients per view and triplet within 1e-4, the oracle's gradient taken
with dL/dl = 2 (l_ref - y).  Targets are rendered at other poses, so the
residuals are of the order of l itself."""
import math

import numpy as np
import pytest
import torch

import synth
from paper_2508_13304_amd import N_VARIANTS
from synth import Geom
from test_gpu_parity import check_grads, check_values, f32, f64, say

pytestmark = pytest.mark.gpu


def _fused_case(dp, oracle, g, vol, angles, poses, y, name, variant=None):
    say(f"fused case {name}: vol {vol.shape} det {g.nv}x{g.nu} V={len(angles)}")
    if variant is not None:
        dp.set_variant(dp.OP_FWD_SSD, variant)
    try:
        l, loss, gp = dp.project_fwd_ssd_grad_pose(g, f64(angles), f64(poses), f32(vol), f32(y))
    finally:
        if variant is not None:
            dp.set_variant(dp.OP_FWD_SSD, -1)
    l_ref = oracle.project_fwd(g, angles, poses, vol)
    check_values(f"{name} fused proj", l.cpu().numpy(), l_ref)
    r = l_ref - y
    loss_ref = (r * r).reshape(len(angles), -1).sum(1)
    rel = np.abs(loss.cpu().numpy() - loss_ref) / np.maximum(loss_ref, 1e-30)
    say(f"{name} fused loss: max rel err {rel.max():.3e}")
    assert rel.max() <= 1e-5
    g_ref = oracle.project_fwd_grad_pose(g, angles, poses, vol, (2.0 * r).astype(np.float32))
    check_grads(f"{name} fused grad", gp.cpu().numpy(), g_ref)


def test_fused_config1(dp, oracle):
    c = synth.config1_inputs()
    g = c["geom"]
    y = oracle.project_fwd(g, c["angles"], c["target_pose"], c["vol"]).astype(np.float32)
    _fused_case(dp, oracle, g, c["vol"], c["angles"], c["poses"], y, "config1")


@pytest.mark.parametrize("variant", range(N_VARIANTS))
def test_fused_ragged_multiview_every_variant(dp, oracle, variant):
    rng = synth.rng_for(210)
    g = Geom(37, 29, 23, 1.3, 1.1, 1.7, 45, 27, 1.9, 2.3, off_u=1.25, off_v=-0.75)
    vol = rng.uniform(0, 0.05, g.vol_shape).astype(np.float32)
    V = 5
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 8.0, 15.0, rng)
    y = oracle.project_fwd(g, angles, synth.random_poses(V, 8.0, 15.0, rng), vol).astype(np.float32)
    _fused_case(dp, oracle, g, vol, angles, poses, y, f"ragged-v{variant}", variant)


def test_fused_edges_and_misses(dp, oracle):
    """Content on the faces, large rotations, and a view that misses the
    volume entirely (l = 0, loss = sum y^2, zero gradient)."""
    rng = synth.rng_for(211)
    g = Geom(20, 20, 20, 2.0, 2.0, 2.0, 40, 36, 2.5, 2.5)
    vol = rng.uniform(0.0, 1.0, g.vol_shape).astype(np.float32)
    angles = np.array([0.0, 0.5 * math.pi, 1.0])
    poses = np.array([[0, 0, 0, 0.5 * math.pi, 0, 0],
                      [25.0, -20.0, 10.0, 0.7, -1.2, 2.5],
                      [0.0, 400.0, 0.0, 0, 0, 0]])
    y = rng.uniform(0.0, 5.0, (3, 36, 40)).astype(np.float32)
    _fused_case(dp, oracle, g, vol, angles, poses, y, "edges")
    l, loss, gp = dp.project_fwd_ssd_grad_pose(g, f64(angles), f64(poses), f32(vol), f32(y))
    assert torch.all(l[2] == 0) and torch.all(gp[2] == 0)


def test_fused_source_inside_volume(dp, oracle):
    """Single-pass SSD with the source inside the volume (rays start inside)."""
    rng = synth.rng_for(207)
    g = Geom(24, 24, 24, 2.0, 2.0, 2.0, 40, 36, 2.0, 2.0, sad=20.0, sdd=40.0)
    vol = rng.uniform(0, 0.05, g.vol_shape).astype(np.float32)
    V = 3
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 2.0, 20.0, rng)
    y = oracle.project_fwd(g, np.zeros(1), np.zeros((1, 6)), vol).astype(np.float32)
    y = np.repeat(y, V, axis=0)
    _fused_case(dp, oracle, g, vol, angles, poses, y, "source-inside")


def test_fused_tiny(dp, oracle):
    g = Geom(1, 1, 1, 3.0, 3.0, 3.0, 1, 1, 2.0, 2.0)
    vol = np.array([[[0.7]]], np.float32)
    _fused_case(dp, oracle, g, vol, np.array([0.2]), np.array([[0.3, -0.2, 0.1, 0.01, 0.02, -0.03]]),
                np.array([[[0.5]]], np.float32), "1x1x1")


def test_fused_full_size_two_views(dp, oracle):
    """The registration-scale volume and detector (256^3 at 0.8 mm, 512x512 at
    0.6 mm), two of the candidate poses, in full."""
    c = synth.config2_inputs()
    g = c["geom"]
    angles, poses = c["angles"][:2], c["poses"][:2]
    y = np.repeat(oracle.project_fwd(g, [0.0], c["target_pose"], c["vol"]), 2, axis=0).astype(np.float32)
    _fused_case(dp, oracle, g, c["vol"], angles, poses, y, "full-size")


def test_fused_matches_two_call_path(dp, oracle):
    """Same outputs as project_fwd followed by project_fwd_grad_pose with
    w = 2 (l - y), up to FP32 summation grouping."""
    c = synth.config1_inputs()
    g = c["geom"]
    y = f32(oracle.project_fwd(g, c["angles"], c["target_pose"], c["vol"]))
    a, p, v = f64(c["angles"]), f64(c["poses"]), f32(c["vol"])
    l1, loss, g1 = dp.project_fwd_ssd_grad_pose(g, a, p, v, y)
    l2 = dp.project_fwd(g, a, p, v)
    g2 = dp.project_fwd_grad_pose(g, a, p, v, 2.0 * (l2 - y))
    assert torch.allclose(l1, l2, rtol=0, atol=1e-6 * float(l2.abs().max()))
    check_grads("fused vs two-call", g1.cpu().numpy(), g2.cpu().numpy())


@pytest.mark.parametrize("case", ["config1", "ragged"])
def test_gauss_newton_matrix_matches_oracle(dp, oracle, case):
    """dp_project_fwd_ssd_gauss_newton: the same projections, SSD and
    gradient as the plain fused entry (bitwise: same kernel sums), and the
    Gauss-Newton matrix 2 sum J J^T against the oracle's per-ray Jacobian,
    per view ||H - H_ref||_F <= 1e-4 ||H_ref||_F (FP32 per-ray products and
    block sums, FP64 across blocks)."""
    if case == "config1":
        c = synth.config1_inputs()
        g, vol, angles, poses = c["geom"], c["vol"], c["angles"], c["poses"]
        y = oracle.project_fwd(g, angles, c["target_pose"], vol).astype(np.float32)
    else:
        rng = synth.rng_for(212)
        g = Geom(37, 29, 23, 1.3, 1.1, 1.7, 45, 27, 1.9, 2.3, off_u=1.25, off_v=-0.75)
        vol = synth.ellipsoid_phantom(37, 1.3, 6, rng)[:23, :29, :37].copy()
        angles = rng.uniform(0, 2 * math.pi, 4)
        poses = synth.random_poses(4, 8.0, 15.0, rng)
        y = oracle.project_fwd(g, angles, synth.random_poses(4, 8.0, 15.0, rng), vol).astype(np.float32)
    a, p, v, t = f64(angles), f64(poses), f32(vol), f32(y)
    l1, L1, g1 = dp.project_fwd_ssd_grad_pose(g, a, p, v, t)
    l2, L2, g2, H = dp.project_fwd_ssd_gauss_newton(g, a, p, v, t)
    assert torch.equal(l1, l2) and torch.equal(L1, L2) and torch.equal(g1, g2)
    H_ref = oracle.gauss_newton_ssd(g, angles, poses, vol)
    Hg = H.cpu().numpy()
    assert np.allclose(Hg, np.transpose(Hg, (0, 2, 1)))
    err = np.linalg.norm(Hg - H_ref, axis=(1, 2)) / np.linalg.norm(H_ref, axis=(1, 2))
    say(f"{case} Gauss-Newton matrix: worst per-view rel err {err.max():.3e}")
    assert err.max() <= 1e-4


def test_fused_full_launch_the_bench_times(dp, oracle):
    """The registration-scale launch exactly as the bench times it (256^3,
    64 poses, 512x512, one single-pass launch).  Targets equal the launch's
    own projections (a first launch; the kernel is deterministic) except on
    64 random rays per view, where they are offset by N(0, 100^2); so
    dL/dl = 2 (l - y) lives exactly on those rays and the oracle can evaluate
    it ray by ray: sampled projections (<= 1e-5), the per-view SSD (<= 1e-5
    relative) and the pose gradients (<= 1e-4) against the oracle with
    dL/dl = 2 (l_ref - y) on the selected rays and 0 elsewhere."""
    c = synth.config2_inputs()
    g, vol, angles, poses = c["geom"], c["vol"], c["angles"], c["poses"]
    V = len(angles)
    a, p, v = f64(angles), f64(poses), f32(vol)
    l_fwd = dp.project_fwd_ssd_grad_pose(g, a, p, v, dp.project_fwd(g, a, p, v))[0]
    rng = np.random.default_rng(13)
    npix = g.nu * g.nv
    sel = np.stack([rng.choice(npix, 64, replace=False) for _ in range(V)])
    ids = (sel + np.arange(V)[:, None] * npix).ravel()
    delta = rng.normal(0.0, 100.0, ids.size).astype(np.float32)
    y = l_fwd.clone().reshape(-1)
    y[torch.from_numpy(ids).cuda()] += torch.from_numpy(delta).cuda()
    y = y.reshape(V, g.nv, g.nu)
    l, loss, gp = dp.project_fwd_ssd_grad_pose(g, a, p, v, y)
    assert torch.equal(l, l_fwd)
    l_ref = oracle.project_fwd_rays(g, angles, poses, vol, ids)
    got = l.cpu().numpy().reshape(-1)[ids]
    err = np.abs(got - l_ref).max() / np.abs(l_ref).max()
    say(f"full launch sampled projections: max rel err {err:.3e}")
    assert err <= 1e-5
    y_sel = y.cpu().numpy().reshape(-1)[ids]
    r_ref = (l_ref - y_sel).reshape(V, 64)
    loss_ref = (r_ref.astype(np.float64) ** 2).sum(1)
    rel = np.abs(loss.cpu().numpy() - loss_ref) / loss_ref
    say(f"full launch per-view SSD: max rel err {rel.max():.3e}")
    assert rel.max() <= 1e-5
    w = np.zeros(V * npix, np.float32)
    w[ids] = (2.0 * (l_ref - y_sel)).astype(np.float32)
    g_ref = oracle.project_fwd_grad_pose(g, angles, poses, vol, w.reshape(V, g.nv, g.nu))
    check_grads("full launch fused gradient", gp.cpu().numpy(), g_ref)


@pytest.mark.parametrize("variant", range(N_VARIANTS))
def test_sparse_rays_unstaged_tiles(dp, oracle, variant):
    """Rays much sparser than voxels (1.33 mm pixels at the isocentre over
    0.5 mm voxels): a 16 x 16 tile's chunk box exceeds the LDS capacity even
    one sample deep, so every tile gathers (mu, Gx, Gy, Gz) per trilinear
    corner from the padded copy the library makes for sparse-ray geometries.  Fused SSD entry, Gauss-Newton matrix and the
    plain gradient entry against the oracle; ragged detector tail."""
    rng = synth.rng_for(214)
    g = Geom(80, 72, 64, 0.5, 0.5, 0.5, 40, 36, 2.0, 2.0, off_u=0.5)
    vol = synth.ellipsoid_phantom(80, 0.5, 8, rng)[:64, :72, :80].copy()
    V = 3
    angles = np.array([0.3, 1.9, 4.0])
    poses = synth.random_poses(V, 2.0, 4.0, rng)
    y = oracle.project_fwd(g, angles, synth.random_poses(V, 2.0, 4.0, rng), vol).astype(np.float32)
    _fused_case(dp, oracle, g, vol, angles, poses, y, f"sparse-v{variant}", variant)
    a, p, v, t = f64(angles), f64(poses), f32(vol), f32(y)
    try:
        dp.set_variant(dp.OP_FWD_SSD, variant)
        dp.set_variant(dp.OP_FWD_GRAD, variant)
        _, _, _, H = dp.project_fwd_ssd_gauss_newton(g, a, p, v, t)
        w = rng.standard_normal((V, g.nv, g.nu)).astype(np.float32)
        gp = dp.project_fwd_grad_pose(g, a, p, v, f32(w))
    finally:
        dp.set_variant(dp.OP_FWD_SSD, -1)
        dp.set_variant(dp.OP_FWD_GRAD, -1)
    H_ref = oracle.gauss_newton_ssd(g, angles, poses, vol)
    err = np.linalg.norm(H.cpu().numpy() - H_ref, axis=(1, 2)) / np.linalg.norm(H_ref, axis=(1, 2))
    say(f"sparse-v{variant} Gauss-Newton matrix: worst per-view rel err {err.max():.3e}")
    assert err.max() <= 1e-4
    check_grads(f"sparse-v{variant} grad", gp.cpu().numpy(),
                oracle.project_fwd_grad_pose(g, angles, poses, vol, w))


def test_fused_full_size_oracle_targets_dense(dp, oracle):
    """Registration scale at full size (256^3 phantom, 512x512 detector) with
    the target DRR rendered by the oracle at the true pose, as the
    registration workload has it, and 8 candidate poses in one launch: every
    pixel carries a residual, so dL/dl = 2 (l - y) is dense on all 8 views.
    Whole projections (<= 1e-5), per-view SSD (<= 1e-5 relative) and pose
    gradients (<= 1e-4, oracle gradient with dL/dl = 2 (l_ref - y))."""
    c = synth.config2_inputs()
    g, vol = c["geom"], c["vol"]
    V = 8
    angles, poses = c["angles"][:V], c["poses"][:V]
    y1 = oracle.project_fwd(g, c["angles"][:1], c["target_pose"], vol).astype(np.float32)
    y = np.repeat(y1, V, axis=0)
    _fused_case(dp, oracle, g, vol, angles, poses, y, "full-size dense")


@pytest.mark.parametrize("variant", range(N_VARIANTS))
def test_oblique_tiles_gathering_from_the_volume(dp, oracle, variant):
    """Pixel footprint at the isocentre just below the sparse-ray threshold
    (0.42 mm over 0.5 mm voxels: no (mu, G) copy is made) with diagonal views
    and large rotations: the chunk boxes of a 16 x 16 tile's diagonal rays
    outgrow the LDS even one sample deep, so those tiles form (mu, Gx, Gy,
    Gz) at each trilinear corner from the 32 voxels around it.  Fused SSD
    entry and the plain gradient entry against the oracle."""
    rng = synth.rng_for(215)
    g = Geom(40, 44, 36, 0.5, 0.5, 0.5, 60, 52, 0.63, 0.63)
    vol = synth.ellipsoid_phantom(44, 0.5, 8, rng)[:36, :44, :40].copy()
    V = 3
    angles = np.radians([45.0, 135.0, 200.0])
    poses = synth.random_poses(V, 2.0, 25.0, rng)
    y = oracle.project_fwd(g, angles, synth.random_poses(V, 2.0, 25.0, rng), vol).astype(np.float32)
    _fused_case(dp, oracle, g, vol, angles, poses, y, f"oblique-v{variant}", variant)
    w = rng.standard_normal((V, g.nv, g.nu)).astype(np.float32)
    try:
        dp.set_variant(dp.OP_FWD_GRAD, variant)
        gp = dp.project_fwd_grad_pose(g, f64(angles), f64(poses), f32(vol), f32(w))
    finally:
        dp.set_variant(dp.OP_FWD_GRAD, -1)
    check_grads(f"oblique-v{variant} grad", gp.cpu().numpy(),
                oracle.project_fwd_grad_pose(g, angles, poses, vol, w))


@pytest.mark.parametrize("case", ["shallow-boxes", "aligned-rows"])
def test_box_staging_paths(dp, oracle, case):
    """Both staging paths of the ray kernels against the oracle, for the
    forward, the gradient-only and the single-pass kernels, on volumes whose
    rows are 16-byte aligned (nx a multiple of 4, the vector path's
    condition).  shallow-boxes: 0.1 mm pixels at the isocentre over 3 mm
    voxels, so a 16x16 tile spans about half a voxel and the interior chunk
    boxes are 2-3 planes deep (fewer than the vector path's 4-plane items:
    the scalar path stages them).  aligned-rows: 0.6 mm at the isocentre over
    0.7 mm voxels, boxes many planes deep whose x range starts and ends
    inside 4-voxel segments (the vector path, last z run overlapping)."""
    from test_gpu_parity import _fwd_case
    rng = synth.rng_for(230 if case == "shallow-boxes" else 231)
    if case == "shallow-boxes":
        g = Geom(32, 24, 16, 3.0, 3.0, 3.0, 48, 40, 0.15, 0.15, off_u=0.3, off_v=-0.2)
        vol = synth.ellipsoid_phantom(32, 3.0, 6, rng)[:16, :24, :32].copy()
    else:
        g = Geom(48, 44, 40, 0.7, 0.7, 0.7, 64, 60, 0.9, 0.9, off_u=-0.4, off_v=0.6)
        vol = synth.ellipsoid_phantom(48, 0.7, 8, rng)[:40, :44, :48].copy()
    V = 3
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 1.0, 4.0, rng)
    _fwd_case(dp, oracle, g, vol, angles, poses, name=case)
    y = oracle.project_fwd(g, angles, synth.random_poses(V, 1.0, 4.0, rng), vol).astype(np.float32)
    _fused_case(dp, oracle, g, vol, angles, poses, y, case)


@pytest.mark.parametrize("du", [1.8, 2.2])
def test_many_chunks_per_tile(dp, oracle, du):
    """Wide tiles over a deep volume (96 x 128 x 128 at 1 mm, pixels of 1.2 /
    1.5 mm at the isocentre, rays of ~200 samples): the chunk length drops
    to 2-6 samples (1.8 mm pixels) or to a single sample, ~195 chunks per
    tile with the box records of all four wavefronts in use (2.2 mm; that
    geometry's other tiles gather from the volume), for the forward, the
    gradient-only and the single-pass kernels against the oracle."""
    from test_gpu_parity import _fwd_case
    rng = synth.rng_for(232)
    g = Geom(96, 128, 128, 1.0, 1.0, 1.0, 48, 48, du, du)
    vol = synth.ellipsoid_phantom(128, 1.0, 10, rng)[:, :, 16:112].copy()
    angles = np.array([0.0, 0.02])
    poses = np.array([[0.5, -0.3, 0.2, 0.01, 0.02, -0.01], [-0.4, 0.2, 0.1, -0.02, 0.01, 0.015]])
    _fwd_case(dp, oracle, g, vol, angles, poses, name=f"many-chunks-{du}")
    y = oracle.project_fwd(g, angles, synth.random_poses(2, 1.0, 2.0, rng), vol).astype(np.float32)
    _fused_case(dp, oracle, g, vol, angles, poses, y, f"many-chunks-{du}")
