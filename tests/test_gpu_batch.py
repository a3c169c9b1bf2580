"""Uneven batches in one launch, kernel variants / autotuner, graph capture."""
import math

import numpy as np
import pytest
import torch

import synth
from paper_2508_13304_amd import N_VARIANTS
from synth import Geom

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def T(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


def _problem(rng, n, h, nu, du, V):
    g = Geom(n, n, n, h, h, h, nu, nu, du, du)
    vol = synth.ellipsoid_phantom(n, h, 6, rng)
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 5.0, 3.0, rng)
    return g, vol, angles, poses


def _uneven(seed):
    rng = synth.rng_for(seed)
    specs = [(48, 2.0, 64, 2.2, 3), (32, 3.0, 40, 3.1, 1), (64, 1.5, 80, 1.7, 2), (24, 4.0, 33, 4.4, 5)]
    return [_problem(rng, *sp) for sp in specs], rng


def test_batch_forward_and_gradient_equal_single_launches(dp, oracle):
    probs, rng = _uneven(500)
    fwd, grad, singles = [], [], []
    for g, vol, angles, poses in probs:
        V = len(angles)
        w = rng.standard_normal((V, g.nv, g.nu)).astype(np.float32)
        d = dict(geom=g, angles=T(angles), poses=T(poses), vol=T(vol, torch.float32),
                 proj=torch.empty((V, g.nv, g.nu), dtype=torch.float32, device=DEV),
                 grad_proj=T(w, torch.float32),
                 grad_pose=torch.empty((V, 6), dtype=torch.float64, device=DEV))
        fwd.append(d)
        singles.append((dp.project_fwd(g, d["angles"], d["poses"], d["vol"]),
                        dp.project_fwd_grad_pose(g, d["angles"], d["poses"], d["vol"], d["grad_proj"])))
    dp.project_fwd_batch(fwd)
    dp.project_fwd_grad_pose_batch(fwd)
    torch.cuda.synchronize()
    for d, (l1, g1) in zip(fwd, singles):
        assert torch.equal(d["proj"], l1)
        assert torch.equal(d["grad_pose"], g1)
    # and one of them against the oracle
    g, vol, angles, poses = probs[2]
    ref = oracle.project_fwd(g, angles, poses, vol)
    err = np.abs(fwd[2]["proj"].cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 1e-5


def test_batch_of_more_than_sixteen_problems(dp):
    rng = synth.rng_for(501)
    items = []
    for i in range(20):
        g, vol, angles, poses = _problem(rng, 16 + (i % 3) * 8, 2.0, 24, 2.5, 1 + i % 2)
        V = len(angles)
        items.append(dict(geom=g, angles=T(angles), poses=T(poses), vol=T(vol, torch.float32),
                          proj=torch.empty((V, g.nv, g.nu), dtype=torch.float32, device=DEV)))
    dp.project_fwd_batch(items)
    for d in items:
        ref = dp.project_fwd(d["geom"], d["angles"], d["poses"], d["vol"])
        assert torch.equal(d["proj"], ref)


@pytest.mark.parametrize("variant", range(N_VARIANTS))
def test_every_variant_meets_oracle_tolerance(dp, oracle, variant):
    rng = synth.rng_for(502)
    g = Geom(56, 48, 40, 1.2, 1.3, 1.4, 70, 50, 1.6, 1.8)
    vol = synth.ellipsoid_phantom(56, 1.2, 8, rng)[:40, :48, :56].copy()
    V = 3
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 6, 20, rng)
    w = rng.standard_normal((V, g.nv, g.nu)).astype(np.float32)
    try:
        dp.set_variant(dp.OP_FWD, variant)
        dp.set_variant(dp.OP_FWD_GRAD, variant)
        l = dp.project_fwd(g, T(angles), T(poses), T(vol, torch.float32)).cpu().numpy()
        gp = dp.project_fwd_grad_pose(g, T(angles), T(poses), T(vol, torch.float32),
                                      T(w, torch.float32)).cpu().numpy()
    finally:
        dp.set_variant(dp.OP_FWD, -1)
        dp.set_variant(dp.OP_FWD_GRAD, -1)
    ref = oracle.project_fwd(g, angles, poses, vol)
    assert np.abs(l - ref).max() <= 1e-5 * np.abs(ref).max()
    gref = oracle.project_fwd_grad_pose(g, angles, poses, vol, w)
    for v in range(V):
        for sl in (slice(0, 3), slice(3, 6)):
            assert np.linalg.norm(gp[v, sl] - gref[v, sl]) <= 1e-4 * np.linalg.norm(gref[v, sl])


def test_autotune_records_choice(dp):
    rng = synth.rng_for(503)
    g = Geom(64, 64, 64, 1.0, 1.0, 1.0, 96, 96, 1.2, 1.2)
    vol = T(synth.ellipsoid_phantom(64, 1.0, 8, rng), torch.float32)
    V = 4
    angles, poses = T(rng.uniform(0, 6, V)), T(synth.random_poses(V, 5, 5, rng))
    out = torch.empty((V, g.nv, g.nu), dtype=torch.float32, device=DEV)
    best, ms = dp.autotune(dp.OP_FWD, g, angles, poses, vol, out, reps=2)
    assert 0 <= best < dp.N_VARIANTS and all(m > 0 for m in ms)
    assert ms[best] == min(ms)
    assert dp.get_variant(g, V, dp.OP_FWD) == best
    gp = torch.empty((V, 6), dtype=torch.float64, device=DEV)
    w = torch.ones((V, g.nv, g.nu), dtype=torch.float32, device=DEV)
    bestg, msg = dp.autotune(dp.OP_FWD_GRAD, g, angles, poses, vol, gp, grad_proj=w, reps=2)
    assert dp.get_variant(g, V, dp.OP_FWD_GRAD) == bestg


def test_autotune_single_pass_ssd(dp, oracle):
    """Autotuning the single-pass SSD launch: every variant is timed, the
    fastest is cached for the shape class and used by later calls, and the
    caller's outputs hold a valid evaluation (its DRRs match the oracle)."""
    rng = synth.rng_for(505)
    g = Geom(48, 48, 48, 1.5, 1.5, 1.5, 64, 64, 1.6, 1.6)
    vol = synth.ellipsoid_phantom(48, 1.5, 8, rng)
    V = 3
    angles, poses = rng.uniform(0, 6, V), synth.random_poses(V, 4, 4, rng)
    y = T(oracle.project_fwd(g, angles, synth.random_poses(V, 4, 4, rng), vol), torch.float32)
    proj = torch.empty((V, g.nv, g.nu), dtype=torch.float32, device=DEV)
    best, ms = dp.autotune(dp.OP_FWD_SSD, g, T(angles), T(poses), T(vol, torch.float32), proj,
                           grad_proj=y, reps=2)
    assert 0 <= best < dp.N_VARIANTS and all(m > 0 for m in ms) and ms[best] == min(ms)
    assert dp.get_variant(g, V, dp.OP_FWD_SSD) == best
    ref = oracle.project_fwd(g, angles, poses, vol)
    assert np.abs(proj.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max()


def test_graph_captured_registration_step_replays_like_eager(dp):
    """One registration iteration (forward, SSD gradient, pose gradient, step)
    captured once and replayed several times, with eager work and
    synchronisations in between; every replay equals the eager iteration."""
    rng = synth.rng_for(504)
    g = Geom(48, 48, 48, 1.5, 1.5, 1.5, 64, 64, 1.6, 1.6)
    vol = T(synth.ellipsoid_phantom(48, 1.5, 8, rng), torch.float32)
    V = 4
    angles = T(rng.uniform(0, 6, V))
    target = dp.project_fwd(g, angles, T(synth.random_poses(V, 4, 4, rng)), vol)
    p0 = T(synth.random_poses(V, 4, 4, rng))
    ws_f = torch.empty(dp.workspace_bytes(g, V, dp.OP_FWD), dtype=torch.uint8, device=DEV)
    ws_g = torch.empty(dp.workspace_bytes(g, V, dp.OP_FWD_GRAD), dtype=torch.uint8, device=DEV)
    poses = p0.clone()
    l = torch.empty((V, g.nv, g.nu), dtype=torch.float32, device=DEV)
    w = torch.empty_like(l)
    gp = torch.empty((V, 6), dtype=torch.float64, device=DEV)
    lr = torch.tensor([0.05] * 3 + [1e-3] * 3, dtype=torch.float64, device=DEV)

    def step(stream=None):
        dp.project_fwd(g, angles, poses, vol, out=l, ws=ws_f, stream=stream)
        torch.sub(l, target, out=w)
        w.mul_(2.0)
        dp.project_fwd_grad_pose(g, angles, poses, vol, w, out=gp, ws=ws_g, stream=stream)
        poses.sub_(lr * torch.sign(gp))

    # eager reference trajectory
    ref = []
    for _ in range(3):
        step()
        ref.append(poses.clone())
    torch.cuda.synchronize()
    poses.copy_(p0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step(stream=s)  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    poses.copy_(p0)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step(stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    poses.copy_(p0)
    for i in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(poses, ref[i]), i
        _ = (l.sum() + 1.0).item()  # eager work between replays


def test_per_kernel_profiler(dp):
    """The event-based per-kernel timer: every library kernel a call launches
    is counted once per launch with a positive time, collecting resets the
    counts, and nothing is recorded while it is off."""
    rng = synth.rng_for(506)
    g = Geom(32, 32, 32, 2.0, 2.0, 2.0, 40, 40, 2.4, 2.4)
    vol = T(synth.ellipsoid_phantom(32, 2.0, 6, rng), torch.float32)
    V = 2
    a, p = T(rng.uniform(0, 6, V)), T(synth.random_poses(V, 3, 3, rng))
    dp.profile_collect()  # drop anything recorded before
    dp.profile_enable(True)
    try:
        l = dp.project_fwd(g, a, p, vol)
        dp.project_fwd_ssd_grad_pose(g, a, p, vol, l)
        dp.backproject(g, a, p, l, dp.W_FDK)
        got = dp.profile_collect()
    finally:
        dp.profile_enable(False)
    for k, n in (("setup", 3), ("rd_fwd", 1), ("rd_fused", 1), ("finalize", 1),
                 ("det_prep", 1), ("vd_bp", 1)):
        assert got[k][1] == n and got[k][0] > 0, (k, got.get(k))
    # dense rays (1.6 mm pixels at the isocentre over 2 mm voxels): the
    # ray-driven kernels stage the volume themselves, no volume pass
    assert "vol_prep" not in got
    assert dp.profile_collect() == {}
    dp.project_fwd(g, a, p, vol)
    assert dp.profile_collect() == {}
