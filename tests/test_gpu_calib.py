"""Device-resident batched calibration: the single-pass SSD / Gauss-Newton
batch launch, the FP64 Levenberg-Marquardt update kernel, and the whole
iteration replayed from a HIP graph."""
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


def say(msg):
    print(msg, flush=True)


SPECS = [(48, 2.0, 64, 2.2, 3), (32, 3.0, 40, 3.1, 1), (64, 1.5, 80, 1.7, 2), (24, 4.0, 33, 4.4, 5)]


def _problems(dp, seed, t_mm=3.0, r_deg=2.0, specs=SPECS):
    """Uneven problems: own phantom, geometry and views each; target DRRs at
    the true poses, start at truth + a perturbation."""
    rng = synth.rng_for(seed)
    probs, truth, init = [], [], []
    for n, h, nu, du, V in specs:
        g = Geom(n, n, n, h, h, h, nu, nu, du, du)
        vol = T(synth.ellipsoid_phantom(n, h, 6, rng), torch.float32)
        angles = T(rng.uniform(0, 2 * math.pi, V))
        tp = T(synth.random_poses(V, 5.0, 3.0, rng))
        probs.append(dict(geom=g, angles=angles, vol=vol, target=dp.project_fwd(g, angles, tp, vol)))
        truth.append(tp)
        init.append(tp + T(synth.random_poses(V, t_mm, r_deg, rng)))
    return probs, torch.cat(truth), torch.cat(init)


def _with_outputs(probs, poses):
    out, a = [], 0
    for q in probs:
        g, V = q["geom"], q["angles"].numel()
        out.append(dict(q, poses=poses[a:a + V].contiguous(),
                        proj=torch.empty((V, g.nv, g.nu), dtype=torch.float32, device=DEV),
                        grad_pose=torch.empty((V, 6), dtype=torch.float64, device=DEV),
                        hess=torch.empty((V, 21), dtype=torch.float64, device=DEV),
                        loss=torch.empty(V, dtype=torch.float64, device=DEV)))
        a += V
    return out


@pytest.mark.parametrize("variant", range(N_VARIANTS))
def test_ssd_batch_equals_single_launches(dp, oracle, variant):
    """Every problem of the batch gets bit for bit what the single-problem
    entry gives with the same kernel variant (same tiles, same block sums),
    LDS-staged and direct-gather tiles alike; one problem also against the
    oracle's Gauss-Newton matrix."""
    # the last problem has rays much sparser than its voxels (1.33 mm pixels
    # at the isocentre over 0.5 mm voxels): its tiles take the direct path
    probs, truth, init = _problems(dp, 610, specs=SPECS + [(80, 0.5, 40, 2.0, 2)])
    items = _with_outputs(probs, init)
    dp.project_fwd_ssd_gauss_newton_batch(items, variant=variant)
    try:
        dp.set_variant(dp.OP_FWD_SSD, variant)
        for d in items:
            l, L, gp, H = dp.project_fwd_ssd_gauss_newton(d["geom"], d["angles"], d["poses"],
                                                         d["vol"], d["target"])
            assert torch.equal(d["proj"], l)
            assert torch.equal(d["loss"], L)
            assert torch.equal(d["grad_pose"], gp)
            assert torch.equal(dp.unpack_sym6(d["hess"]), H)
    finally:
        dp.set_variant(dp.OP_FWD_SSD, -1)
    d = items[2]
    H_ref = oracle.gauss_newton_ssd(d["geom"], d["angles"].cpu().numpy(), d["poses"].cpu().numpy(),
                                    d["vol"].cpu().numpy())
    Hg = dp.unpack_sym6(d["hess"]).cpu().numpy()
    err = np.linalg.norm(Hg - H_ref, axis=(1, 2)) / np.linalg.norm(H_ref, axis=(1, 2))
    say(f"variant {variant}: batch Gauss-Newton matrix worst rel err {err.max():.3e}")
    assert err.max() <= 1e-4


def test_ssd_batch_validates_arguments(dp):
    probs, truth, init = _problems(dp, 611, specs=SPECS[:2])
    items = _with_outputs(probs, init)
    items[1]["hess"] = None
    with pytest.raises((TypeError, AttributeError, RuntimeError)):
        dp.project_fwd_ssd_gauss_newton_batch(items)


# --- the update rule, element by element -----------------------------------------

SCALE = np.array([1.0] * 3 + [math.pi / 180.0] * 3)


def _lm_ref(trial, f, g, h21, st, tol, lam_max=1e10):
    """The update rule written with numpy (solve by LU), one view at a time."""
    iu = np.triu_indices(6)
    trial = trial.copy()
    st = {k: v.copy() for k, v in st.items()}
    for i in range(len(f)):
        if st["done"][i]:
            continue
        lam = st["lam"][i]
        stop = False
        if f[i] < st["f"][i]:
            step = np.max(np.abs(trial[i] - st["pose"][i]) / SCALE)
            first = not np.isfinite(st["f"][i])
            st["pose"][i], st["g"][i], st["h"][i], st["f"][i] = trial[i], g[i], h21[i], f[i]
            if not first:
                lam /= 3.0
                stop = step < tol
        else:
            lam *= 4.0
        stop = stop or lam > lam_max
        st["lam"][i] = lam
        if stop:
            st["done"][i] = 1
            trial[i] = st["pose"][i]
            continue
        H = np.zeros((6, 6))
        H[iu] = st["h"][i]
        H = H + np.triu(H, 1).T
        Hz = H * np.outer(SCALE, SCALE)
        A = Hz + lam * np.diag(np.diag(Hz) + 1e-12)
        d = np.linalg.solve(A, -st["g"][i] * SCALE)
        trial[i] = st["pose"][i] + d * SCALE
    return trial, st


def test_lm_update_kernel_matches_rule(dp):
    """Accept, reject, first evaluation (state f = inf), NaN trial value,
    convergence by step size, lam above its cap and already-finished views,
    all in one launch, against the same rule in numpy."""
    rng = np.random.default_rng(620)
    n = 70  # more than one block of the update kernel
    J = rng.standard_normal((n, 40, 6)) * np.array([1, 2, 0.5, 30, 10, 60])
    H = 2 * np.einsum("npi,npj->nij", J, J)
    iu = np.triu_indices(6)
    h21 = H[:, iu[0], iu[1]].copy()
    g = rng.standard_normal((n, 6)) * 5
    f = rng.uniform(1, 10, n)
    st = dict(pose=rng.standard_normal((n, 6)) * 0.1, f=rng.uniform(1, 10, n),
              g=rng.standard_normal((n, 6)), h=h21[::-1].copy(), lam=10.0 ** rng.uniform(-4, 2, n),
              done=np.zeros(n, dtype=np.int32))
    trial = st["pose"] + rng.standard_normal((n, 6)) * 0.01
    st["f"][0:5] = np.inf                                  # first evaluation
    f[5:8] = np.nan                                        # failed evaluation: rejected
    trial[8:12] = st["pose"][8:12] + 1e-7                  # converged step (if accepted)
    f[8:12] = st["f"][8:12] - 1.0
    st["lam"][12:14] = 5e9                                 # reject pushes lam over the cap
    f[12:14] = st["f"][12:14] + 1.0
    st["done"][14:17] = 1                                  # finished views stay as they are
    tr_ref, st_ref = _lm_ref(trial, f, g, h21, st, 1e-4)
    t_trial = T(trial)
    t_state = {k: T(v, torch.int32 if k == "done" else torch.float64) for k, v in st.items()}
    dp.lm_update(t_trial, T(f), T(g), T(h21), t_state, tol=1e-4)
    torch.cuda.synchronize()
    assert np.array_equal(t_state["done"].cpu().numpy(), st_ref["done"])
    for k in ("f", "lam", "pose", "g", "h"):
        assert np.allclose(t_state[k].cpu().numpy(), st_ref[k], rtol=0, atol=0), k
    err = np.abs(t_trial.cpu().numpy() - tr_ref).max()
    say(f"LM update: max trial-pose difference to the numpy rule {err:.3e}")
    assert err <= 1e-12
    assert st_ref["done"][8:17].all() and not st_ref["done"][:5].any()


def test_lm_update_validates_arguments(dp):
    z = torch.zeros((3, 6), dtype=torch.float64, device=DEV)
    st = dict(pose=z.clone(), f=torch.zeros(3, dtype=torch.float64, device=DEV), g=z.clone(),
              h=torch.zeros((3, 21), dtype=torch.float64, device=DEV),
              lam=torch.ones(3, dtype=torch.float64, device=DEV),
              done=torch.zeros(3, dtype=torch.float32, device=DEV))
    with pytest.raises(TypeError):
        dp.lm_update(z.clone(), st["f"], z, st["h"], st)
    st["done"] = torch.zeros(3, dtype=torch.int32, device=DEV)
    with pytest.raises(RuntimeError):
        dp.lm_update(z.clone(), st["f"], z, st["h"], st, tol=-1.0)


# --- whole registrations ------------------------------------------------------------

def test_batch_lm_matches_host_lm(dp):
    """The device-resident batch LM and the host-driven LM (one problem at a
    time, torch solve) follow the same rule on the same evaluations: the same
    converged poses, and both reach the true poses."""
    from paper_2508_13304_amd.registration import BatchLM, pose_errors, register_lm
    probs, truth, init = _problems(dp, 630)
    lm = BatchLM(probs, init)
    lm.run(60, graph=False)
    pose, conv, f = lm.result()
    assert bool(conv.all())
    a = 0
    for q in probs:
        V = q["angles"].numel()
        r = register_lm(q["geom"], q["vol"], q["angles"], q["target"], init[a:a + V])
        assert bool(r.converged.all())
        d = (pose[a:a + V] - r.poses).abs()
        say(f"problem of {V} views: max |batch - host| {d[:, :3].max():.2e} mm "
            f"{math.degrees(d[:, 3:].max()):.2e} deg")
        assert float(d[:, :3].max()) <= 1e-3 and math.degrees(float(d[:, 3:].max())) <= 1e-3
        a += V
    te, re = pose_errors(pose, truth)
    say(f"batch LM: worst error {float(te.max()):.3e} mm {float(re.max()):.3e} deg over {lm.n} views")
    assert float(te.max()) <= 0.1 and float(re.max()) <= 0.1


def test_batch_lm_graph_replays_like_eager(dp):
    """The captured iteration (batch launch + update) replayed with eager
    work and synchronisations between replays equals the eager iterations
    bit for bit, state and trial poses."""
    from paper_2508_13304_amd.registration import BatchLM
    probs, truth, init = _problems(dp, 631)
    lm = BatchLM(probs, init)
    ref = []
    for _ in range(4):
        lm.step()
        ref.append((lm.state["pose"].clone(), lm.state["lam"].clone(), lm.trial.clone()))
    lm.reset(init)
    lm.capture()
    torch.cuda.synchronize()
    assert torch.equal(lm.trial, init)
    for i, (p, lam, tr) in enumerate(ref):
        lm.run(1)
        torch.cuda.synchronize()
        assert torch.equal(lm.state["pose"], p), i
        assert torch.equal(lm.state["lam"], lam), i
        assert torch.equal(lm.trial, tr), i
        _ = (lm.loss.sum() + 1.0).item()  # eager work between replays


def test_batch_lm_beyond_sixteen_problems(dp):
    """18 problems run as launches of 16 + 2 sharing one workspace: the
    iterations equal those of two separate batches bit for bit, and the
    workspace query reports the larger chunk."""
    from paper_2508_13304_amd.registration import BatchLM
    specs = [(16 + 4 * (i % 3), 3.0, 24 + 4 * (i % 2), 3.1, 1 + i % 2) for i in range(18)]
    probs, truth, init = _problems(dp, 640, specs=specs)
    n16 = sum(q["angles"].numel() for q in probs[:16])
    both = BatchLM(probs, init)
    first, second = BatchLM(probs[:16], init[:n16]), BatchLM(probs[16:], init[n16:])
    assert both.ws.numel() == max(first.ws.numel(), second.ws.numel())
    for _ in range(3):
        both.step()
        first.step()
        second.step()
    torch.cuda.synchronize()
    assert torch.equal(both.state["pose"], torch.cat([first.state["pose"], second.state["pose"]]))
    assert torch.equal(both.trial, torch.cat([first.trial, second.trial]))


def test_calibration_batch_full_size_sampled(dp, oracle):
    """The uneven calibration batch at full size in the launch the bench
    times (16 problems of 128^3-384^3 with 256^2-768^2 detectors, 82 views,
    one batched single-pass Gauss-Newton launch), at the identity pose of the
    first calibration iteration.  Targets equal the launch's own projections
    (a first launch) except on 32 random rays per view, offset by
    N(0, 100^2), so the residual lives exactly on rays the oracle can
    evaluate one by one: sampled projections (<= 1e-5 of
    max), per-view SSD (<= 1e-5 relative) for every problem, pose gradients
    (<= 1e-4 per triplet) for four problems; the Gauss-Newton matrices are
    checked by property (symmetric positive semi-definite) and against the
    single-problem entry bit for bit."""
    from test_gpu_parity import check_grads
    probs = synth.config4_problems(DEV)
    rng = np.random.default_rng(17)
    items, picks = [], []
    for q in probs:
        g, V = q["geom"], q["angles"].numel()
        poses = torch.zeros((V, 6), dtype=torch.float64, device=DEV)
        npix = g.nu * g.nv
        sel = np.stack([rng.choice(npix, 32, replace=False) for _ in range(V)])
        ids = (sel + np.arange(V)[:, None] * npix).ravel()
        items.append(dict(geom=g, angles=q["angles"], vol=q["vol"], poses=poses,
                          target=dp.project_fwd(g, q["angles"], poses, q["vol"]),
                          proj=torch.empty((V, g.nv, g.nu), dtype=torch.float32, device=DEV),
                          grad_pose=torch.empty((V, 6), dtype=torch.float64, device=DEV),
                          hess=torch.empty((V, 21), dtype=torch.float64, device=DEV),
                          loss=torch.empty(V, dtype=torch.float64, device=DEV)))
        picks.append(ids)
    dp.project_fwd_ssd_gauss_newton_batch(items)
    for d, ids in zip(items, picks):
        y = d["proj"].clone().reshape(-1)
        y[torch.from_numpy(ids).to(DEV)] += torch.from_numpy(rng.normal(0.0, 100.0, ids.size)).float().to(DEV)
        d["target"] = y.reshape(d["proj"].shape)
    dp.project_fwd_ssd_gauss_newton_batch(items)
    torch.cuda.synchronize()
    order = sorted(range(len(items)), key=lambda i: items[i]["geom"].nx * items[i]["geom"].nu)
    grad_check = {order[0], order[-1], order[len(order) // 2], order[len(order) // 3]}
    worst_l = worst_s = 0.0
    for i, (d, ids) in enumerate(zip(items, picks)):
        g, V = d["geom"], d["angles"].numel()
        a = d["angles"].cpu().numpy()
        p = np.zeros((V, 6))
        vol = d["vol"].cpu().numpy()
        l_ref = oracle.project_fwd_rays(g, a, p, vol, ids)
        got = d["proj"].cpu().numpy().reshape(-1)[ids]
        worst_l = max(worst_l, np.abs(got - l_ref).max() / np.abs(l_ref).max())
        y_sel = d["target"].cpu().numpy().reshape(-1)[ids]
        loss_ref = ((l_ref - y_sel).astype(np.float64) ** 2).reshape(V, -1).sum(1)
        worst_s = max(worst_s, float((np.abs(d["loss"].cpu().numpy() - loss_ref) / loss_ref).max()))
        H = dp.unpack_sym6(d["hess"]).cpu().numpy()
        ev = np.linalg.eigvalsh(H)
        assert (ev.min(axis=1) >= -1e-6 * ev.max(axis=1)).all(), i
        if i in grad_check:
            w = np.zeros(V * g.nu * g.nv, np.float32)
            w[ids] = (2.0 * (l_ref - y_sel)).astype(np.float32)
            g_ref = oracle.project_fwd_grad_pose(g, a, p, vol, w.reshape(V, g.nv, g.nu))
            check_grads(f"calibration problem {i} ({g.nx}^3, {g.nu}^2, {V} views)",
                        d["grad_pose"].cpu().numpy(), g_ref)
            _, L1, g1, H1 = dp.project_fwd_ssd_gauss_newton(g, d["angles"], d["poses"], d["vol"],
                                                           d["target"], packed=True)
            assert torch.equal(L1, d["loss"]) and torch.equal(g1, d["grad_pose"])
            assert torch.equal(H1, d["hess"])
    say(f"calibration batch full size: sampled projections max rel err {worst_l:.3e}, "
        f"per-view SSD max rel err {worst_s:.3e}")
    assert worst_l <= 1e-5 and worst_s <= 1e-5
