"""Batched gradient-based 2D/3D rigid registration (Sec. II-D, 2D/3D
registration task): estimate theta* = argmin_theta loss(A(M(theta)) mu, l)
for many independent registrations at once.

Each registration is one view of a single projector launch (its own gantry
angle, pose and target image), so one iteration costs one forward and one
pose-gradient launch for the whole batch.  Two optimisers:

* ``register`` -- Adam (the optimiser the paper plugs its projector into)
  with separate step sizes for translations (mm) and rotations (deg), a
  step-size decay, and per-registration stopping: a registration whose
  largest update falls below a tolerance for a few consecutive iterations is
  frozen and dropped from later launches (stop="step"), or the registration
  experiment's rule (stop="paper", Sec. III-A): stop once the loss changes by
  less than 1e-5 between iterations or the NCC with the target exceeds
  0.999; a registration ending below NCC 0.99 counts as failed.
* ``register_bfgs`` -- quasi-Newton (BFGS inverse-Hessian updates on the six
  parameters in units of 1 mm / 1 deg, Armijo acceptance, a shorter step after
  each rejection).  It uses the same analytic gradient and converges to the
  exact optimum in a few tens of iterations, where Adam's fixed step sizes
  leave the weakly observed depth translation of a single view short.
* ``register_lm`` -- Levenberg-Marquardt for the SSD: the single-pass kernel
  also returns the Gauss-Newton matrix 2 sum J J^T built from the per-ray
  pose Jacobians (the gradient's sums before weighting), so each iteration
  is one launch and converges quadratically near the optimum.  Optionally
  coarse to fine: the same iterations first on a resolution pyramid
  (`coarsen`: volume averaged over 2x2x2 voxels, targets binned 2x2, an
  eighth of the samples per level), the full-resolution problem only for
  the last few steps.

Losses: SSD, or NCC (the paper's registration loss), per view.
"""
from __future__ import annotations

import dataclasses
import math
import time
import types

import torch

from .autograd import ProjectFwd


def ncc_per_view(l: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Normalised cross-correlation of each view pair ([V][nv][nu] -> [V])."""
    lv = l.reshape(l.shape[0], -1).to(torch.float64)
    yv = y.reshape(y.shape[0], -1).to(torch.float64)
    lv = lv - lv.mean(dim=1, keepdim=True)
    yv = yv - yv.mean(dim=1, keepdim=True)
    return (lv * yv).sum(1) / (lv.norm(dim=1) * yv.norm(dim=1) + 1e-30)


def loss_per_view(l, y, kind: str):
    if kind == "ssd":
        return ((l.to(torch.float64) - y.to(torch.float64)) ** 2).reshape(l.shape[0], -1).sum(1)
    if kind == "ncc":
        return 1.0 - ncc_per_view(l, y)
    raise ValueError(f"unknown loss {kind}")


@dataclasses.dataclass
class RegistrationResult:
    poses: torch.Tensor          # [B][6] final estimates
    iterations: torch.Tensor     # [B] iterations each registration ran
    converged: torch.Tensor      # [B] stopping rule met
    final_loss: torch.Tensor     # [B]
    seconds: float
    launches: int                # forward + gradient launch pairs
    ncc: torch.Tensor | None = None     # [B] NCC at the last evaluation (stop="paper")
    failed: torch.Tensor | None = None  # [B] NCC < 0.99 at the end (stop="paper")
    level_launches: list | None = None  # launches per pyramid level, finest first


def pose_errors(est: torch.Tensor, truth: torch.Tensor):
    """Max abs translation error (mm) and max abs rotation error (deg) per registration."""
    d = (est - truth).abs()
    return d[:, :3].max(dim=1).values, torch.rad2deg(d[:, 3:].max(dim=1).values)


def success(est, truth, t_tol_mm=0.1, r_tol_deg=0.1):
    et, er = pose_errors(est, truth)
    return (et < t_tol_mm) & (er < r_tol_deg)


def register(geom, vol, angles, targets, init_poses, loss="ssd", iters=300, lr_t=2.0,
             lr_r_deg=2.0, decay=0.985, min_lr_frac=0.01, tol_t=1e-3, tol_r_deg=1e-3,
             patience=5, compact_every=10, betas=(0.9, 0.999), eps=1e-12,
             project=None, stop="step", dloss_tol=1e-5, ncc_stop=0.999,
             ncc_fail=0.99) -> RegistrationResult:
    """Register every target image to the volume, starting from init_poses.

    geom: projector geometry; vol [nz][ny][nx] f32; angles [B] f64;
    targets [B][nv][nu] f32; init_poses [B][6] f64 (all on the GPU).
    `project` overrides the differentiable projector (defaults to ProjectFwd).
    stop: "step" (updates below tol_t / tol_r_deg for `patience` iterations)
    or "paper" (|loss change| < dloss_tol or NCC > ncc_stop; NCC < ncc_fail
    at the end marks a failure).
    """
    if stop not in ("step", "paper"):
        raise ValueError(f"unknown stopping rule {stop}")
    proj_fn = project or (lambda p, a: ProjectFwd.apply(p, vol, geom, a))
    B = init_poses.shape[0]
    dev = init_poses.device
    poses = init_poses.detach().clone().to(torch.float64)
    lr = torch.tensor([lr_t] * 3 + [math.radians(lr_r_deg)] * 3, dtype=torch.float64, device=dev)
    tol = torch.tensor([tol_t] * 3 + [math.radians(tol_r_deg)] * 3, dtype=torch.float64, device=dev)
    m = torch.zeros_like(poses)
    v = torch.zeros_like(poses)
    its = torch.zeros(B, dtype=torch.int64, device=dev)
    calm = torch.zeros(B, dtype=torch.int64, device=dev)
    done = torch.zeros(B, dtype=torch.bool, device=dev)
    last_loss = torch.zeros(B, dtype=torch.float64, device=dev)
    ncc = torch.zeros(B, dtype=torch.float64, device=dev)
    active = torch.arange(B, device=dev)
    launches = 0
    t0 = time.perf_counter()
    for it in range(iters):
        if active.numel() == 0:
            break
        p = poses[active].clone().requires_grad_(True)
        l = proj_fn(p, angles[active])
        L = loss_per_view(l, targets[active], loss)
        L.sum().backward()
        launches += 1
        g = p.grad.detach()
        with torch.no_grad():
            k = its[active] + 1
            ma = betas[0] * m[active] + (1 - betas[0]) * g
            va = betas[1] * v[active] + (1 - betas[1]) * g * g
            mh = ma / (1 - betas[0] ** k.to(torch.float64))[:, None]
            vh = va / (1 - betas[1] ** k.to(torch.float64))[:, None]
            scale = max(decay ** it, min_lr_frac)
            upd = lr * scale * mh / (vh.sqrt() + eps)
            poses[active] = p.detach() - upd
            m[active], v[active], its[active] = ma, va, k
            if stop == "paper":
                # the rule judges the pose just evaluated: freeze it there
                c = ncc_per_view(l.detach(), targets[active])
                stalled = (k > 1) & ((L.detach() - last_loss[active]).abs() < dloss_tol)
                hit = stalled | (c > ncc_stop)
                poses[active] = torch.where(hit[:, None], p.detach(), poses[active])
                ncc[active] = c
                done[active] = hit
            else:
                small = (upd.abs() < tol).all(dim=1)
                calm[active] = torch.where(small, calm[active] + 1, torch.zeros_like(calm[active]))
                done[active] = calm[active] >= patience
            last_loss[active] = L.detach()
            # the paper's rule freezes a registration at the pose it judged
            if stop == "paper" or (it + 1) % compact_every == 0:
                active = active[~done[active]]
    torch.cuda.synchronize(dev) if dev.type == "cuda" else None
    res = RegistrationResult(poses=poses, iterations=its, converged=done, final_loss=last_loss,
                             seconds=time.perf_counter() - t0, launches=launches)
    if stop == "paper":
        res.ncc = ncc
        res.failed = ncc < ncc_fail
    return res


def autotune_registration(geom, vol, angles, poses, targets, reps=3):
    """Autotune the registration kernels (the single-pass SSD kernel, and the
    forward and pose-gradient kernels used by other losses) for every
    view-count octave a batched registration of len(poses) problems passes
    through while it drops converged registrations (the variant cache is
    keyed by octave).  Returns {views: (ssd, fwd, grad variants)}."""
    from . import OP_FWD, OP_FWD_GRAD, OP_FWD_SSD, autotune
    B = poses.shape[0]
    chosen = {}
    v = B
    while v >= 1:
        proj = torch.empty((v, geom.nv, geom.nu), dtype=torch.float32, device=vol.device)
        gp = torch.empty((v, 6), dtype=torch.float64, device=vol.device)
        a, p, y = angles[:v].contiguous(), poses[:v].contiguous(), targets[:v].contiguous()
        bs, _ = autotune(OP_FWD_SSD, geom, a, p, vol, proj, grad_proj=y, reps=reps)
        bf, _ = autotune(OP_FWD, geom, a, p, vol, proj, reps=reps)
        bg, _ = autotune(OP_FWD_GRAD, geom, a, p, vol, gp, grad_proj=y, reps=reps)
        chosen[v] = (bs, bf, bg)
        v //= 2
    return chosen


def _fused_ssd(geom, vol):
    """Loss and pose gradient of the SSD from the single-pass kernel."""
    from . import project_fwd_ssd_grad_pose

    def fn(poses, angles, targets):
        _, L, g = project_fwd_ssd_grad_pose(geom, angles.contiguous(), poses.contiguous(), vol,
                                            targets.contiguous())
        return L, g
    return fn


def _loss_and_grad(proj_fn, poses, angles, targets, loss):
    if callable(loss):
        return loss(poses.detach().to(torch.float64).contiguous(), angles, targets)
    p = poses.detach().clone().requires_grad_(True)
    l = proj_fn(p, angles)
    L = loss_per_view(l, targets, loss)
    L.sum().backward()
    return L.detach(), p.grad.detach()


def register_bfgs(geom, vol, angles, targets, init_poses, loss="ssd", iters=150,
                  first_step=2.0, max_step=4.0, c1=1e-4, shrink=0.3, tol=1e-4,
                  min_scale=1e-4, project=None) -> RegistrationResult:
    """Batched BFGS registration of every target image, from init_poses.

    Parameters are scaled to z = (t / 1 mm, gamma / 1 deg).  Each iteration
    evaluates loss and analytic gradient at the trial point z + d,
    d = -scale H g (|d| capped at max_step), for all active registrations in
    one launch pair; the inverse-Hessian estimate H is updated from
    (s, y) = (d, g_trial - g) whenever s.y > 0 (the first update rescales
    H to s.y / y.y), and the trial point is accepted if it satisfies the
    Armijo condition f_trial <= f + c1 g.d (scale reset to 1), otherwise
    scale *= shrink.  A registration stops once an accepted step is below
    tol in every scaled parameter, or when scale falls below min_scale
    (no further decrease resolvable in FP32).  The first step has length
    first_step along the negative gradient.  With the default projector and
    the SSD loss, loss and gradient come from the single-pass kernel.
    """
    proj_fn = project or (lambda p, a: ProjectFwd.apply(p, vol, geom, a))
    if project is None and loss == "ssd":
        loss = _fused_ssd(geom, vol)
    B = init_poses.shape[0]
    dev = init_poses.device
    f64 = torch.float64
    D = torch.tensor([1.0] * 3 + [math.radians(1.0)] * 3, dtype=f64, device=dev)
    z = (init_poses.detach().to(f64) / D).clone()
    t0 = time.perf_counter()
    f, g = _loss_and_grad(proj_fn, z * D, angles, targets, loss)
    g = g * D
    launches = 1
    eye = torch.eye(6, dtype=f64, device=dev)
    gn = g.norm(dim=1).clamp_min(1e-300)
    H = eye.expand(B, 6, 6) * (first_step / gn)[:, None, None]
    scale = torch.ones(B, dtype=f64, device=dev)
    fresh = torch.ones(B, dtype=torch.bool, device=dev)
    done = gn <= 1e-300
    its = torch.zeros(B, dtype=torch.int64, device=dev)
    active = torch.nonzero(~done).flatten()
    for _ in range(iters):
        if active.numel() == 0:
            break
        za, fa, ga, Ha, sc = z[active], f[active], g[active], H[active], scale[active]
        d = -torch.einsum("bij,bj->bi", Ha, ga) * sc[:, None]
        dn = d.norm(dim=1)
        d = d * torch.clamp(max_step / dn.clamp_min(1e-300), max=1.0)[:, None]
        ft, gt = _loss_and_grad(proj_fn, (za + d) * D, angles[active], targets[active], loss)
        gt = gt * D
        launches += 1
        with torch.no_grad():
            y = gt - ga
            sy = (d * y).sum(1)
            upd = sy > 1e-12 * d.norm(dim=1) * y.norm(dim=1)
            Hs = torch.where((fresh[active] & upd)[:, None, None],
                             eye * (sy / (y * y).sum(1).clamp_min(1e-300))[:, None, None], Ha)
            rho = torch.where(upd, 1.0 / sy.where(upd, torch.ones_like(sy)), torch.zeros_like(sy))
            Lm = eye - rho[:, None, None] * d[:, :, None] * y[:, None, :]
            Hn = Lm @ Hs @ Lm.transpose(1, 2) + rho[:, None, None] * d[:, :, None] * d[:, None, :]
            H[active] = torch.where(upd[:, None, None], Hn, Ha)
            fresh[active] = fresh[active] & ~upd
            acc = ft <= fa + c1 * (ga * d).sum(1)
            z[active] = torch.where(acc[:, None], za + d, za)
            f[active] = torch.where(acc, ft, fa)
            g[active] = torch.where(acc[:, None], gt, ga)
            scale[active] = torch.where(acc, torch.ones_like(sc), sc * shrink)
            its[active] += 1
            stop = (acc & (d.abs().max(dim=1).values < tol)) | (scale[active] < min_scale)
            done[active] = stop
            active = active[~stop]
    if dev.type == "cuda":
        torch.cuda.synchronize(dev)
    return RegistrationResult(poses=z * D, iterations=its, converged=done, final_loss=f,
                              seconds=time.perf_counter() - t0, launches=launches)


def coarsen(geom, vol, targets):
    """One level down a resolution pyramid: the volume averaged over 2x2x2
    voxels, every target averaged over 2x2 pixels (detector binning: the mean
    of four line integrals stands for the one through the binned pixel's
    centre), and the geometry with doubled voxel and pixel sizes, halved
    detector offsets (in pixels) and a doubled march step.  Voxel and pixel
    centres of the coarse grids are the centroids of the fine cells they
    replace, so both levels describe the same object and detector.  Every
    grid dimension must be even.  Returns (geom, vol, targets)."""
    from . import DPGeom
    dims = (geom.nx, geom.ny, geom.nz, geom.nu, geom.nv)
    if any(n % 2 or n < 2 for n in dims):
        raise ValueError(f"coarsen needs even grid sizes, got {dims}")
    fields = {f: getattr(geom, f) for f, _ in DPGeom._fields_}
    fields.update(nx=geom.nx // 2, ny=geom.ny // 2, nz=geom.nz // 2, vx=2 * geom.vx,
                  vy=2 * geom.vy, vz=2 * geom.vz, nu=geom.nu // 2, nv=geom.nv // 2,
                  du=2 * geom.du, dv=2 * geom.dv, off_u=geom.off_u / 2, off_v=geom.off_v / 2,
                  step=2 * geom.step)
    gc = (dataclasses.replace(geom, **fields) if dataclasses.is_dataclass(geom)
          else types.SimpleNamespace(**fields))
    F = torch.nn.functional
    vc = F.avg_pool3d(vol[None, None], 2)[0, 0].contiguous()
    yc = F.avg_pool2d(targets[:, None], 2)[:, 0].contiguous()
    return gc, vc, yc


def register_lm(geom, vol, angles, targets, init_poses, iters=60, lam0=1e-3, up=4.0, down=3.0,
                tol=1e-4, lam_max=1e10, rule="step", levels=0,
                coarse_tol=None) -> RegistrationResult:
    """Batched Levenberg-Marquardt registration on the SSD.

    Each launch evaluates, at one point per registration, the DRR, the SSD
    f, its analytic pose gradient g and the Gauss-Newton matrix
    H = 2 sum J J^T (one pass of the fused kernel).  In the scaled
    parameters z = (t / 1 mm, gamma / 1 deg) the step solves
    (H + lam diag(H)) d = -g; the next launch evaluates z + d, which is
    accepted if the SSD decreased (lam /= down) and otherwise discarded
    (lam *= up, the previous f, g, H kept).  A registration stops when lam
    exceeds lam_max (no decrease resolvable in FP32) or, with rule="step",
    once an accepted step is below tol in every scaled parameter; with
    rule="newton", once the undamped Gauss-Newton step -H^-1 g at the
    accepted point is below tol in every scaled parameter (near the optimum
    that step is the remaining distance, so the evaluation that would only
    confirm convergence is skipped; the rule is also applied at the starting
    point).

    levels > 0 runs coarse to fine: the same method first on the problem
    `coarsen`ed `levels` times (stopping with coarse_tol, default tol), each
    finer level starting from the coarser level's poses.  The coarse optimum
    is biased by the lost detail, so only the full-resolution stage decides
    the result; it starts close to it and needs a launch or two.  The
    result's time and launches cover every level (level_launches splits
    them, finest first).
    """
    if rule not in ("step", "newton"):
        raise ValueError(f"unknown stopping rule {rule}")
    if levels > 0:
        t0 = time.perf_counter()
        gc, vc, yc = coarsen(geom, vol, targets)
        ct = tol if coarse_tol is None else coarse_tol
        c = register_lm(gc, vc, angles, yc, init_poses, iters, lam0, up, down, ct, lam_max, rule,
                        levels - 1, coarse_tol)
        r = register_lm(geom, vol, angles, targets, c.poses, iters, lam0, up, down, tol, lam_max,
                        rule)
        if init_poses.device.type == "cuda":
            torch.cuda.synchronize(init_poses.device)
        return RegistrationResult(poses=r.poses, iterations=r.iterations + c.iterations,
                                  converged=r.converged, final_loss=r.final_loss,
                                  seconds=time.perf_counter() - t0,
                                  launches=r.launches + c.launches,
                                  level_launches=[r.launches] + c.level_launches)
    from . import project_fwd_ssd_gauss_newton
    B = init_poses.shape[0]
    dev = init_poses.device
    f64 = torch.float64
    D = torch.tensor([1.0] * 3 + [math.radians(1.0)] * 3, dtype=f64, device=dev)
    DD = D[:, None] * D[None, :]

    def evaluate(z, idx):
        _, L, g, H = project_fwd_ssd_gauss_newton(geom, angles[idx].contiguous(),
                                                  (z * D).contiguous(), vol,
                                                  targets[idx].contiguous())
        return L, g * D, H * DD

    eye = torch.eye(6, dtype=f64, device=dev)

    def newton_small(Hn, gn):
        reg = 1e-12 * (torch.diagonal(Hn, dim1=1, dim2=2)[:, :, None] + 1.0) * eye
        return torch.linalg.solve(Hn + reg, -gn).abs().max(dim=1).values < tol

    t0 = time.perf_counter()
    z = (init_poses.detach().to(f64) / D).clone()
    allidx = torch.arange(B, device=dev)
    f, g, H = evaluate(z, allidx)
    launches = 1
    lam = torch.full((B,), lam0, dtype=f64, device=dev)
    its = torch.zeros(B, dtype=torch.int64, device=dev)
    done = torch.zeros(B, dtype=torch.bool, device=dev)
    if rule == "newton":
        done = newton_small(H, g)
    active = allidx[~done]
    for _ in range(iters):
        if active.numel() == 0:
            break
        Ha, ga = H[active], g[active]
        A = Ha + lam[active, None, None] * (torch.diagonal(Ha, dim1=1, dim2=2)[:, :, None] * eye
                                            + 1e-12 * eye)
        d = torch.linalg.solve(A, -ga)
        zt = z[active] + d
        ft, gt, Ht = evaluate(zt, active)
        launches += 1
        with torch.no_grad():
            acc = ft < f[active]
            z[active] = torch.where(acc[:, None], zt, z[active])
            f[active] = torch.where(acc, ft, f[active])
            g[active] = torch.where(acc[:, None], gt, ga)
            H[active] = torch.where(acc[:, None, None], Ht, Ha)
            lam[active] = torch.where(acc, lam[active] / down, lam[active] * up)
            its[active] += 1
            if rule == "step":
                small = acc & (d.abs().max(dim=1).values < tol)
            else:
                small = newton_small(H[active], g[active])
            stop = small | (lam[active] > lam_max)
            done[active] = stop
            active = active[~stop]
    if dev.type == "cuda":
        torch.cuda.synchronize(dev)
    return RegistrationResult(poses=z * D, iterations=its, converged=done, final_loss=f,
                              seconds=time.perf_counter() - t0, launches=launches,
                              level_launches=[launches])


class BatchLM:
    """Levenberg-Marquardt registration of an uneven batch of problems (each
    with its own volume, geometry and views; every view its own 6-DoF pose)
    that runs entirely on the device.  More than 16 problems run as
    consecutive batch launches of 16 sharing one workspace.

    One iteration is two library launches: the single-pass SSD batch
    (DRR, per-view SSD, analytic pose gradient and Gauss-Newton matrix for
    every view of every problem in one ray launch) and the FP64 update
    kernel (accept/reject against the last accepted point, damped 6 x 6
    Cholesky solve, next trial pose).  No host round trip, no allocation,
    so `capture()` records one iteration into a HIP graph that `run()`
    replays.  Same rule as `register_lm`: scaled parameters
    z = (t / 1 mm, gamma / 1 deg), step (H + lam diag H) d = -g, lam /= 3 on
    accept, *= 4 on reject; a view stops when an accepted step is below tol
    in every scaled parameter or lam exceeds 1e10.

    problems: list of dicts with geom, angles [V] f64, vol [nz][ny][nx] f32
    and target [V][nv][nu] f32 (CUDA tensors).
    """

    def __init__(self, problems, init_poses, lam0=1e-3, tol=1e-4, variant=-1, stream=None):
        from . import OP_FWD_SSD, batch_workspace_bytes
        f64 = torch.float64
        dev = problems[0]["vol"].device
        counts = [int(q["angles"].numel()) for q in problems]
        self.n = sum(counts)
        self.lam0, self.tol, self.variant, self.stream = lam0, tol, variant, stream
        self.trial = torch.empty((self.n, 6), dtype=f64, device=dev)
        self.loss = torch.empty(self.n, dtype=f64, device=dev)
        self.grad = torch.empty((self.n, 6), dtype=f64, device=dev)
        self.hess = torch.empty((self.n, 21), dtype=f64, device=dev)
        self.state = dict(pose=torch.empty((self.n, 6), dtype=f64, device=dev),
                          f=torch.empty(self.n, dtype=f64, device=dev),
                          g=torch.zeros((self.n, 6), dtype=f64, device=dev),
                          h=torch.zeros((self.n, 21), dtype=f64, device=dev),
                          lam=torch.empty(self.n, dtype=f64, device=dev),
                          done=torch.empty(self.n, dtype=torch.int32, device=dev))
        self.problems = []
        a = 0
        for q, V in zip(problems, counts):
            g = q["geom"]
            self.problems.append(dict(
                geom=g, angles=q["angles"], vol=q["vol"], target=q["target"],
                poses=self.trial[a:a + V], grad_pose=self.grad[a:a + V],
                hess=self.hess[a:a + V], loss=self.loss[a:a + V],
                proj=torch.empty((V, g.nv, g.nu), dtype=torch.float32, device=dev)))
            a += V
        need = batch_workspace_bytes(self.problems, OP_FWD_SSD)
        if need == 0:
            raise ValueError("invalid batch (geometry or sizes rejected by the library)")
        self.ws = torch.empty(need, dtype=torch.uint8, device=dev)
        self.graph = None
        self.reset(init_poses)

    def reset(self, init_poses):
        """Start again from init_poses [n][6] (all views, problem by problem)."""
        self.trial.copy_(init_poses)
        self.state["pose"].copy_(init_poses)
        self.state["f"].fill_(math.inf)
        self.state["lam"].fill_(self.lam0)
        self.state["done"].zero_()

    def step(self, stream=None):
        """One iteration: evaluate the trial poses, update the state."""
        from . import lm_update, project_fwd_ssd_gauss_newton_batch
        st = stream if stream is not None else self.stream
        project_fwd_ssd_gauss_newton_batch(self.problems, ws=self.ws, variant=self.variant, stream=st)
        lm_update(self.trial, self.loss, self.grad, self.hess, self.state, tol=self.tol, stream=st)

    def step_sequential(self, ws, stream=None):
        """The same iteration with one single-problem SSD launch per problem
        (ws: a workspace large enough for the largest problem)."""
        from . import lm_update, project_fwd_ssd_gauss_newton
        st = stream if stream is not None else self.stream
        for q in self.problems:
            project_fwd_ssd_gauss_newton(q["geom"], q["angles"], q["poses"], q["vol"], q["target"],
                                         proj=q["proj"], loss=q["loss"], grad=q["grad_pose"],
                                         hess=q["hess"], ws=ws, stream=st, packed=True)
        lm_update(self.trial, self.loss, self.grad, self.hess, self.state, tol=self.tol, stream=st)

    def capture(self):
        """Record one iteration into a HIP graph (after one eager warm-up
        iteration on a side stream; the state is restored afterwards)."""
        saved = {k: v.clone() for k, v in self.state.items()}
        trial = self.trial.clone()
        s2 = torch.cuda.Stream()
        s2.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s2):
            self.step(torch.cuda.current_stream())
        torch.cuda.current_stream().wait_stream(s2)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.step(torch.cuda.current_stream())
        for k, v in saved.items():
            self.state[k].copy_(v)
        self.trial.copy_(trial)

    def run(self, iters, graph=True):
        """iters iterations (graph replays if captured and graph=True)."""
        for _ in range(iters):
            if graph and self.graph is not None:
                self.graph.replay()
            else:
                self.step()

    def result(self):
        """(accepted poses [n][6], converged [n] bool, SSD at the accepted poses [n])."""
        return (self.state["pose"].clone(), self.state["done"].bool(), self.state["f"].clone())
