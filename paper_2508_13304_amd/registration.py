"""Batched gradient-based 2D/3D rigid registration (Sec. II-D, 2D/3D
registration task): estimate theta* = argmin_theta loss(A(M(theta)) mu, l)
for many independent registrations at once.

Each registration is one view of a single projector launch (its own gantry
angle, pose and target image), so one iteration costs one forward and one
pose-gradient launch for the whole batch.  The optimiser is Adam (as in the
paper) with separate step sizes for translations (mm) and rotations (deg),
a step-size decay, and per-registration stopping: a registration whose
largest update falls below a tolerance for a few consecutive iterations is
frozen and dropped from later launches.  Losses: SSD, or NCC (the paper's
registration loss), per view.
"""
from __future__ import annotations

import dataclasses
import math
import time

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
             project=None) -> RegistrationResult:
    """Register every target image to the volume, starting from init_poses.

    geom: projector geometry; vol [nz][ny][nx] f32; angles [B] f64;
    targets [B][nv][nu] f32; init_poses [B][6] f64 (all on the GPU).
    `project` overrides the differentiable projector (defaults to ProjectFwd).
    """
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
            last_loss[active] = L.detach()
            small = (upd.abs() < tol).all(dim=1)
            calm[active] = torch.where(small, calm[active] + 1, torch.zeros_like(calm[active]))
            done[active] = calm[active] >= patience
            if (it + 1) % compact_every == 0:
                active = active[~done[active]]
    torch.cuda.synchronize(dev) if dev.type == "cuda" else None
    return RegistrationResult(poses=poses, iterations=its, converged=done, final_loss=last_loss,
                              seconds=time.perf_counter() - t0, launches=launches)
