"""Motion-compensated FDK reconstruction (the paper's motion-compensated
analytical reconstruction task, Sec. III-B): estimate per-view rigid poses
theta by minimising an image-sharpness loss of the FDK reconstruction
mu(theta) = A^T(M(theta)) Ramp(l), with the analytic back-projection pose
gradient (Eqs. final_back / dis_back) as the gradient of the reconstruction
with respect to theta.

One iteration: back-project the pre-filtered projections at the current
poses (FDK weight), evaluate the loss and dL/dmu on the volume, back-project
the pose gradient, and take an Adam step.  The poses follow a motion model
theta = B c (B = identity for independent per-view poses, or a periodic
piecewise-linear interpolation over K nodes); the gradient is projected to
zero mean over the views, because a rigid motion common to all views only
moves the reconstruction and is not observable from sharpness.
"""
from __future__ import annotations

import dataclasses
import math
import time

import torch

from . import W_FDK, backproject, backproject_grad_pose, fdk_filter, gradient_entropy, sharpness


def motion_basis(n_views: int, nodes: int, device) -> torch.Tensor:
    """[V][K] periodic piecewise-linear interpolation from K equally spaced
    nodes over the orbit (K = 0: identity, independent per-view poses)."""
    if nodes <= 0:
        return torch.eye(n_views, dtype=torch.float64, device=device)
    B = torch.zeros((n_views, nodes), dtype=torch.float64)
    for v in range(n_views):
        x = v * nodes / n_views
        k0 = int(math.floor(x))
        f = x - k0
        B[v, k0 % nodes] += 1.0 - f
        B[v, (k0 + 1) % nodes] += f
    return B.to(device)


def sharpness_loss(vol):
    """The negative sum of squared forward differences and its gradient (library kernel)."""
    return sharpness(vol)


def gradient_entropy_loss(vol):
    """Gradient entropy (the paper's sharpness criterion) and its gradient (library kernel)."""
    return gradient_entropy(vol)


@dataclasses.dataclass
class MocoResult:
    poses: torch.Tensor        # [V][6] final estimate
    losses: list               # loss per iteration (before the step)
    seconds: float


def reconstruct(geom, angles, poses, q, out=None, ws=None):
    """FDK reconstruction of pre-filtered projections q at the given poses."""
    return backproject(geom, angles, poses, q, W_FDK, out=out, ws=ws)


def prefilter(geom, proj):
    """FDK pre-filter for a full circular orbit of len(proj) views."""
    return fdk_filter(geom, proj, math.pi / proj.shape[0])


def estimate_motion(geom, angles, q, iters=80, nodes=0, lr_t=0.1, lr_r_deg=0.07,
                    loss=gradient_entropy_loss, init=None, betas=(0.9, 0.999), decay=1.0,
                    callback=None) -> MocoResult:
    """Minimise loss(reconstruct(theta)) over theta = B c with Adam (step
    sizes lr_t mm and lr_r_deg deg, multiplied by decay**iteration).

    geom: reconstruction grid + detector; angles [V] f64; q [V][nv][nu] f32
    pre-filtered projections; loss(vol) -> (0-d loss tensor, dL/dvol f32).
    """
    dev = q.device
    V = q.shape[0]
    B = motion_basis(V, nodes, dev)
    c = torch.zeros((B.shape[1], 6), dtype=torch.float64, device=dev)
    base = torch.zeros((V, 6), dtype=torch.float64, device=dev) if init is None else init.clone()
    lr = torch.tensor([lr_t] * 3 + [math.radians(lr_r_deg)] * 3, dtype=torch.float64, device=dev)
    m = torch.zeros_like(c)
    v2 = torch.zeros_like(c)
    vol = torch.empty((geom.nz, geom.ny, geom.nx), dtype=torch.float32, device=dev)
    gp = torch.empty((V, 6), dtype=torch.float64, device=dev)
    losses = []
    t0 = time.perf_counter()
    for it in range(iters):
        poses = (base + B @ c).contiguous()
        reconstruct(geom, angles, poses, q, out=vol)
        L, e = loss(vol)
        backproject_grad_pose(geom, angles, poses, q, e, W_FDK, out=gp)
        gc = B.T @ gp
        gc = gc - gc.mean(dim=0, keepdim=True)
        k = it + 1
        m.mul_(betas[0]).add_(gc, alpha=1 - betas[0])
        v2.mul_(betas[1]).addcmul_(gc, gc, value=1 - betas[1])
        c -= (decay ** it) * lr * (m / (1 - betas[0] ** k)) / ((v2 / (1 - betas[1] ** k)).sqrt() + 1e-300)
        losses.append(float(L))
        if callback:
            callback(it, float(L), base + B @ c)
    torch.cuda.synchronize(dev)
    return MocoResult(poses=(base + B @ c), losses=losses, seconds=time.perf_counter() - t0)


def demeaned_rms_error(est, truth):
    """RMS over views of the pose error after removing its mean over views
    (mm for translations, degrees for rotations)."""
    d = est - truth
    d = d - d.mean(dim=0, keepdim=True)
    return (float(d[:, :3].pow(2).mean().sqrt()),
            math.degrees(float(d[:, 3:].pow(2).mean().sqrt())))


def view_frame_errors(est, truth, angles):
    """RMS over views of the demeaned translation error resolved in each
    view's detector frame: along e_u (detector row), e_v (axial) and e_w
    (depth, towards the detector), in mm.  Depth translations barely change
    a view's contribution to the reconstruction."""
    d = est - truth
    d = d - d.mean(dim=0, keepdim=True)
    cb, sb = torch.cos(angles), torch.sin(angles)
    eu = torch.stack([-sb, cb, torch.zeros_like(cb)], dim=1)
    ew = torch.stack([-cb, -sb, torch.zeros_like(cb)], dim=1)
    t = d[:, :3]
    return (float((t * eu).sum(1).pow(2).mean().sqrt()), float(t[:, 2].pow(2).mean().sqrt()),
            float((t * ew).sum(1).pow(2).mean().sqrt()))
