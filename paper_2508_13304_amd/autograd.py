"""torch.autograd integration of the projector (the paper's PyTorch-compatible
interface, Sec. II-C: the gradient kernels plug into auto-differentiation).

ProjectFwd: DRRs as a differentiable function of the per-view poses; the
backward is the analytic pose gradient of Eqs. final_forward / dis_forward,
which recomputes the ray samples instead of storing them (Sec. IV).

Backproject: back-projected volume as a differentiable function of the
per-view poses; the backward is the analytic pose gradient of Eqs. final_back
/ dis_back.

Gradients with respect to the volume (forward) or the projections (back)
are not part of the method's motion gradients and are not provided: the
inputs must not require them.
"""
from __future__ import annotations

import torch

from . import backproject as _bp
from . import backproject_grad_pose as _bp_grad
from . import project_fwd as _fwd
from . import project_fwd_grad_pose as _fwd_grad


def _no_data_grad(t: torch.Tensor, name: str):
    if t.requires_grad:
        raise NotImplementedError(f"gradient with respect to {name} is not provided; "
                                  f"pass {name}.detach()")


class ProjectFwd(torch.autograd.Function):
    """l = A(M(theta)) mu;  dL/dtheta = analytic pose gradient given dL/dl."""

    @staticmethod
    def forward(ctx, poses, vol, geom, angles, ws=None):
        _no_data_grad(vol, "vol")
        ctx.geom = geom
        ctx.save_for_backward(poses, vol, angles)
        with torch.no_grad():
            return _fwd(geom, angles, poses.detach().contiguous(), vol, ws=ws)

    @staticmethod
    def backward(ctx, grad_l):
        poses, vol, angles = ctx.saved_tensors
        g = None
        if ctx.needs_input_grad[0]:
            g = _fwd_grad(ctx.geom, angles, poses.detach().contiguous(), vol,
                          grad_l.contiguous().to(torch.float32))
        return g, None, None, None, None


class Backproject(torch.autograd.Function):
    """mu = A^T(M(theta)) l;  dL/dtheta = analytic pose gradient given dL/dmu."""

    @staticmethod
    def forward(ctx, poses, proj, geom, angles, weight_mode=0, ws=None):
        _no_data_grad(proj, "proj")
        ctx.geom, ctx.mode = geom, weight_mode
        ctx.save_for_backward(poses, proj, angles)
        with torch.no_grad():
            return _bp(geom, angles, poses.detach().contiguous(), proj, weight_mode, ws=ws)

    @staticmethod
    def backward(ctx, grad_mu):
        poses, proj, angles = ctx.saved_tensors
        g = None
        if ctx.needs_input_grad[0]:
            g = _bp_grad(ctx.geom, angles, poses.detach().contiguous(), proj,
                         grad_mu.contiguous().to(torch.float32), ctx.mode)
        return g, None, None, None, None, None


def project(poses, vol, geom, angles):
    """Differentiable forward projection (poses [V][6] f64 -> DRRs [V][nv][nu] f32)."""
    return ProjectFwd.apply(poses, vol, geom, angles)


def backproject(poses, proj, geom, angles, weight_mode=0):
    """Differentiable back-projection (poses [V][6] f64 -> volume f32)."""
    return Backproject.apply(poses, proj, geom, angles, weight_mode)
