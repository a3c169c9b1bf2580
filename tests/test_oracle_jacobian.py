"""Pins for the oracle's per-ray pose Jacobian and the SSD Gauss-Newton
matrix built from it: central finite differences of the forward projection
(the derivative of the imaging model itself, to the discretisation accuracy
the paper reports for its gradients, Sec. III-A), and exactness of the
Gauss-Newton model for a pose-linear residual."""
import math

import numpy as np

import oracle
import synth
from synth import Geom


def _case():
    rng = synth.rng_for(600)
    g = Geom(40, 40, 40, 1.5, 1.5, 1.5, 48, 40, 2.0, 2.0)
    vol = synth.ellipsoid_phantom(40, 1.5, 8, rng)
    angles = np.array([0.3, 2.1])
    poses = synth.random_poses(2, 3.0, 4.0, rng)
    return g, vol, angles, poses


def test_jacobian_columns_match_finite_differences():
    """Each column dl/dtheta_c (an image) against central differences of the
    oracle's projections (h = 1e-3 mm / rad).  The analytic form
    differentiates the central-difference gradient field while the sampled
    model's true derivative follows the trilinear interpolant, so the
    columns agree at the method's discretisation level (Sec. III-A), not to
    rounding: cosine >= 0.985 and norm within 7 % per view and parameter,
    mean cosine >= 0.99 (measured 0.987-0.9997, mean 0.9945).  A sign,
    axis or frame slip in any column drops its cosine far below that."""
    g, vol, angles, poses = _case()
    J = oracle.project_fwd_jacobian(g, angles, poses, vol)
    h = 1e-3
    coss = []
    for c in range(6):
        dp = poses.copy()
        dm = poses.copy()
        dp[:, c] += h
        dm[:, c] -= h
        fd = (oracle.project_fwd(g, angles, dp, vol) - oracle.project_fwd(g, angles, dm, vol)) / (2 * h)
        for v in range(len(angles)):
            a, b = J[v, :, :, c].ravel(), fd[v].ravel()
            cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
            ratio = np.linalg.norm(a) / np.linalg.norm(b)
            coss.append(cos)
            assert cos >= 0.985 and abs(ratio - 1) < 0.07, (c, v, cos, ratio)
    assert np.mean(coss) >= 0.99


def test_weighted_jacobian_sum_is_the_pose_gradient():
    """sum_rays w J = dL/dtheta for an arbitrary dL/dl = w (the two oracle
    routes contract the same sums in different orders)."""
    g, vol, angles, poses = _case()
    J = oracle.project_fwd_jacobian(g, angles, poses, vol)
    w = np.random.default_rng(1).standard_normal((2, g.nv, g.nu))
    ref = oracle.project_fwd_grad_pose(g, angles, poses, vol, w)
    got = np.einsum("vbac,vba->vc", J, w)
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_gauss_newton_matrix_predicts_a_small_step():
    """For a small pose step d the SSD to the projections at poses + d is
    d^T H d / 2 to second order (zero residual at d = 0).  The analytic J
    carries the few-percent discretisation bias measured above, so the
    model is held to 10 % at two step sizes (measured ~5 % at both)."""
    g, vol, angles, poses = _case()
    H = oracle.gauss_newton_ssd(g, angles, poses, vol)
    assert np.allclose(H, np.transpose(H, (0, 2, 1)))
    assert np.all(np.linalg.eigvalsh(H) > 0)
    d = np.array([0.2, -0.1, 0.15, math.radians(0.2), math.radians(-0.1), math.radians(0.15)])
    base = oracle.project_fwd(g, angles, poses, vol)
    errs = []
    for s in (1.0, 0.5):
        l = oracle.project_fwd(g, angles, poses + s * d, vol)
        ssd = ((l - base) ** 2).reshape(2, -1).sum(1)
        model = 0.5 * np.einsum("i,vij,j->v", s * d, H, s * d)
        errs.append(np.abs(ssd - model) / model)
    assert np.all(errs[0] < 0.1) and np.all(errs[1] < 0.1)
