"""Pins for the FP64 oracle against facts that do not come from the oracle.

Each test ties one part of the oracle to something independent of its code:
a library routine (scipy rotations, scipy interpolation), a closed form, an
exact invariance (integer shifts, 90-degree rotations), an adjoint identity,
hand-derived worked examples (tests/golden), or central finite differences
of the oracle's own forward model (the method's gradient is an
approximation, so the finite-difference agreement is statistical, floored
by the accuracy the paper reports in Sec. III-A).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.ndimage import map_coordinates
from scipy.spatial.transform import Rotation

import synth
from synth import Geom

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))


def R_scipy(gamma):
    """R = Rz(gz) Ry(gy) Rx(gx): scipy's intrinsic Z-Y'-X'' Euler sequence."""
    return Rotation.from_euler("ZYX", [gamma[2], gamma[1], gamma[0]]).as_matrix()


# ---------------------------------------------------------------------------
# Pose algebra
# ---------------------------------------------------------------------------

def test_rotation_matches_scipy_zyx(oracle):
    rng = np.random.default_rng(1)
    for _ in range(20):
        gam = rng.uniform(-math.pi, math.pi, 3)
        np.testing.assert_allclose(oracle.rotation(gam), R_scipy(gam), atol=1e-14)


def test_rotation_partials_match_finite_differences(oracle):
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(10):
        gam = rng.uniform(-1, 1, 3)
        dR = oracle.rotation_partials(gam)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            fd = (R_scipy(gam + e) - R_scipy(gam - e)) / (2 * h)
            np.testing.assert_allclose(dR[a], fd, atol=1e-9)


def test_contraction_equals_omega_form(oracle):
    """Literal <dM/dtheta, dL/dM> equals the generator form dR/dg_a = [w_a]x R
    with w_x = Rz Ry e_x, w_y = Rz e_y, w_z = e_z (the form the GPU uses)."""
    rng = np.random.default_rng(3)
    for _ in range(10):
        pose = np.concatenate([rng.uniform(-5, 5, 3), rng.uniform(-1, 1, 3)])
        dLdM = rng.standard_normal((3, 4))
        got = oracle.contract_pose(pose, dLdM)
        gx, gy, gz = pose[3:]
        Rz = R_scipy([0, 0, gz])
        Ry = R_scipy([0, gy, 0])
        R = R_scipy(pose[3:])
        omegas = [Rz @ Ry @ np.array([1.0, 0, 0]), Rz @ np.array([0, 1.0, 0]), np.array([0, 0, 1.0])]

        def skew(w):
            return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])

        exp = np.concatenate([dLdM[:, 3], [np.sum((skew(w) @ R) * dLdM[:, :3]) for w in omegas]])
        np.testing.assert_allclose(got, exp, rtol=1e-12, atol=1e-12)


def test_pinhole_worked_example(oracle):
    gd = GOLD["pinhole"]
    g = Geom(1, 1, 1, 1, 1, 1, gd["geometry"]["nu"], gd["geometry"]["nv"], 1.5, 1.5)
    r = np.array(gd["point_mm"] + [1.0])
    for beta, key in ((0.0, "beta0_expected_ab"), (math.pi / 2, "beta90_expected_ab")):
        uvw = oracle.projection_matrix(g, beta) @ r
        np.testing.assert_allclose(uvw[:2] / uvw[2], gd[key], rtol=1e-13)


def test_projection_matrix_maps_pixel_rays(oracle):
    """Every point on the ray from the source through pixel centre (a, b)
    projects to (a, b); the source itself has depth 0 (Eq. projmatrix)."""
    g = Geom(1, 1, 1, 1, 1, 1, 37, 29, 0.7, 0.9, off_u=1.3, off_v=-2.1)
    rng = np.random.default_rng(4)
    for beta in rng.uniform(0, 2 * math.pi, 5):
        P = oracle.projection_matrix(g, beta)
        src = 1000.0 * np.array([math.cos(beta), math.sin(beta), 0.0])
        ew = -src / 1000.0
        eu = np.array([-math.sin(beta), math.cos(beta), 0.0])
        ev = np.array([0.0, 0.0, 1.0])
        assert abs(P[2] @ np.append(src, 1.0)) < 1e-9
        for a, b in [(0, 0), (36, 28), (17.5, 3.25)]:
            cu, cv = (g.nu - 1) / 2 + g.off_u, (g.nv - 1) / 2 + g.off_v
            q = src + 1500.0 * ew + (a - cu) * g.du * eu + (b - cv) * g.dv * ev
            for lam in (0.3, 0.66, 1.0):
                uvw = P @ np.append(src + lam * (q - src), 1.0)
                np.testing.assert_allclose(uvw[:2] / uvw[2], [a, b], atol=1e-9)


# ---------------------------------------------------------------------------
# Forward projector values
# ---------------------------------------------------------------------------

def _geom_cube(n, h, nu, nv, du=1.5):
    return Geom(n, n, n, h, h, h, nu, nv, du, du)


def test_single_voxel_worked_example(oracle):
    gd = GOLD["single_voxel_central_ray"]
    gg = gd["geometry"]
    g = _geom_cube(gg["n"], gg["h_mm"], gg["nu"], gg["nv"])
    vol = np.zeros(g.vol_shape)
    vol[2, 2, 2] = 1.0
    l = oracle.project_fwd(g, [0.0], np.zeros(6), vol)
    assert abs(l[0, 1, 1] - gd["expected_central_pixel"]) < 1e-12


@pytest.mark.parametrize("beta", [0.0, math.pi / 2, math.pi, 1.5 * math.pi])
def test_cube_chord_exact(oracle, beta):
    gd = GOLD["cube_chord"]
    gg = gd["geometry"]
    g = _geom_cube(gg["n"], gg["h_mm"], gg["nu"], gg["nv"])
    vol = np.zeros(g.vol_shape)
    vol[5:16, 5:16, 5:16] = 0.02
    l = oracle.project_fwd(g, [beta], np.zeros(6), vol)
    assert abs(l[0, 2, 2] - gd["expected_central_pixel"]) < 1e-12
    # An integer translation along the central ray leaves the chord unchanged.
    t = np.array([math.cos(beta), math.sin(beta), 0.0]) * 3.0
    l2 = oracle.project_fwd(g, [beta], np.concatenate([np.rint(t), np.zeros(3)]), vol)
    assert abs(l2[0, 2, 2] - gd["expected_central_pixel"]) < 1e-12


def test_sphere_chord_closed_form(oracle):
    """Chord 2 mu0 sqrt(rho^2 - d^2) through a partial-volume sphere."""
    n, h, rho, mu0 = 48, 1.0, 15.0, 0.03
    c = synth.voxel_centres(n, h)
    sub = (np.arange(4) + 0.5) / 4 - 0.5
    acc = np.zeros((n, n, n))
    for dz in sub:
        for dy in sub:
            for dx in sub:
                Z, Y, X = np.meshgrid(c + dz * h, c + dy * h, c + dx * h, indexing="ij")
                acc += (X ** 2 + Y ** 2 + Z ** 2) <= rho ** 2
    vol = mu0 * acc / 64.0
    g = Geom(n, n, n, h, h, h, 41, 41, 1.0, 1.0)
    l = oracle.project_fwd(g, [0.3], np.zeros(6), vol)[0]
    beta = 0.3
    src = 1000.0 * np.array([math.cos(beta), math.sin(beta), 0.0])
    ew, eu, ev = -src / 1000.0, np.array([-math.sin(beta), math.cos(beta), 0.0]), np.array([0, 0, 1.0])
    central = []
    for b in range(g.nv):
        for a in range(g.nu):
            q = src + 1500.0 * ew + (a - 20) * eu + (b - 20) * ev
            u = (q - src) / np.linalg.norm(q - src)
            d = np.linalg.norm(-src - np.dot(-src, u) * u)  # distance of the ray to the centre
            if d <= 0.8 * rho:
                exp = 2 * mu0 * math.sqrt(rho ** 2 - d ** 2)
                rel = (l[b, a] - exp) / exp
                # partial-volume + interpolation blur grows towards the rim
                assert abs(rel) <= (0.01 if d <= 0.6 * rho else 0.035), (a, b, l[b, a], exp)
                if d <= 0.5 * rho:
                    central.append(rel)
    assert len(central) > 100
    assert abs(np.mean(central)) < 3e-3  # no magnification / offset bias


def _brute_project(vol, g, beta, pose, rays):
    """Independent forward model: explicit geometry + scipy trilinear
    interpolation with zero extension (map_coordinates, grid-constant)."""
    R = R_scipy(pose[3:])
    t = np.asarray(pose[:3])
    src = g.sad * np.array([math.cos(beta), math.sin(beta), 0.0])
    ew = np.array([-math.cos(beta), -math.sin(beta), 0.0])
    eu = np.array([-math.sin(beta), math.cos(beta), 0.0])
    ev = np.array([0.0, 0.0, 1.0])
    cu, cv = (g.nu - 1) / 2 + g.off_u, (g.nv - 1) / 2 + g.off_v
    h = np.array([g.vx, g.vy, g.vz])
    cidx = (np.array([g.nx, g.ny, g.nz]) - 1) / 2
    k = np.arange(int((g.sad - 200) / g.step), int((g.sad + 200) / g.step))
    out = []
    for a, b in rays:
        q = src + g.sdd * ew + (a - cu) * g.du * eu + (b - cv) * g.dv * ev
        u = (q - src) / np.linalg.norm(q - src)
        r = src[None, :] + (k * g.step)[:, None] * u[None, :]
        rp = (r - t) @ R  # rows: R^T (r - t)
        X = rp / h + cidx
        inside = np.all((X > -1) & (X < np.array([g.nx, g.ny, g.nz])), axis=1)
        vals = map_coordinates(vol, [X[:, 2], X[:, 1], X[:, 0]], order=1, mode="grid-constant", cval=0.0)
        out.append(g.step * np.sum(vals[inside]))
    return np.array(out)


def test_forward_matches_library_interpolation(oracle):
    rng = synth.rng_for(100)
    g = Geom(20, 18, 16, 1.3, 1.1, 1.7, 24, 20, 2.0, 2.2, off_u=0.7, off_v=-1.2)
    vol = rng.uniform(0, 1, g.vol_shape)
    rays = [(a, b) for a in range(0, 24, 3) for b in range(0, 20, 3)]
    for beta, pose in [(0.0, np.zeros(6)), (1.1, np.array([3.0, -2.0, 1.5, 0.2, -0.3, 0.4]))]:
        l = oracle.project_fwd(g, [beta], pose, vol)[0]
        got = np.array([l[b, a] for a, b in rays])
        np.testing.assert_allclose(got, _brute_project(vol, g, beta, pose, rays), rtol=1e-12, atol=1e-12)


def test_integer_shift_invariance(oracle):
    g = _geom_cube(24, 1.5, 30, 30, du=2.0)
    vol = synth.ellipsoid_phantom(24, 1.5, 4, synth.rng_for(101))
    vol = np.asarray(vol, np.float64)
    n = (2, -1, 3)
    shifted = np.roll(vol, shift=(n[2], n[1], n[0]), axis=(0, 1, 2))
    pose = np.array([n[0] * 1.5, n[1] * 1.5, n[2] * 1.5, 0, 0, 0])
    for beta in (0.0, 0.7):
        a = oracle.project_fwd(g, [beta], pose, vol)
        b = oracle.project_fwd(g, [beta], np.zeros(6), shifted)
        np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-12)


def _rotate_volume_90(vol, gamma):
    """nu(r) = mu(R^T r) for a signed-permutation R (multiples of 90 deg)."""
    R = np.rint(R_scipy(gamma)).astype(int)
    n = vol.shape[0]
    c = (n - 1) / 2
    idx = np.arange(n) - c
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    P = np.stack([X, Y, Z], -1) @ R  # R^T r for each output voxel
    src = np.rint(P + c).astype(int)
    return vol[src[..., 2], src[..., 1], src[..., 0]]


@pytest.mark.parametrize("gamma_deg", [(90, 0, 0), (0, 90, 0), (0, 0, 90), (90, 0, 90), (0, 90, 90), (90, 90, 0)])
def test_quarter_turn_rotations_pin_order_and_signs(oracle, gamma_deg):
    n = 20
    g = _geom_cube(n, 1.0, 26, 26, du=1.5)
    rng = synth.rng_for(102)
    vol = np.zeros((n, n, n))
    vol[3:17, 3:17, 3:17] = rng.uniform(0, 1, (14, 14, 14))  # asymmetric content
    gam = np.deg2rad(gamma_deg)
    rot = _rotate_volume_90(vol, gam)
    for beta in (0.0, 0.4):
        a = oracle.project_fwd(g, [beta], np.concatenate([np.zeros(3), gam]), vol)
        b = oracle.project_fwd(g, [beta], np.zeros(6), rot)
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-11)


def test_adjoint_identity_rd(oracle):
    rng = synth.rng_for(103)
    g = Geom(12, 10, 9, 2.0, 2.5, 1.8, 16, 12, 3.0, 3.5)
    angles = [0.2, 2.0]
    poses = np.array([[1, -2, 0.5, 0.1, 0.2, -0.3], [-3, 1, 2, -0.2, 0.1, 0.5]])
    x = rng.standard_normal(g.vol_shape)
    y = rng.standard_normal(g.proj_shape(2))
    lhs = np.sum(oracle.project_fwd(g, angles, poses, x) * y)
    rhs = np.sum(x * oracle.project_fwd_T(g, angles, poses, y))
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1.0)


@pytest.mark.parametrize("mode", [0, 1])
def test_adjoint_identity_vd(oracle, mode):
    rng = synth.rng_for(104)
    g = Geom(12, 10, 9, 4.0, 4.5, 3.8, 20, 16, 6.0, 6.5)
    angles = [0.2, 2.0, 4.0]
    poses = synth.random_poses(3, 5.0, 5.0, rng)
    x = rng.standard_normal(g.vol_shape)
    y = rng.standard_normal(g.proj_shape(3))
    lhs = np.sum(oracle.vd_splat(g, angles, poses, x, mode) * y)
    rhs = np.sum(x * oracle.backproject(g, angles, poses, y, mode))
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1.0)


# ---------------------------------------------------------------------------
# Back-projector values
# ---------------------------------------------------------------------------

def test_backproject_constant_detector(oracle):
    g = Geom(10, 10, 10, 3.0, 3.0, 3.0, 40, 40, 3.0, 3.0)
    V = 5
    angles = synth.circular_angles(V)
    poses = synth.random_poses(V, 3.0, 3.0, synth.rng_for(105))
    proj = np.full(g.proj_shape(V), 0.7)
    mu = oracle.backproject(g, angles, poses, proj, 0)
    np.testing.assert_allclose(mu, 0.7 * V, rtol=1e-13)
    # FDK weight: sum_v (D / depth_v)^2 with depth = e_w . r + D, r = R p + t.
    mu_f = oracle.backproject(g, angles, poses, proj, 1)
    c = synth.voxel_centres(10, 3.0)
    for (i, j, k) in [(0, 0, 0), (9, 4, 2), (5, 5, 5)]:
        p = np.array([c[i], c[j], c[k]])
        exp = 0.0
        for v in range(V):
            r = R_scipy(poses[v, 3:]) @ p + poses[v, :3]
            depth = -math.cos(angles[v]) * r[0] - math.sin(angles[v]) * r[1] + 1000.0
            exp += 0.7 * (1000.0 / depth) ** 2
        assert abs(mu_f[k, j, i] - exp) < 1e-12 * exp


def test_backproject_single_pixel_hat(oracle):
    """A single unit pixel back-projects as the bilinear hat around the
    pinhole projection of each voxel (beta = 0, theta applied by scipy)."""
    g = Geom(12, 12, 12, 2.0, 2.0, 2.0, 31, 27, 1.5, 1.5)
    pose = np.array([1.0, -2.0, 0.5, 0.05, -0.1, 0.2])
    a_s, b_s = 16, 12
    proj = np.zeros(g.proj_shape(1))
    proj[0, b_s, a_s] = 1.0
    mu = oracle.backproject(g, [0.0], pose, proj, 0)
    c = synth.voxel_centres(12, 2.0)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r = np.stack([X, Y, Z], -1) @ R_scipy(pose[3:]).T + pose[:3]
    depth = 1000.0 - r[..., 0]
    a = 15.0 + 1500.0 * r[..., 1] / (depth * 1.5)
    b = 13.0 + 1500.0 * r[..., 2] / (depth * 1.5)
    exp = np.maximum(0, 1 - np.abs(a - a_s)) * np.maximum(0, 1 - np.abs(b - b_s))
    np.testing.assert_allclose(mu, exp, atol=1e-12)
    assert exp.max() > 0.3


def test_backproject_matches_library_interpolation(oracle):
    rng = synth.rng_for(106)
    g = Geom(9, 8, 7, 5.0, 5.0, 5.0, 22, 19, 4.0, 4.0, off_u=0.5)
    V = 3
    angles = [0.0, 1.0, 4.0]
    poses = synth.random_poses(V, 4.0, 4.0, rng)
    proj = rng.standard_normal(g.proj_shape(V))
    mu = oracle.backproject(g, angles, poses, proj, 1)
    c = [synth.voxel_centres(n, 5.0) for n in (9, 8, 7)]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    exp = np.zeros(g.vol_shape)
    for v in range(V):
        P = oracle.projection_matrix(g, angles[v])  # pinned above
        r = np.stack([X, Y, Z], -1) @ R_scipy(poses[v, 3:]).T + poses[v, :3]
        uvw = np.concatenate([r, np.ones(r.shape[:-1] + (1,))], -1) @ P.T
        A, B = uvw[..., 0] / uvw[..., 2], uvw[..., 1] / uvw[..., 2]
        val = map_coordinates(proj[v], [B.ravel(), A.ravel()], order=1, mode="grid-constant", cval=0.0)
        exp += (1000.0 / uvw[..., 2]) ** 2 * val.reshape(A.shape)
    np.testing.assert_allclose(mu, exp, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# Gradients
# ---------------------------------------------------------------------------

def _fd_geom():
    return Geom(24, 24, 24, 2.0, 2.0, 2.0, 32, 32, 3.0, 3.0)


def test_forward_grad_materialized_route_equals_fused(oracle):
    g = Geom(14, 13, 12, 2.0, 2.0, 2.0, 16, 14, 3.0, 3.0)
    rng = synth.rng_for(107)
    vol = synth.ellipsoid_phantom(14, 2.0, 4, rng)[:12, :13, :14]
    poses = synth.random_poses(2, 5, 5, rng)
    w = rng.standard_normal(g.proj_shape(2))
    a = oracle.project_fwd_grad_M(g, [0.1, 1.2], poses, vol, w)
    b = oracle.project_fwd_grad_M_materialized(g, [0.1, 1.2], poses, vol, w)
    np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-12 * np.abs(a).max())


def _cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def _triplet_agreement(ga, fd):
    """(cosine, norm ratio) of the translation and of the rotation triplet."""
    out = []
    for sl in (slice(0, 3), slice(3, 6)):
        out.append((_cos(ga[sl], fd[sl]), np.linalg.norm(ga[sl]) / np.linalg.norm(fd[sl])))
    return out


def _check_triplets(parts, floor):
    """A scale or sign slip confined to one triplet (translation or rotation)
    must fail even when the other triplet dominates the full vector."""
    parts = np.array(parts)  # [n][2 triplets][cos, ratio]
    for t in range(2):
        c, r = parts[:, t, 0], parts[:, t, 1]
        assert np.median(c) >= floor, (t, np.sort(c)[:5])
        assert abs(np.median(r) - 1.0) < 0.03, (t, np.median(r))


def _fd_steps():
    return np.array([1e-2] * 3 + [np.deg2rad(1e-2)] * 3)


def test_forward_grad_vs_central_fd(oracle):
    """O-FD1: analytic forward pose gradient vs central FD of the SSD loss."""
    g = _fd_geom()
    rng = synth.rng_for(108)
    vol = synth.ellipsoid_phantom(24, 2.0, 10, rng).astype(np.float64)
    n_real = 48
    poses = synth.random_poses(n_real, 10.0, 10.0, rng)
    targets = synth.random_poses(n_real, 10.0, 10.0, rng)
    betas = rng.uniform(0, 2 * math.pi, n_real)
    hs = _fd_steps()
    cos, parts = [], []
    for i in range(n_real):
        beta, th = [betas[i]], poses[i]
        y = oracle.project_fwd(g, beta, targets[i], vol)

        def L(theta):
            return float(np.sum((oracle.project_fwd(g, beta, theta, vol) - y) ** 2))

        w = 2.0 * (oracle.project_fwd(g, beta, th, vol) - y)
        ga = oracle.project_fwd_grad_pose(g, beta, th, vol, w)[0]
        fd = np.zeros(6)
        for q in range(6):
            e = np.zeros(6)
            e[q] = hs[q]
            fd[q] = (L(th + e) - L(th - e)) / (2 * hs[q])
        cos.append(_cos(ga, fd))
        parts.append(_triplet_agreement(ga, fd))
    cos = np.array(cos)
    floor = GOLD["paper_gradient_accuracy"]["forward_rd_mean_cosine"]
    assert cos.mean() >= floor, cos
    assert np.quantile(cos, 0.05) >= 0.98, np.sort(cos)[:5]
    _check_triplets(parts, floor)


def _bp_setup(seed):
    # Detector fine enough to resolve the blobs: the analytic gradient uses
    # central differences of l, which only approximate the derivative of the
    # bilinear interpolant when image features span several pixels.
    g = Geom(16, 16, 16, 4.0, 4.0, 4.0, 96, 80, 1.5, 1.5)
    rng = synth.rng_for(seed)
    V = 8
    angles = synth.circular_angles(V)
    proj = synth.smooth_images(V, g.nv, g.nu, rng, n_blobs=6).astype(np.float64)
    return g, rng, V, angles, proj


def _sharpness_and_grad(mu):
    """S = -sum of squared forward differences inside the grid, and dS/dmu."""
    S = 0.0
    grad = np.zeros_like(mu)
    for ax in range(3):
        d = np.diff(mu, axis=ax)
        S -= np.sum(d * d)
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[ax] = slice(1, None)
        sl_lo[ax] = slice(None, -1)
        grad[tuple(sl_hi)] -= 2 * d
        grad[tuple(sl_lo)] += 2 * d
    return S, grad


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("loss", ["l2", "sharpness"])
def test_backproject_grad_vs_central_fd(oracle, mode, loss):
    """O-FD2: analytic back-projection pose gradient vs central FD."""
    g, rng, V, angles, proj = _bp_setup(109)
    hs = _fd_steps()
    cos, parts = [], []
    for real in range(6):
        poses = synth.random_poses(V, 5.0, 5.0, rng)
        target = oracle.backproject(g, angles, synth.random_poses(V, 5.0, 5.0, rng), proj, mode)

        def L_and_e(p):
            mu = oracle.backproject(g, angles, p, proj, mode)
            if loss == "l2":
                return float(np.sum((mu - target) ** 2)), 2 * (mu - target)
            return _sharpness_and_grad(mu)

        _, e = L_and_e(poses)
        ga = oracle.backproject_grad_pose(g, angles, poses, proj, e, mode)
        fd = np.zeros((V, 6))
        for v in range(V):
            for q in range(6):
                pp = poses.copy()
                pm = poses.copy()
                pp[v, q] += hs[q]
                pm[v, q] -= hs[q]
                fd[v, q] = (L_and_e(pp)[0] - L_and_e(pm)[0]) / (2 * hs[q])
        cos += [_cos(ga[v], fd[v]) for v in range(V)]
        parts += [_triplet_agreement(ga[v], fd[v]) for v in range(V)]
    cos = np.array(cos)
    gold = GOLD["paper_gradient_accuracy"]
    assert cos.mean() >= gold["backprojector_vd_mean_cosine"], np.sort(cos)[:5]
    assert np.quantile(cos, 0.05) >= gold["backprojector_vd_p95_cosine"], np.sort(cos)[:5]
    _check_triplets(parts, gold["backprojector_vd_mean_cosine"])


def test_count_samples_consistent(oracle):
    g = Geom(16, 16, 16, 2.0, 2.0, 2.0, 20, 20, 3.0, 3.0)
    poses = synth.random_poses(3, 5, 5, synth.rng_for(110))
    c = oracle.count_samples_per_ray(g, [0, 1, 2], poses)
    assert c.sum() == oracle.count_samples(g, [0, 1, 2], poses)
    # The central ray of a 16-voxel cube at 2 mm crosses the open support
    # x in (-17, 17) mm; samples sit at multiples of 0.5 mm (D / step is an
    # integer), so x = -16.5 .. 16.5: 67 samples.
    c0 = oracle.count_samples_per_ray(Geom(16, 16, 16, 2.0, 2.0, 2.0, 21, 21, 3.0, 3.0), [0.0], np.zeros(6))
    assert c0[0, 10, 10] == 67


# ---------------------------------------------------------------------------
# Sampled entry points: the id -> (view, row, column) and id -> (i, j, k)
# decoding of the per-ray and per-voxel checkers used at full size
# ---------------------------------------------------------------------------

def test_project_fwd_rays_equals_full_projection(oracle):
    """project_fwd_rays at ray id v*nv*nu + b*nu + a returns exactly the full
    projection's l_v[b][a] (bit-equal), on a ragged grid with nu != nv and
    several views, for every id including the first and the last."""
    g = Geom(13, 11, 9, 2.0, 1.7, 2.3, 23, 17, 3.0, 2.6)
    rng = synth.rng_for(120)
    vol = rng.uniform(0.0, 1.0, (g.nz, g.ny, g.nx))
    angles = np.array([0.2, 1.9, 4.0])
    poses = synth.random_poses(3, 5.0, 5.0, rng)
    full = oracle.project_fwd(g, angles, poses, vol)
    assert full.shape == (3, g.nv, g.nu)
    order = rng.permutation(np.arange(full.size, dtype=np.int64))
    got = oracle.project_fwd_rays(g, angles, poses, vol, order)
    back = np.empty_like(got)
    back[order] = got
    assert np.array_equal(back, full.ravel())
    # a hand-picked id decodes to (v, b, a) = (2, 16, 22), the last pixel
    last = oracle.project_fwd_rays(g, angles, poses, vol, np.array([2 * 17 * 23 + 16 * 23 + 22]))
    assert last[0] == full[2, 16, 22]
    # (v, b, a) = (1, 3, 5): transposed decoding (b <-> a) would pick (1, 5, 3)
    one = oracle.project_fwd_rays(g, angles, poses, vol, np.array([1 * 17 * 23 + 3 * 23 + 5]))
    assert one[0] == full[1, 3, 5] and full[1, 3, 5] != full[1, 5, 3]
    assert np.any(full != 0.0)


@pytest.mark.parametrize("mode", [0, 1])
def test_backproject_voxels_equals_full_backprojection(oracle, mode):
    """backproject_voxels at voxel id (k*ny + j)*nx + i returns exactly the
    full back-projection's mu[k][j][i] (bit-equal), on a ragged grid
    (nx, ny, nz all different) with several views and both weights."""
    g = Geom(9, 7, 5, 2.0, 2.5, 1.5, 21, 15, 3.0, 3.0)
    rng = synth.rng_for(121)
    angles = np.array([0.4, 2.2, 3.9])
    poses = synth.random_poses(3, 5.0, 5.0, rng)
    proj = rng.uniform(0.0, 1.0, (3, g.nv, g.nu))
    full = oracle.backproject(g, angles, poses, proj, mode)
    assert full.shape == (g.nz, g.ny, g.nx)
    order = rng.permutation(np.arange(full.size, dtype=np.int64))
    got = oracle.backproject_voxels(g, angles, poses, proj, order, mode)
    back = np.empty_like(got)
    back[order] = got
    assert np.array_equal(back, full.ravel())
    # (i, j, k) = (8, 6, 4) is the last voxel; (i, j, k) = (2, 5, 1) would be
    # (5, 2, 1) under an i <-> j mix-up
    last = oracle.backproject_voxels(g, angles, poses, proj, np.array([(4 * 7 + 6) * 9 + 8]), mode)
    assert last[0] == full[4, 6, 8]
    one = oracle.backproject_voxels(g, angles, poses, proj, np.array([(1 * 7 + 5) * 9 + 2]), mode)
    assert one[0] == full[1, 5, 2] and full[1, 5, 2] != full[1, 2, 5]
