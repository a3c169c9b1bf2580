"""Pins for the FDK pre-filter and sharpness oracle (oracle/fdk.py): the ramp
filter's frequency response, an end-to-end FDK reconstruction of a uniform
ball from its analytic (chord-length) projections, and closed forms and
finite differences for the sharpness loss."""
import math

import numpy as np
import pytest

import oracle
from oracle import fdk
from synth import Geom


@pytest.mark.parametrize("w_tau", [1 / 8, 1 / 5, 1 / 3, 0.45])
def test_ramlak_passes_a_cosine_with_gain_equal_to_its_frequency(w_tau):
    """The band-limited ramp kernel sampled at pitch tau has frequency response
    |w| below Nyquist: filtering cos(2 pi w x) returns |w| cos(2 pi w x)
    (away from the row ends)."""
    nu, tau = 4096, 1.5
    g = Geom(8, 8, 8, 1, 1, 1, nu, 1, tau, tau, sad=1e12, sdd=1e12)  # unit magnification, cos weight 1
    w = w_tau / tau
    n = np.arange(nu) - (nu - 1) / 2
    p = np.cos(2 * np.pi * w * n * tau)
    q = fdk.fdk_filter(g, p[None, None, :], 1.0)[0, 0]
    mid = slice(nu // 2 - 64, nu // 2 + 64)
    assert np.abs(q[mid] - w * p[mid]).max() < 1e-4 * w


def test_ramlak_kernel_values():
    h = fdk.ramlak(5, 2.0)  # k = -4..4
    k = np.arange(-4, 5)
    assert h[4] == pytest.approx(1 / 16)
    assert np.all(h[(k % 2 == 0) & (k != 0)] == 0)
    assert h[5] == pytest.approx(-1 / (math.pi ** 2 * 4))
    assert h[7] == pytest.approx(-1 / (math.pi ** 2 * 9 * 4))
    assert np.allclose(h, h[::-1])


def _ball_projections(g, angles, centre, radius, mu):
    """Exact line integrals of a uniform ball (chord length x mu) per pixel."""
    V = len(angles)
    out = np.zeros((V, g.nv, g.nu))
    cu, cv = (g.nu - 1) / 2 + g.off_u, (g.nv - 1) / 2 + g.off_v
    x = (np.arange(g.nu) - cu) * g.du
    y = (np.arange(g.nv) - cv) * g.dv
    for i, b in enumerate(angles):
        s = g.sad * np.array([math.cos(b), math.sin(b), 0.0])
        ew = np.array([-math.cos(b), -math.sin(b), 0.0])
        eu = np.array([-math.sin(b), math.cos(b), 0.0])
        ev = np.array([0.0, 0.0, 1.0])
        P = s + g.sdd * ew + x[None, :, None] * eu + y[:, None, None] * ev
        d = P - s
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        cs = np.asarray(centre) - s
        perp = cs - (d @ cs)[..., None] * d
        dist2 = np.sum(perp * perp, axis=-1)
        out[i] = 2.0 * np.sqrt(np.maximum(radius ** 2 - dist2, 0.0)) * mu
    return out


def test_fdk_reconstructs_a_uniform_ball():
    """Filtered projections of a ball, back-projected with the (SAD/U)^2 weight
    and the pi/V angular factor, give the ball's attenuation: to 0.2 % near the
    mid-plane, where FDK is exact up to discretisation, and to a few percent
    off it (cone-beam approximation) and outside the ball.  The short
    source distance (fan half-angle ~ 12 deg) makes the cosine weight matter:
    without it the mid-plane error is 0.6 %."""
    g = Geom(32, 32, 32, 3.0, 3.0, 3.0, 200, 160, 1.2, 1.2, sad=300.0, sdd=450.0)
    V = 360  # view aliasing stays below the bar inside the ball
    angles = np.arange(V) * 2 * math.pi / V
    centre, R, mu = np.array([3.0, -2.0, 0.0]), 40.0, 0.02
    proj = _ball_projections(g, angles, centre, R, mu)
    q = fdk.fdk_filter(g, proj, math.pi / V)
    rec = oracle.backproject(g, angles, np.zeros((V, 6)), q, oracle.W_FDK)
    c = (np.arange(32) - 15.5) * 3.0
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    dist = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2)
    inside = dist < R - 6.0
    mid = inside & (np.abs(Z) < 5.0)
    err = rec / mu - 1.0
    assert abs(err[mid].mean()) < 1e-3 and np.abs(err[mid]).max() < 2e-3
    assert abs(err[inside].mean()) < 5e-3 and np.abs(err[inside]).max() < 3e-2
    outside = (dist > R + 6.0) & (np.abs(Z) < 20.0)
    assert outside.sum() > 1000
    assert np.abs(rec[outside]).max() < 0.05 * mu


def test_sharpness_of_a_linear_ramp():
    nz, ny, nx, s = 5, 6, 7, 0.3
    vol = np.broadcast_to(np.arange(nx) * s, (nz, ny, nx)) + 4.0
    assert fdk.sharpness(vol) == pytest.approx(-(nx - 1) * ny * nz * s * s, rel=1e-12)


def test_sharpness_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    vol = rng.standard_normal((4, 5, 6))
    g = fdk.sharpness_grad(vol)
    h = 1e-5
    for idx in [(0, 0, 0), (3, 4, 5), (1, 2, 3), (2, 0, 5), (0, 4, 2)]:
        e = np.zeros_like(vol)
        e[idx] = h
        fd = (fdk.sharpness(vol + e) - fdk.sharpness(vol - e)) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-7, abs=1e-9)
    # invariant under a constant offset, so the gradient sums to zero
    assert abs(g.sum()) < 1e-9


def test_gradient_entropy_of_a_ramp_is_log_of_its_support():
    """A linear ramp along x has equal gradient magnitude on the (nx-1) ny nz
    voxels with a +x neighbour and (up to sqrt(eps)) zero elsewhere: its
    gradient entropy is that of a uniform distribution, log((nx-1) ny nz)."""
    nz, ny, nx = 4, 5, 9
    vol = np.broadcast_to(np.arange(nx) * 0.01, (nz, ny, nx))
    assert fdk.gradient_entropy(vol, eps=1e-20) == pytest.approx(math.log((nx - 1) * ny * nz), abs=1e-7)


def test_gradient_entropy_invariances_and_sharpening():
    """GE does not change when the volume is scaled or offset (eps -> 0), and
    blurring an edge raises it."""
    rng = np.random.default_rng(3)
    vol = rng.random((6, 7, 8))
    ge = fdk.gradient_entropy(vol, eps=1e-24)
    assert fdk.gradient_entropy(3.0 * vol + 5.0, eps=1e-24) == pytest.approx(ge, rel=1e-10)
    edge = np.zeros((8, 8, 16))
    edge[:, :, 8:] = 1.0
    blurred = edge.copy()
    blurred[:, :, 7] = 0.25
    blurred[:, :, 8] = 0.75
    assert fdk.gradient_entropy(blurred) > fdk.gradient_entropy(edge) + 0.5


def test_gradient_entropy_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    vol = rng.random((4, 5, 6))
    g = fdk.gradient_entropy_grad(vol)
    h = 1e-6
    for idx in [(0, 0, 0), (3, 4, 5), (1, 2, 3), (2, 0, 5), (0, 4, 2), (3, 0, 0)]:
        e = np.zeros_like(vol)
        e[idx] = h
        fd = (fdk.gradient_entropy(vol + e) - fdk.gradient_entropy(vol - e)) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-10)
