"""Pins for the oracle's footprint projector pairs -- separable footprint
(SF) and distance-driven (DD) -- and their pose gradients: hand-derived
single-voxel footprints, the adjoint identity of each pair, exact chord
lengths through a uniform cube, and central finite differences (Sec. III-A
reports forward gradients at mean cosines of 0.9978 (SF) and 0.9977 (DD))."""
import pytest
import json
import math
import os

import numpy as np

import oracle
import synth
from synth import Geom

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))


@pytest.mark.parametrize("kind", ["sf", "dd"])
def test_single_voxel_footprint_worked_example(kind):
    ex = GOLDEN[f"{kind}_single_voxel"]
    gm = ex["geometry"]
    g = Geom(gm["nx"], gm["ny"], gm["nz"], gm["vx"], gm["vy"], gm["vz"], gm["nu"], gm["nv"],
             gm["du"], gm["dv"], sad=gm["sad"], sdd=gm["sdd"])
    l = oracle.fp_project(g, [gm["angle"]], np.zeros((1, 6)), np.ones((1, 1, 1)), kind)[0]
    for a, b, val in ex["expected"]:
        assert abs(l[b, a] - val) < 1e-12, (a, b, l[b, a], val)


@pytest.mark.parametrize("kind", ["sf", "dd"])
def test_pair_is_exactly_adjoint(kind):
    rng = np.random.default_rng(1)
    g = Geom(12, 10, 8, 1.5, 1.7, 2.0, 20, 16, 2.0, 1.8, off_u=0.5, off_v=-0.25)
    angles = rng.uniform(0, 6, 3)
    poses = synth.random_poses(3, 5, 10, rng)
    x = rng.standard_normal((8, 10, 12))
    y = rng.standard_normal((3, 16, 20))
    lhs = np.sum(oracle.fp_project(g, angles, poses, x, kind) * y)
    rhs = np.sum(x * oracle.fp_backproject(g, angles, poses, y, kind))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _cube_chords(g, beta, half):
    """Exact chord of each pixel's ray through the cube [-half, half]^3."""
    cu, cv = (g.nu - 1) / 2 + g.off_u, (g.nv - 1) / 2 + g.off_v
    s = g.sad * np.array([math.cos(beta), math.sin(beta), 0.0])
    ew = np.array([-math.cos(beta), -math.sin(beta), 0.0])
    eu = np.array([-math.sin(beta), math.cos(beta), 0.0])
    ev = np.array([0.0, 0.0, 1.0])
    A, B = np.meshgrid(np.arange(g.nu), np.arange(g.nv))
    d = g.sdd * ew + ((A - cu) * g.du)[..., None] * eu + ((B - cv) * g.dv)[..., None] * ev
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (-half - s) / d
        t2 = (half - s) / d
    lo = np.nanmax(np.minimum(t1, t2), axis=-1)
    hi = np.nanmin(np.maximum(t1, t2), axis=-1)
    return np.maximum(hi - lo, 0.0)


@pytest.mark.parametrize("kind", ["sf", "dd"])
@pytest.mark.parametrize("beta", [0.3, 1.0])
def test_uniform_cube_gives_chord_lengths(kind, beta):
    """A uniform cube of 40^3 voxels: away from the silhouette edges (central
    20x20 pixels) the line integrals equal the exact chords within 1 %,
    and their median error over the whole shadow is below 0.5 %."""
    g = Geom(40, 40, 40, 1.0, 1.0, 1.0, 64, 64, 1.0, 1.0)
    l = oracle.fp_project(g, [beta], np.zeros((1, 6)), np.ones((40, 40, 40)), kind)[0]
    c = _cube_chords(g, beta, 20.0)
    rel = np.abs(l - c) / np.maximum(c, 1e-9)
    centre = (slice(22, 42), slice(22, 42))
    assert rel[centre].max() < 0.01
    assert np.median(rel[c > 5]) < 0.005


@pytest.mark.parametrize("kind", ["sf", "dd"])
def test_forward_gradient_matches_finite_differences(kind):
    """Forward: L = ||A(theta) mu - y||^2; the analytic gradient (G_f
    projected with the same footprint weights) against central differences:
    mean cosine >= 0.99 over 8 random motions, none below 0.95."""
    rng = synth.rng_for(610)
    g = Geom(32, 32, 32, 2.0, 2.0, 2.0, 48, 48, 2.0, 2.0)
    vol = synth.ellipsoid_phantom(32, 2.0, 8, rng, sigma=1.5)
    V = 8
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 5.0, 5.0, rng)
    y = oracle.fp_project(g, angles, synth.random_poses(V, 5.0, 5.0, rng), vol, kind)

    def loss_v(p):
        r = oracle.fp_project(g, angles, p, vol, kind) - y
        return (r * r).reshape(V, -1).sum(1)

    r = oracle.fp_project(g, angles, poses, vol, kind) - y
    grad = oracle.fp_project_grad_pose(g, angles, poses, vol, 2.0 * r, kind)
    cos = []
    h = 1e-4
    base = poses.copy()
    for v in range(V):
        fd = np.zeros(6)
        for q in range(6):
            pp, pm = base.copy(), base.copy()
            pp[v, q] += h
            pm[v, q] -= h
            fd[q] = (loss_v(pp)[v] - loss_v(pm)[v]) / (2 * h)
        cos.append(grad[v] @ fd / (np.linalg.norm(grad[v]) * np.linalg.norm(fd)))
    cos = np.array(cos)
    assert cos.mean() >= 0.99 and cos.min() >= 0.95


@pytest.mark.parametrize("kind", ["sf", "dd"])
def test_backprojection_gradient_is_the_footprint_weighted_continuous_gradient(kind):
    """SF back-projection gradient: the method's rule applies the footprint
    weights to G_b per pixel, i.e. it is the continuous back-projection
    gradient (detector gradient x projection Jacobian x grad_M r) smoothed
    by the footprint.  Pinned against the voxel-driven gradient, itself
    pinned to finite differences: per view the same direction (cosine
    >= 0.998) on a detector fine enough that the footprint only smooths,
    and, for SF, a common scale (the footprint mass L x (2 x 1.5)^2 = 18;
    the DD mass varies with the view's angle to its dominant axis)."""
    rng = synth.rng_for(611)
    g = Geom(24, 24, 24, 2.0, 2.0, 2.0, 128, 120, 1.0, 1.0)
    V = 6
    angles = rng.uniform(0, 2 * math.pi, V)
    proj = synth.smooth_images(V, g.nv, g.nu, rng, n_blobs=4)
    poses = synth.random_poses(V, 3.0, 3.0, rng)
    e = rng.standard_normal((24, 24, 24))
    gs = oracle.fp_backproject_grad_pose(g, angles, poses, proj, e, kind)
    gv = oracle.backproject_grad_pose(g, angles, poses, proj, e)
    cos = np.sum(gs * gv, axis=1) / (np.linalg.norm(gs, axis=1) * np.linalg.norm(gv, axis=1))
    ratio = np.linalg.norm(gs, axis=1) / np.linalg.norm(gv, axis=1)
    assert cos.min() >= 0.998
    if kind == "sf":
        assert np.all(np.abs(ratio / 18.0 - 1.0) < 0.05)
    else:
        assert np.all((ratio > 0.95 * 18.0) & (ratio < 1.45 * 18.0))


@pytest.mark.parametrize("kind", ["sf", "dd"])
def test_backprojection_gradient_against_finite_differences(kind):
    """Against central differences of the SF back-projection loss itself the
    agreement is lower than for the voxel-driven pair: the footprint's
    trapezoid breakpoints, axial rectangle and central chord change with
    the pose, and the method's gradient omits those weight derivatives
    (Sec. III-A reports wider SF/DD back-projection distributions with
    lower minima).  Held to: median cosine >= 0.95, every view >= 0.5."""
    rng = synth.rng_for(611)
    g = Geom(24, 24, 24, 2.0, 2.0, 2.0, 80, 72, 1.0, 1.0)
    V = 6
    angles = rng.uniform(0, 2 * math.pi, V)
    proj = synth.smooth_images(V, g.nv, g.nu, rng, n_blobs=4)
    poses = synth.random_poses(V, 3.0, 3.0, rng)
    ref = oracle.fp_backproject(g, angles, synth.random_poses(V, 3.0, 3.0, rng), proj, kind)
    cos = []
    h = 1e-4
    for v in range(V):
        def loss(p):
            r = oracle.fp_backproject(g, angles[v:v + 1], p[v:v + 1], proj[v:v + 1], kind) - ref / V
            return float(np.sum(r * r))
        r = oracle.fp_backproject(g, angles[v:v + 1], poses[v:v + 1], proj[v:v + 1], kind) - ref / V
        gv = oracle.fp_backproject_grad_pose(g, angles[v:v + 1], poses[v:v + 1], proj[v:v + 1],
                                             2.0 * r, kind)[0]
        fd = np.zeros(6)
        for q in range(6):
            pp, pm = poses.copy(), poses.copy()
            pp[v, q] += h
            pm[v, q] -= h
            fd[q] = (loss(pp) - loss(pm)) / (2 * h)
        cos.append(gv @ fd / (np.linalg.norm(gv) * np.linalg.norm(fd)))
    cos = np.array(cos)
    assert np.median(cos) >= 0.95 and cos.min() >= 0.5
