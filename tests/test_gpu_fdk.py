"""GPU parity of the FDK pre-filter and the sharpness loss against the FP64
oracle (oracle/fdk.py).  Tolerances: filtered projections max|gpu - ref| <=
1e-5 max|ref| (the kernel accumulates in FP64, so only the FP32 input and
output roundings remain); sharpness within 1e-5 relative, its gradient
within 1e-5 of max|grad| elementwise (FP32 differences of FP32 voxels)."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import fdk as ofdk
from synth import Geom

pytestmark = pytest.mark.gpu


def f32(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")


def _filter_case(dp, g, V, seed, scale):
    rng = np.random.default_rng(seed)
    proj = synth.smooth_images(V, g.nv, g.nu, rng, n_blobs=4, signed=True).astype(np.float32)
    got = dp.fdk_filter(g, f32(proj), scale).cpu().numpy()
    ref = ofdk.fdk_filter(g, proj, scale)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"fdk_filter {g.nu}x{g.nv} V={V}: max rel err {err:.3e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("nu,nv,off_u,off_v", [(512, 24, 0.0, 0.0), (37, 5, 1.25, -0.5),
                                               (1, 3, 0.0, 0.0), (1023, 2, -3.0, 0.0)])
def test_fdk_filter_matches_oracle(dp, nu, nv, off_u, off_v):
    g = Geom(8, 8, 8, 1.0, 1.0, 1.0, nu, nv, 0.776, 0.776, off_u=off_u, off_v=off_v)
    _filter_case(dp, g, 3, nu * 7 + nv, math.pi / 360)


def test_fdk_filter_full_size_sampled_views(dp):
    """The motion-compensated reconstruction workload (360 views of 512x384):
    every view filtered in one launch, three views checked in full."""
    g = synth.geom_c3_recon()
    V = 360
    rng = np.random.default_rng(31)
    proj = synth.smooth_images(V, g.nv, g.nu, rng, n_blobs=4, signed=True).astype(np.float32)
    got = dp.fdk_filter(g, f32(proj), math.pi / V).cpu().numpy()
    for v in (0, 179, 359):
        ref = ofdk.fdk_filter(g, proj[v:v + 1], math.pi / V)[0]
        err = np.abs(got[v] - ref).max() / np.abs(ref).max()
        print(f"fdk_filter full-size view {v}: max rel err {err:.3e}", flush=True)
        assert err <= 1e-5


def test_fdk_filter_in_place_and_rejects_long_rows(dp):
    g = Geom(8, 8, 8, 1.0, 1.0, 1.0, 64, 6, 1.0, 1.0)
    x = f32(np.random.default_rng(2).standard_normal((2, 6, 64)))
    ref = dp.fdk_filter(g, x.clone(), 0.5)
    dp.fdk_filter(g, x, 0.5, out=x)
    assert torch.equal(x, ref)
    big = Geom(8, 8, 8, 1.0, 1.0, 1.0, 4001, 1, 1.0, 1.0)
    with pytest.raises(RuntimeError, match="4000"):
        dp.fdk_filter(big, torch.zeros((1, 1, 4001), device="cuda:0"), 1.0)


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 1, 7), (17, 9, 33), (64, 64, 64)])
def test_sharpness_matches_oracle(dp, shape):
    rng = np.random.default_rng(sum(shape))
    vol = (rng.standard_normal(shape) * 0.02 + 0.01).astype(np.float32)
    loss, grad = dp.sharpness(f32(vol))
    ref_l, ref_g = ofdk.sharpness(vol), ofdk.sharpness_grad(vol)
    print(f"sharpness {shape}: loss {float(loss):.6e} ref {ref_l:.6e}", flush=True)
    assert abs(float(loss) - ref_l) <= 1e-5 * max(abs(ref_l), 1e-30)
    scale = max(np.abs(ref_g).max(), 1e-30)
    assert np.abs(grad.cpu().numpy() - ref_g).max() <= 1e-5 * scale


def test_sharpness_full_size_and_repeatable(dp):
    """512^3 reconstruction grid: loss against the oracle's, gradient on
    sampled voxels, two calls bitwise equal."""
    g = synth.geom_c3_recon()
    gen = torch.Generator(device="cuda:0").manual_seed(4)
    vol = torch.rand((g.nz, g.ny, g.nx), device="cuda:0", generator=gen) * 0.05
    loss, grad = dp.sharpness(vol)
    loss2, grad2 = dp.sharpness(vol)
    assert torch.equal(loss, loss2) and torch.equal(grad, grad2)
    v = vol.cpu().numpy()
    ref_l = ofdk.sharpness(v)
    assert abs(float(loss) - ref_l) <= 1e-5 * abs(ref_l)
    sl = (slice(0, 3), slice(250, 262), slice(500, 512))
    ref_g = ofdk.sharpness_grad(v[0:4, 249:263, 499:512])[0:3, 1:13, 1:13]
    got = grad[sl].cpu().numpy()
    assert np.abs(got - ref_g).max() <= 1e-5 * np.abs(ref_g).max()


@pytest.mark.parametrize("shape", [(1, 1, 2), (5, 3, 9), (33, 17, 40)])
def test_gradient_entropy_matches_oracle(dp, shape):
    """Gradient entropy: loss within 1e-6 relative; gradient within 1e-4 of
    max|grad| (FP32 logarithms and quotients per voxel)."""
    rng = np.random.default_rng(100 + sum(shape))
    vol = (rng.standard_normal(shape) * 0.01 + 0.02).astype(np.float32)
    loss, grad = dp.gradient_entropy(f32(vol))
    ref_l, ref_g = ofdk.gradient_entropy(vol), ofdk.gradient_entropy_grad(vol)
    print(f"gradient_entropy {shape}: {float(loss):.9f} ref {ref_l:.9f}", flush=True)
    assert abs(float(loss) - ref_l) <= 1e-6 * abs(ref_l)
    assert np.abs(grad.cpu().numpy() - ref_g).max() <= 1e-4 * np.abs(ref_g).max()


def test_gradient_entropy_smooth_phantom(dp):
    """A smoothed ellipsoid phantom (large flat regions, g near sqrt(eps))."""
    vol = synth.ellipsoid_phantom(48, 2.0, 8, synth.rng_for(7, 5), shell=True)
    loss, grad = dp.gradient_entropy(f32(vol))
    ref_l, ref_g = ofdk.gradient_entropy(vol), ofdk.gradient_entropy_grad(vol)
    assert abs(float(loss) - ref_l) <= 1e-6 * abs(ref_l)
    assert np.abs(grad.cpu().numpy() - ref_g).max() <= 1e-4 * np.abs(ref_g).max()
