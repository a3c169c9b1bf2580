"""Seeded input generators: determinism, ranges and the phantom recipe."""
import numpy as np

import synth


def test_phantom_is_seeded_and_has_zero_margin():
    a = synth.ellipsoid_phantom(32, 1.0, 10, synth.rng_for(0))
    b = synth.ellipsoid_phantom(32, 1.0, 10, synth.rng_for(0))
    assert a.dtype == np.float32 and a.shape == (32, 32, 32)
    np.testing.assert_array_equal(a, b)
    assert a.min() >= 0 and 0.01 <= a.max() <= 0.5
    # bounding spheres stop 4 voxels short of the face; smoothing (4 sigma
    # truncation) may reach at most 4 more voxels, never the outer shell
    assert np.all(a[0] == 0) and np.all(a[-1] == 0)
    assert np.all(a[:, 0] == 0) and np.all(a[:, :, -1] == 0)


def test_shell_value():
    v = synth.ellipsoid_phantom(64, 0.8, 5, synth.rng_for(1), shell=True, sigma=0.0)
    assert np.isclose(v.max(), 0.08) or v.max() > 0.08 - 1e-6


def test_poses_ranges():
    p = synth.random_poses(1000, 10.0, 5.0, synth.rng_for(2))
    assert p.shape == (1000, 6)
    assert np.abs(p[:, :3]).max() <= 10.0
    assert np.abs(p[:, 3:]).max() <= np.deg2rad(5.0)


def test_gaussian_smoothing_preserves_mass_inside():
    v = np.zeros((21, 21, 21))
    v[10, 10, 10] = 1.0
    s = synth.gaussian_smooth(v, 1.0)
    assert abs(s.sum() - 1.0) < 1e-12
    assert abs(s[10, 10, 11] / s[10, 10, 10] - np.exp(-0.5)) < 1e-3


def test_motion_amplitude():
    m = synth.sinusoidal_motion(360, 3.0, 2.0, synth.rng_for(3))
    assert np.abs(m[:, :3]).max() <= 3.0 + 1e-12
    assert np.abs(m[:, 3:]).max() <= np.deg2rad(2.0) + 1e-12


def test_torch_phantom_matches_numpy_recipe():
    """The bulk (torch) phantom generator draws the same ellipsoids as the
    numpy one and agrees with it to FP32 rounding."""
    a = synth.ellipsoid_phantom_torch(40, 2.0, 8, synth.rng_for(9, 3), "cpu", shell=True)
    b = synth.ellipsoid_phantom(40, 2.0, 8, synth.rng_for(9, 3), shell=True)
    assert np.abs(a.numpy() - b).max() < 1e-6


def test_poisson_log_noise_statistics():
    """Counts are Poisson with mean photons * exp(-l): the re-logged values
    average l (to first order) with variance exp(l) / photons."""
    import torch
    gen = torch.Generator().manual_seed(1)
    l = torch.full((200000,), 2.0, dtype=torch.float64)
    y = synth.poisson_log_noise(l, 1e5, gen)
    assert abs(float(y.mean()) - 2.0) < 1e-3
    assert abs(float(y.var()) / (np.exp(2.0) / 1e5) - 1.0) < 0.02
    # zero counts clamp to one photon: finite values
    y0 = synth.poisson_log_noise(torch.full((10,), 40.0, dtype=torch.float64), 1e5, gen)
    assert torch.isfinite(y0).all() and float(y0.max()) <= np.log(1e5) + 1e-9
    # scaled attenuation: the noise is that of scale * l, returned in l's units
    ys = synth.poisson_log_noise(torch.full((200000,), 10.0, dtype=torch.float64), 1e5, gen, 0.2)
    assert abs(float(ys.mean()) - 10.0) < 5e-3
    assert abs(float(ys.var()) / (np.exp(2.0) / 1e5 / 0.04) - 1.0) < 0.02


def test_transmission_noise_floor_matches_the_drawn_noise():
    """The expected SSD at the true pose that the learned pipeline's fallback
    allows for (first-order variance exp(s l) / (N s^2), evaluated on the
    noisy measurement) agrees with the SSD of the noise actually drawn."""
    import torch
    from paper_2508_13304_amd.proposal import transmission_noise_ssd
    gen = torch.Generator().manual_seed(11)
    l = torch.rand((3, 128, 128), dtype=torch.float64, generator=gen) * 28.0
    for photons, scale in ((1e5, 5.0 / 28.0), (1e4, 0.1)):
        y = synth.poisson_log_noise(l, photons, gen, scale)
        got = transmission_noise_ssd(y, photons, scale)
        drawn = ((y - l) ** 2).reshape(3, -1).sum(1)
        assert torch.allclose(got, drawn, rtol=0.03), (photons, got, drawn)
