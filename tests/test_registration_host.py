"""Host-side pieces of the registration drivers (no GPU).

`coarsen` builds one level of the resolution pyramid that the coarse-to-fine
Levenberg-Marquardt driver climbs: the volume averaged over 2x2x2 voxels, the
targets binned 2x2, and the geometry with doubled cell sizes.  Pinned here:
the coarse voxel and pixel centres are the centroids of the fine cells they
replace (the geometry conventions of the forward model, Eq. final_fwd's
parametrisation of the detector and grid), the averages themselves, and,
through the FP64 oracle, that the coarse model of the coarse volume images
the same object onto the same detector positions as the binned fine images
(a wrong detector offset or voxel size shows up as a misregistration of the
two images).
"""
import math

import numpy as np
import pytest
import torch

from synth import Geom
from paper_2508_13304_amd.registration import coarsen


def _voxel_centres(n, h):
    return (np.arange(n) - (n - 1) / 2) * h


def _pixel_centres(n, d, off):
    return (np.arange(n) - (n - 1) / 2 - off) * d


def test_coarse_cells_are_centroids_of_the_fine_cells():
    g = Geom(12, 10, 8, 0.8, 0.7, 0.9, 14, 6, 0.6, 1.1, off_u=1.5, off_v=-0.75, step=0.4)
    gc, vc, yc = coarsen(g, torch.zeros(8, 10, 12), torch.zeros(3, 6, 14))
    assert (gc.nx, gc.ny, gc.nz, gc.nu, gc.nv) == (6, 5, 4, 7, 3)
    assert gc.step == pytest.approx(0.8) and (gc.sad, gc.sdd) == (g.sad, g.sdd)
    for n, h, nc, hc in ((g.nx, g.vx, gc.nx, gc.vx), (g.ny, g.vy, gc.ny, gc.vy),
                         (g.nz, g.vz, gc.nz, gc.vz)):
        fine = _voxel_centres(n, h).reshape(nc, 2).mean(1)
        np.testing.assert_allclose(_voxel_centres(nc, hc), fine, rtol=0, atol=1e-12)
    for n, d, off, nc, dc, offc in ((g.nu, g.du, g.off_u, gc.nu, gc.du, gc.off_u),
                                    (g.nv, g.dv, g.off_v, gc.nv, gc.dv, gc.off_v)):
        fine = _pixel_centres(n, d, off).reshape(nc, 2).mean(1)
        np.testing.assert_allclose(_pixel_centres(nc, dc, offc), fine, rtol=0, atol=1e-12)
    assert tuple(vc.shape) == (4, 5, 6) and tuple(yc.shape) == (3, 3, 7)


def test_coarse_values_are_cell_means():
    rng = np.random.default_rng(7)
    v = rng.standard_normal((4, 6, 8)).astype(np.float32)
    y = rng.standard_normal((2, 4, 6)).astype(np.float32)
    g = Geom(8, 6, 4, 1.0, 1.0, 1.0, 6, 4, 1.0, 1.0)
    _, vc, yc = coarsen(g, torch.from_numpy(v), torch.from_numpy(y))
    for k, j, i in np.ndindex(2, 3, 4):
        want = v[2 * k:2 * k + 2, 2 * j:2 * j + 2, 2 * i:2 * i + 2].astype(np.float64).mean()
        assert float(vc[k, j, i]) == pytest.approx(want, abs=1e-6)
    for b, j, i in np.ndindex(2, 2, 3):
        want = y[b, 2 * j:2 * j + 2, 2 * i:2 * i + 2].astype(np.float64).mean()
        assert float(yc[b, j, i]) == pytest.approx(want, abs=1e-6)


def test_odd_grid_is_rejected():
    g = Geom(8, 8, 7, 1.0, 1.0, 1.0, 8, 8, 1.0, 1.0)
    with pytest.raises(ValueError):
        coarsen(g, torch.zeros(7, 8, 8), torch.zeros(1, 8, 8))
    g = Geom(8, 8, 8, 1.0, 1.0, 1.0, 9, 8, 1.0, 1.0)
    with pytest.raises(ValueError):
        coarsen(g, torch.zeros(8, 8, 8), torch.zeros(1, 8, 9))


def _blob(n, h, centre, sigma):
    x = _voxel_centres(n, h)
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    r2 = (xx - centre[0]) ** 2 + (yy - centre[1]) ** 2 + (zz - centre[2]) ** 2
    return np.exp(-r2 / (2 * sigma ** 2)).astype(np.float32)


def test_coarse_model_images_the_object_where_the_binned_targets_do(oracle):
    """A smooth off-centre blob, an off-centre detector and a non-identity
    pose: the oracle's projection of the coarsened volume through the
    coarsened geometry matches the 2x2-binned fine projection to within the
    smoothing error of the coarser interpolant (1.5 % of the peak for a
    blob of 5 mm standard deviation on 1 mm voxels; it falls as the blob
    widens), with the same total, and a coarse geometry whose detector offset
    was not halved does not."""
    g = Geom(48, 48, 48, 1.0, 1.0, 1.0, 48, 48, 1.8, 1.8, off_u=3.0, off_v=-2.0, step=0.25)
    vol = _blob(48, 1.0, (3.0, -2.0, 1.5), 5.0)
    angles = np.array([0.3, 1.9])
    poses = np.array([[1.0, -0.5, 0.7, math.radians(3), math.radians(-2), math.radians(5)],
                      [-0.8, 0.4, -0.3, math.radians(-4), math.radians(1), math.radians(-3)]])
    fine = oracle.project_fwd(g, angles, poses, vol)
    gc, vc, yc = coarsen(g, torch.from_numpy(vol), torch.from_numpy(fine.astype(np.float32)))
    coarse = oracle.project_fwd(gc, angles, poses, vc.numpy())
    binned = yc.numpy().astype(np.float64)
    err = np.abs(coarse - binned).max() / np.abs(binned).max()
    assert err < 0.03, err
    assert coarse.sum() / binned.sum() == pytest.approx(1.0, abs=2e-3)
    wrong = oracle.project_fwd(gc.replace(off_u=g.off_u, off_v=g.off_v), angles, poses, vc.numpy())
    err_wrong = np.abs(wrong - binned).max() / np.abs(binned).max()
    assert err_wrong > 10 * err, (err, err_wrong)
