"""The allocation-free single-pass SSD entry (dp_project_fwd_ssd_grad_pose_noalloc,
whose workspace is the library's fixed device array) against the entry with a
caller workspace (dp_project_fwd_ssd_grad_pose): the same kernels on the same
inputs, so DRRs, per-view SSD and pose gradients must be bit-identical.  Two
calls in a row, the second with a smaller problem (the array keeps the first
call's contents), and the size limit rejected before any launch."""
import numpy as np
import pytest
import torch

import synth
from synth import Geom

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _inputs(g, V, salt):
    rng = synth.rng_for(600, salt)
    n = max(g.nx, g.ny, g.nz)
    vol = synth.ellipsoid_phantom(n, g.vx, 8, rng)[:g.nz, :g.ny, :g.nx].copy()
    angles = rng.uniform(0.0, 2 * np.pi, V)
    poses = synth.random_poses(V, 5.0, 5.0, rng)
    T = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)  # noqa: E731
    a, p, v = T(angles, torch.float64), T(poses, torch.float64), T(vol, torch.float32)
    target_poses = T(synth.random_poses(V, 5.0, 5.0, rng), torch.float64)
    return a, p, v, target_poses


def _compare(dp, g, V, salt):
    a, p, v, tp = _inputs(g, V, salt)
    y = dp.project_fwd(g, a, tp, v)
    l_ws, loss_ws, g_ws = dp.project_fwd_ssd_grad_pose(g, a, p, v, y)
    l_na, loss_na, g_na = dp.project_fwd_ssd_grad_pose_noalloc(g, a, p, v, y)
    torch.cuda.synchronize()
    print(f"no-alloc case {salt}: vol {tuple(v.shape)} det {g.nv}x{g.nu} V={V}", flush=True)
    assert torch.equal(l_na, l_ws)
    assert torch.equal(loss_na, loss_ws)
    assert torch.equal(g_na, g_ws)
    assert float(loss_ws.abs().max()) > 0 and float(g_ws.abs().max()) > 0


def test_noalloc_matches_workspace_entry_on_two_calls(dp):
    # larger first call, then a smaller one on the same device array
    _compare(dp, Geom(48, 40, 36, 1.5, 1.5, 1.5, 70, 52, 1.6, 1.6, off_u=0.5), 6, 1)
    _compare(dp, Geom(20, 24, 18, 2.0, 2.0, 2.0, 33, 29, 2.2, 2.2), 2, 2)


def test_noalloc_rejects_problems_beyond_its_array(dp):
    g = Geom(32, 32, 32, 1.0, 1.0, 1.0, 512, 512, 0.6, 0.6)
    V = 512
    assert dp.workspace_bytes(g, V, dp.OP_FWD_SSD) > 16 << 20
    T = lambda *s, dt=torch.float32: torch.zeros(s, dtype=dt, device=DEV)  # noqa: E731
    with pytest.raises(RuntimeError, match="scratch"):
        dp.project_fwd_ssd_grad_pose_noalloc(g, T(V, dt=torch.float64), T(V, 6, dt=torch.float64),
                                             T(32, 32, 32), T(V, 512, 512))
