"""What the trained pose-proposal network gains over the plain method.

Unseen phantoms (a seed range the training set never used) with offsets
drawn like the training set (+-30 mm, +-20 deg), one 256x256 view: the
plain analytic-gradient registration from the identity against the
network's proposal refined by the same registration (identity fallback).
The trained weights are the ones the training command committed."""
import os

import pytest
import torch

pytestmark = pytest.mark.gpu


def _net():
    from paper_2508_13304_amd import proposal as pr
    if not os.path.exists(pr.WEIGHTS):
        pytest.skip("no trained proposal weights in the package")
    return pr, pr.ProposalNet.load(pr.WEIGHTS)


def test_proposal_is_closer_than_the_identity(dp):
    """The network's proposal is nearer the truth than the plain method's
    starting point in the components one view pair determines: the in-plane
    translations, the depth translation (through magnification) and the
    rotation about the central ray (median over 64 cases, at least 2x
    closer).  The two out-of-plane rotations are not determined by one
    reference DRR of an unknown phantom and are left to the refinement."""
    import synth
    pr, net = _net()
    geom = synth.geom_c5()
    dev = torch.device("cuda:0")
    errs, offs = [], []
    for i in range(4):
        rng = synth.rng_for(4, 7 * 1_000_003 + i)
        vol = pr.phantom(geom, rng, dev)
        truth = torch.tensor(synth.random_poses(16, pr.T_RANGE_MM, pr.R_RANGE_DEG, rng),
                             dtype=torch.float64, device=dev)
        angles = torch.zeros(16, dtype=torch.float64, device=dev)
        targets = dp.project_fwd(geom, angles, truth, vol)
        ref = dp.project_fwd(geom, angles[:1], torch.zeros_like(truth[:1]), vol)[0]
        theta0 = net.predict(pr.pair_input(ref.expand(16, -1, -1), targets, net.size))
        errs.append((theta0 - truth).abs())
        offs.append(truth.abs())
    e = torch.cat(errs).median(dim=0).values
    o = torch.cat(offs).median(dim=0).values
    print("proposal median |err|", e.cpu().numpy(), "identity", o.cpu().numpy(), flush=True)
    observable = [0, 1, 2, 3]  # tx (depth at gantry angle 0), ty, tz, gamma_x (about the ray)
    assert bool((e[observable] < 0.5 * o[observable]).all())


def test_learned_registration_beats_plain(dp):
    """Learned proposal + refinement reaches 0.1 mm / 0.1 deg at least as often
    as the plain method, with fewer iterations per registration."""
    import synth
    pr, net = _net()
    res = pr.evaluate(net, synth.geom_c5(), n_phantoms=4, per_phantom=16, salt=8)
    print(res, flush=True)
    assert res["learned_success"] >= res["plain_success"]
    assert res["learned_success"] >= 0.9
    assert res["learned_mean_iterations"] < res["plain_mean_iterations"]
