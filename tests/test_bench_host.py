"""Host-side logic of the benchmark (no GPU): the exact sample count that
defines the ray-samples/s metric equals the oracle's brute-force count."""
import math

import numpy as np
import pytest

import synth
from synth import Geom


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_interval_count_matches_oracle(oracle, seed):
    import bench
    rng = synth.rng_for(300 + seed)
    g = Geom(19, 23, 17, 1.3, 1.1, 1.6, 29, 21, 2.1, 1.9, off_u=0.5, off_v=-1.0, step=0.5)
    V = 3
    angles = rng.uniform(0, 2 * math.pi, V)
    poses = synth.random_poses(V, 10.0, 30.0, rng)
    assert bench.count_ray_samples(g, angles, poses) == oracle.count_samples(g, angles, poses)


def test_interval_count_axis_aligned_rays(oracle):
    import bench
    g = Geom(16, 16, 16, 2.0, 2.0, 2.0, 21, 21, 3.0, 3.0)
    for beta in (0.0, 0.5 * math.pi):
        n = bench.count_ray_samples(g, [beta], np.zeros(6))
        assert n == oracle.count_samples(g, [beta], np.zeros(6))


def test_config1_count(oracle):
    import bench
    c = synth.config1_inputs()
    assert bench.count_ray_samples(c["geom"], c["angles"], c["poses"]) == \
        oracle.count_samples(c["geom"], c["angles"], c["poses"])


def test_multi_gpu_request_exits(monkeypatch, capsys):
    import bench
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2


def test_gather_roofline_fields(monkeypatch):
    """The gather roofline divides the measured LDS read bandwidth by 128 B
    per sample (the taps come from LDS), reports the L2 and HBM traffic
    beside, and takes counter figures only while the kernel hash matches."""
    import bench
    probe = {"lds_read_GBps": 127000.0, "l2_read_GBps": 32000.0, "hbm_read_GBps": 7000.0}
    fw = {"n_samples": 6.4e9, "ms_step": 20.0,
          "roofline": {"kernel": "rd_fused", "kernel_ms": 16.0, "traffic": 1.6e11,
                       "source_hash": "nomatch"}}
    g = bench.gather_roofline(fw, probe)
    assert g["ceiling"] == "lds"
    assert g["ceiling_samples_per_s"] == pytest.approx(127000e9 / 128)
    assert g["step_frac"] == pytest.approx(round(6.4e9 / 0.02 / (127000e9 / 128), 4))
    assert g["kernel_frac"] == pytest.approx(round(6.4e9 / 0.016 / (127000e9 / 128), 4))
    assert g["kernel_frac"] < 1.0
    assert g["lds_GBps"] == pytest.approx(round(6.4e9 / 0.016 * 128 / 1e9, 1))
    assert g["l2_bytes_per_launch"] is None and g["l2_frac"] is None  # stale hash
    assert g["beyond_l2_GBps"] == pytest.approx(1.6e11 / 0.016 / 1e9)
    assert g["beyond_l2_frac_of_hbm_stream"] == pytest.approx(round(1.6e11 / 0.016 / 1e9 / 7000.0, 4))
    monkeypatch.setattr(bench, "_traffic",
                        lambda key, h, field="hbm_bytes_per_launch": {"l2_bytes_per_launch": 1.28e11,
                                                                      "l2_hit_rate": 0.3}.get(field))
    g = bench.gather_roofline(fw, probe)
    assert g["l2_GBps"] == pytest.approx(1.28e11 / 0.016 / 1e9)
    assert g["l2_frac"] == pytest.approx(round(1.28e11 / 0.016 / 1e9 / 32000.0, 4))
    assert g["l2_hit_rate"] == 0.3



def test_host_cpu_description():
    import bench
    h = bench._host_cpu()
    assert set(h) == {"cpu_model", "nproc", "usable_cpus"}
    assert h["nproc"] >= 1


def test_oracle_thread_count_changes_only_the_timing():
    """The one-thread CPU baseline calls the same oracle: per-ray forward
    projections do not depend on the OpenMP thread count."""
    import oracle
    g = synth.geom_c1()
    vol = np.random.default_rng(0).random((g.nz, g.ny, g.nx))
    pose = [[1.0, -2.0, 0.5, 0.02, -0.03, 0.01]]
    n = oracle.num_threads()
    ref = oracle.project_fwd(g, [0.3], pose, vol)
    oracle.set_num_threads(1)
    try:
        assert oracle.num_threads() == 1
        one = oracle.project_fwd(g, [0.3], pose, vol)
    finally:
        oracle.set_num_threads(n)
    assert oracle.num_threads() == n
    assert np.array_equal(ref, one)


def test_vd_rooflines_take_each_kernels_tap_source():
    """The back-projection is graded against the L2 gather ceiling (its taps
    come through the cache hierarchy), its gradient against the LDS ceiling
    (taps from the staged rectangle), each against the arithmetic ceiling
    too, whichever is lower."""
    import bench
    probe = {"lds_read_GBps": 120000.0, "l2_read_GBps": 30000.0, "hbm_read_GBps": 7000.0}
    bp = {"voxel_view_updates": 4.8e10, "kernels_ms": {"vd_bp": 30.0, "vd_grad": 60.0}}
    r = bench.vd_rooflines(bp, probe)
    assert r["vd_bp"]["taps_from"] == "l2" and r["vd_grad"]["taps_from"] == "lds"
    assert r["vd_bp"]["gather_ceiling_updates_per_s"] == pytest.approx(30000e9 / 16)
    assert r["vd_grad"]["gather_ceiling_updates_per_s"] == pytest.approx(120000e9 / 48)
    for k in ("vd_bp", "vd_grad"):
        d = r[k]
        ceiling = min(d["gather_ceiling_updates_per_s"], d["alu_ceiling_updates_per_s"])
        assert d["frac"] == pytest.approx(round(d["updates_per_s"] / ceiling, 4))
        assert d["graded_against"] == ("alu" if d["alu_ceiling_updates_per_s"] < d["gather_ceiling_updates_per_s"]
                                       else "gather")


def test_proposal_training_flops():
    """Training-step FLOPs: three products per layer (two for the first,
    which needs no input gradient), counted from the layer shapes."""
    import bench
    from paper_2508_13304_amd import proposal as pr
    net = pr.ProposalNet(size=32, channels=(4, 8), device="cpu")
    # conv0: 32 -> 16, K = 18, Co 4; conv1: 16 -> 8, K = 36, Co 8; head 8*8*8 -> 6
    f0 = 2 * 2 * 16 * 16 * 18 * 4
    f1 = 2 * 2 * 8 * 8 * 36 * 8
    fc = 2 * 2 * 512 * 6
    assert bench.proposal_train_flops(net, 2) == 2 * f0 + 3 * f1 + 3 * fc
