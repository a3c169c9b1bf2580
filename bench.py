"""Benchmark: forward projection + pose gradient throughput (ray-samples/s).

Workload (one step): 256^3 ellipsoid phantom with a high-attenuation shell
at 0.8 mm, 64 candidate poses (+-10 mm / +-10 deg) as 64 views of one
512x512 detector at 0.6 mm (SAD 1000 mm, SDD 1500 mm, 0.5 mm ray steps);
forward-project all 64 DRRs, form the SSD loss gradient against a target
DRR at a true pose, and compute the 64 x 6 pose gradients.  Inputs are
resident in device memory before the timed region.

value = exact in-support sample count of the 64 rays sets / step time.
Extra legs on the same JSON line: per-kernel timings from HIP events on the
launch stream, the roofline entry of the dominant kernel, the FP64 oracle
timed on the host on a bounded sample, and the back-projector at
512^3 / 360 views (voxel-view updates per second).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-bp]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
VALU_PEAK_TFLOPS = 157.3       # fp32 vector, MI355X spec (packed FMA)
# The same chip without packed FP32 (this build keeps it off): 256 CUs x 4
# SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz.  Reported beside the peak; the
# counters show the kernels issuing above it (VALU busy > 100 % of the
# 4-cycle wave64 model), so it is not a hard ceiling either.
VALU_UNPACKED_TFLOPS = 78.6
# Algorithmic FP32 operations of the method per unit of work (FMA counted as 2),
# fixed counts that do not depend on how a kernel arranges its arithmetic:
#   per in-support ray sample: forward ~30 (position, fractions, trilinear
#   interpolation, sum), pose gradient ~120 (position, fractions, the three
#   gradient channels' trilinear interpolation with their moments, the nine
#   per-ray sums); the fused SSD pass does both on one march (150);
#   per voxel-view update: back-projection ~25 (depth, reciprocal, pixel
#   coordinates, bilinear tap, weight), its pose gradient ~90 (the same plus
#   three bilinear fields, the detector-Jacobian row and twelve sums).
FLOPS_PER_SAMPLE = {"rd_fwd": 30, "rd_grad": 120, "rd_fused": 150}
# bytes one forward + gradient sample gathers: 8 trilinear corners x (mu, Gx, Gy, Gz) x 4 B
GATHER_BYTES_PER_SAMPLE = 128
# bytes one voxel-view update gathers: the bilinear cell of l (back-projection),
# of (l, dl/da, dl/db) (its pose gradient), and where the taps come from: the
# back-projection gathers through the cache hierarchy (L2 ceiling), the
# gradient from the detector rectangle each block stages in LDS (LDS ceiling)
VD_GATHER_BYTES_PER_UPDATE = {"vd_bp": 16, "vd_grad": 48}
VD_TAP_SOURCE = {"vd_bp": "l2", "vd_grad": "lds"}
VD_FLOPS_PER_UPDATE = {"vd_bp": 25, "vd_grad": 90}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Exact in-support sample count (the unit of the metric)
# ---------------------------------------------------------------------------

def _rot(g):
    cx, sx, cy, sy, cz, sz = (math.cos(g[0]), math.sin(g[0]), math.cos(g[1]), math.sin(g[1]),
                              math.cos(g[2]), math.sin(g[2]))
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def count_ray_samples(geom, angles, poses) -> int:
    """Number of samples k >= 0 at arc length k*step from the source whose
    object-frame continuous voxel index lies in the open box (-1, n)^3,
    summed over all rays of all views (FP64 interval count per ray)."""
    total = 0
    n = np.array([geom.nx, geom.ny, geom.nz], dtype=np.float64)
    h = np.array([geom.vx, geom.vy, geom.vz])
    c = (n - 1) / 2
    cu = (geom.nu - 1) / 2 + geom.off_u
    cv = (geom.nv - 1) / 2 + geom.off_v
    A, B = np.meshgrid(np.arange(geom.nu), np.arange(geom.nv))
    xa = ((A - cu) * geom.du).ravel()
    yb = ((B - cv) * geom.dv).ravel()
    for beta, th in zip(np.atleast_1d(angles), np.reshape(poses, (-1, 6))):
        cb, sb = math.cos(beta), math.sin(beta)
        src = geom.sad * np.array([cb, sb, 0.0])
        ew, eu, ev = np.array([-cb, -sb, 0.0]), np.array([-sb, cb, 0.0]), np.array([0.0, 0, 1])
        d = geom.sdd * ew[None, :] + xa[:, None] * eu[None, :] + yb[:, None] * ev[None, :]
        u = d / np.linalg.norm(d, axis=1, keepdims=True)
        R = _rot(th[3:])
        alpha = (R.T @ (src - th[:3])) / h + c          # index of the source
        beta_ = (u @ R) / h[None, :]                     # index per mm along the ray
        lo = np.full(u.shape[0], -np.inf)
        hi = np.full(u.shape[0], np.inf)
        empty = np.zeros(u.shape[0], bool)
        for a in range(3):
            ba = beta_[:, a]
            nz = ba != 0
            t1 = np.where(nz, (-1.0 - alpha[a]) / np.where(nz, ba, 1), -np.inf)
            t2 = np.where(nz, (n[a] - alpha[a]) / np.where(nz, ba, 1), np.inf)
            lo = np.maximum(lo, np.where(nz, np.minimum(t1, t2), -np.inf))
            hi = np.minimum(hi, np.where(nz, np.maximum(t1, t2), np.inf))
            if not (-1.0 < alpha[a] < n[a]):
                empty |= ~nz
        kmin = np.maximum(np.floor(lo / geom.step) + 1, 0)
        kmax = np.ceil(hi / geom.step) - 1
        cnt = np.where(empty, 0, np.maximum(kmax - kmin + 1, 0))
        total += int(cnt.sum())
    return total


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------

def _kernel_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2508_13304_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(kernel_key, src_hash, field="hbm_bytes_per_launch"):
    """Bytes per launch measured with rocprofv3 counters (committed under
    profiles/; HBM by default, or the L2 read bytes), valid only while the
    kernel source is unchanged."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p)).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != src_hash:
        return None
    return rec.get(field)


def run_forward(args, dp, torch):
    dev = torch.device("cuda:0")
    log("[bench] generating registration-scale inputs (256^3 phantom, 64 poses)")
    c = synth.config2_inputs()
    g, V = c["geom"], len(c["angles"])
    T = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)  # noqa: E731
    vol = T(c["vol"], torch.float32)
    angles = T(c["angles"], torch.float64)
    poses = T(c["poses"], torch.float64)
    # target DRR at the true pose (synthetic input, generated once), one copy per candidate
    y1 = dp.project_fwd(g, T([0.0], torch.float64), T(c["target_pose"], torch.float64), vol)
    y = y1.expand(V, -1, -1).contiguous()
    ws = torch.empty(max(dp.workspace_bytes(g, V, op) for op in (dp.OP_FWD, dp.OP_FWD_GRAD,
                                                                  dp.OP_FWD_SSD)),
                     dtype=torch.uint8, device=dev)
    proj = torch.empty((V, g.nv, g.nu), dtype=torch.float32, device=dev)
    wgrad = torch.empty_like(proj)
    gpose = torch.empty((V, 6), dtype=torch.float64, device=dev)
    loss = torch.empty(V, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():  # one pass: DRRs, per-view SSD and its pose gradient
        dp.project_fwd_ssd_grad_pose(g, angles, poses, vol, y, proj=proj, loss=loss, grad=gpose,
                                     ws=ws, stream=stream)

    def step_two_calls():  # forward launch, residual, gradient launch
        dp.project_fwd(g, angles, poses, vol, out=proj, ws=ws, stream=stream)
        torch.sub(proj, y, out=wgrad)
        wgrad.mul_(2.0)
        dp.project_fwd_grad_pose(g, angles, poses, vol, wgrad, out=gpose, ws=ws, stream=stream)

    n_samples = count_ray_samples(g, c["angles"], c["poses"])
    log(f"[bench] in-support samples per step: {n_samples:.4e}")

    def measure(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        dp.profile_enable(True)
        dp.profile_collect()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kern = dp.profile_collect()
        dp.profile_enable(False)
        return dt * 1e3 / steps, {k: round(v[0] / v[1], 4) for k, v in kern.items()}

    ms2, per2 = measure(step_two_calls, max(2, args.steps // 2), 1)
    log(f"[bench] two-call step {ms2:.3f} ms; per-kernel avg ms: {per2}")

    # the same step through the autograd Function: ProjectFwd.apply, the SSD
    # in torch, loss.backward() (the pose gradient kernel as the backward)
    from paper_2508_13304_amd.autograd import ProjectFwd

    def step_autograd():
        p = poses.detach().clone().requires_grad_(True)
        l = ProjectFwd.apply(p, vol, g, angles, ws)
        loss_ag = ((l - y) ** 2).sum()
        loss_ag.backward()

    ms_ag, per_ag = measure(step_autograd, max(2, args.steps // 2), 1)
    log(f"[bench] autograd step {ms_ag:.3f} ms; per-kernel avg ms: {per_ag}")
    ms_step, per_kernel = measure(step, args.steps, args.warmup)
    log(f"[bench] fused step {ms_step:.3f} ms/step; per-kernel avg ms: {per_kernel}")
    dominant = "rd_fused"
    dom_ms = per_kernel.get(dominant, 0.0)
    # The ray kernels are bound by VALU issue once their taps come from LDS:
    # roofline = algorithmic FP32 operations per in-support sample (FMA = 2)
    # against the fp32 vector peak.
    flops = FLOPS_PER_SAMPLE[dominant]
    achieved = flops * n_samples / (dom_ms * 1e-3) / 1e12
    src_hash = _kernel_hash("rd.hip", "dp_internal.h")
    other = {}
    for k in ("rd_fwd", "rd_grad"):
        if per2.get(k):
            other[k] = {"ms": per2[k], "flops_per_sample": FLOPS_PER_SAMPLE[k],
                        "tflops": round(FLOPS_PER_SAMPLE[k] * n_samples / (per2[k] * 1e-3) / 1e12, 2),
                        "traffic": _traffic(k + "_registration_scale", src_hash)}
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 4),
                "unpacked_fp32_peak": VALU_UNPACKED_TFLOPS,
                "frac_of_unpacked": round(achieved / VALU_UNPACKED_TFLOPS, 4),
                "traffic": _traffic(dominant + "_registration_scale", src_hash),
                "kernel": dominant, "kernel_ms": dom_ms, "flops_per_sample": flops,
                "source_hash": src_hash, "other": other}
    return dict(geom=g, V=V, n_samples=n_samples, ms_step=ms_step, per_kernel=per_kernel,
                two_call_ms=ms2, two_call_kernels=per2, autograd_ms=ms_ag,
                autograd_kernels=per_ag, roofline=roofline, inputs=c)


def run_cache_probe(dp, torch, quick=False):
    """Measured read bandwidths of this GPU: L2 (every block streams a small
    footprint that stays resident in each XCD's L2) and HBM (the blocks split a
    2 GiB buffer, nontemporal loads).  The best of a small sweep of footprints
    and grid sizes;
    bytes are what the loads request, timed with HIP events on the launch
    stream, median of 5 launches after one warm-up."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    def timed(buf, reps, shared, blocks):
        out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
        dp.read_probe(buf, reps, shared, blocks, out=out, stream=stream)
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dp.read_probe(buf, reps, shared, blocks, out=out, stream=stream)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[2]

    l2 = {}
    for mib in ((2,) if quick else (1, 2)):
        buf = torch.ones(mib * (1 << 18), dtype=torch.float32, device=dev)
        n_vec = buf.numel() // 4
        for blocks in ((2048,) if quick else (1024, 2048, 4096)):
            reps = max(1, (16 << 30) // (blocks * n_vec * 16))  # ~16 GiB requested per launch
            ms = timed(buf, reps, True, blocks)
            l2[f"{mib}MiB_x{blocks}blocks"] = round(blocks * reps * n_vec * 16 / (ms * 1e-3) / 1e9, 1)
        del buf
    hbm = {}
    buf = torch.ones(1 << 29, dtype=torch.float32, device=dev)  # 2 GiB, far above L2 + MALL
    for blocks in ((2048,) if quick else (1024, 2048, 4096)):
        ms = timed(buf, 1, False, blocks)
        hbm[f"2GiB_x{blocks}blocks"] = round(buf.numel() * 4 / (ms * 1e-3) / 1e9, 1)
    del buf
    # LDS: every block reads 16-byte vectors from 32 KiB of LDS, conflict-free
    lds = {}
    for blocks in ((2048,) if quick else (1024, 2048, 4096)):
        reps = 1024
        out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
        dp.lds_probe(reps, blocks, out=out, stream=stream)
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dp.lds_probe(reps, blocks, out=out, stream=stream)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = sorted(ts)[2]
        lds[f"x{blocks}blocks"] = round(blocks * 256 * reps * 128 / (ms * 1e-3) / 1e9, 1)
    res = {"l2_read_GBps": max(l2.values()), "hbm_read_GBps": max(hbm.values()),
           "lds_read_GBps": max(lds.values()),
           "l2_sweep": l2, "hbm_sweep": hbm, "lds_sweep": lds}
    log(f"[bench] read probe: LDS {res['lds_read_GBps']:.0f} GB/s, L2 {res['l2_read_GBps']:.0f} GB/s, "
        f"HBM {res['hbm_read_GBps']:.0f} GB/s")
    return res


def gather_roofline(fw, probe):
    """Gather roofline of the ray kernels: every trilinear tap of a forward +
    gradient sample comes from LDS (8 corners x (mu, Gx, Gy, Gz) x 4 B = 128
    B per sample), so the ceiling is the measured LDS read bandwidth over 128
    B.  The L2 and HBM traffic of the dominant kernel (rocprofv3 counters,
    valid while its source is unchanged) is what the chunk-box staging moves
    into LDS; it is reported beside, against the measured L2 and HBM read
    bandwidths."""
    ceiling = probe["lds_read_GBps"] * 1e9 / GATHER_BYTES_PER_SAMPLE
    rf = fw["roofline"]
    k_ms = rf["kernel_ms"]
    step_rate = fw["n_samples"] / (fw["ms_step"] * 1e-3)
    kern_rate = fw["n_samples"] / (k_ms * 1e-3)
    l2_bytes = _traffic(rf["kernel"] + "_registration_scale", rf["source_hash"], "l2_bytes_per_launch")
    hbm_bytes = rf["traffic"]
    out = {"bytes_per_sample": GATHER_BYTES_PER_SAMPLE,
           "ceiling": "lds",
           "lds_read_GBps_measured": probe["lds_read_GBps"],
           "l2_read_GBps_measured": probe["l2_read_GBps"],
           "hbm_read_GBps_measured": probe["hbm_read_GBps"],
           "ceiling_samples_per_s": ceiling,
           "step_frac": round(step_rate / ceiling, 4),
           "kernel_frac": round(kern_rate / ceiling, 4),
           "kernel": rf["kernel"],
           "lds_GBps": round(kern_rate * GATHER_BYTES_PER_SAMPLE / 1e9, 1),
           "l2_bytes_per_launch": l2_bytes,
           "l2_GBps": round(l2_bytes / (k_ms * 1e-3) / 1e9, 1) if l2_bytes else None,
           "l2_frac": round(l2_bytes / (k_ms * 1e-3) / 1e9 / probe["l2_read_GBps"], 4) if l2_bytes else None,
           "l2_hit_rate": _traffic(rf["kernel"] + "_registration_scale", rf["source_hash"], "l2_hit_rate"),
           # L2 misses (FETCH_SIZE + WRITE_SIZE) are served by the last-level
           # cache or HBM; compared with the measured HBM stream
           "beyond_l2_GBps": round(hbm_bytes / (k_ms * 1e-3) / 1e9, 1) if hbm_bytes else None,
           "beyond_l2_frac_of_hbm_stream":
               round(hbm_bytes / (k_ms * 1e-3) / 1e9 / probe["hbm_read_GBps"], 4) if hbm_bytes else None,
           "probe": probe}
    return out


def vd_rooflines(bp, probe):
    """Both ceilings of each back-projector kernel: the FP32 arithmetic
    ceiling (published FP32 vector peak over the algorithmic operations per
    update) and the gather ceiling (the measured read bandwidth of where its
    taps come from, L2 or LDS, over the bytes an update gathers).  Each
    kernel is graded against the lower ceiling; the texture-addresser busy
    fraction (rocprofv3, while the kernel source is unchanged) is reported
    beside."""
    h = _kernel_hash("vd.hip", "dp_internal.h")
    out = {}
    for k, nbytes in VD_GATHER_BYTES_PER_UPDATE.items():
        ms = bp["kernels_ms"].get(k)
        if not ms:
            continue
        rate = bp["voxel_view_updates"] / (ms * 1e-3)
        src = VD_TAP_SOURCE[k]
        gather = probe[src + "_read_GBps"] * 1e9 / nbytes
        flops = VD_FLOPS_PER_UPDATE[k]
        alu = VALU_PEAK_TFLOPS * 1e12 / flops
        bound = "alu" if alu < gather else "gather"
        ceiling = min(gather, alu)
        out[k] = {"updates_per_s": rate, "gather_bytes_per_update": nbytes, "taps_from": src,
                  "gather_ceiling_updates_per_s": gather, "gather_frac": round(rate / gather, 4),
                  "flops_per_update": flops, "tflops": round(rate * flops / 1e12, 2),
                  "alu_ceiling_updates_per_s": alu, "alu_frac": round(rate / alu, 4),
                  "alu_frac_of_unpacked": round(rate * flops / (VALU_UNPACKED_TFLOPS * 1e12), 4),
                  "graded_against": bound, "frac": round(rate / ceiling, 4),
                  "valu_busy": _traffic(k + "_reconstruction_scale", h, "valu_busy"),
                  "ta_busy": _traffic(k + "_reconstruction_scale", h, "ta_busy"),
                  "l2_hit_rate": _traffic(k + "_reconstruction_scale", h, "l2_hit_rate")}
        l2b = _traffic(k + "_reconstruction_scale", h, "l2_bytes_per_call")  # the call's launches
        out[k]["l2_GBps"] = round(l2b / (ms * 1e-3) / 1e9, 1) if l2b else None
        out[k]["l2_frac"] = round(l2b / (ms * 1e-3) / 1e9 / probe["l2_read_GBps"], 4) if l2b else None
    return out


def run_backproject(args, dp, torch):
    dev = torch.device("cuda:0")
    g = synth.geom_c3_recon()
    m = synth.config3_motion()
    V = len(m["angles"])
    rng = np.random.default_rng(3)
    log("[bench] generating motion-compensated reconstruction inputs (360 views 512x384, 512^3 recon)")
    proj_np = synth.smooth_images(V, g.nv, g.nu, rng, n_blobs=4, signed=True)
    T = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)  # noqa: E731
    angles, poses = T(m["angles"], torch.float64), T(m["poses"], torch.float64)
    proj = T(proj_np, torch.float32)
    del proj_np
    vol = torch.empty((g.nz, g.ny, g.nx), dtype=torch.float32, device=dev)
    e = torch.empty_like(vol).normal_(generator=torch.Generator(device=dev).manual_seed(5))
    gp = torch.empty((V, 6), dtype=torch.float64, device=dev)
    ws = torch.empty(max(dp.workspace_bytes(g, V, dp.OP_BP), dp.workspace_bytes(g, V, dp.OP_BP_GRAD)),
                     dtype=torch.uint8, device=dev)
    reps = max(1, min(args.steps, 5))
    for _ in range(1):
        dp.backproject(g, angles, poses, proj, dp.W_FDK, out=vol, ws=ws)
        dp.backproject_grad_pose(g, angles, poses, proj, e, dp.W_FDK, out=gp, ws=ws)
    torch.cuda.synchronize()
    dp.profile_enable(True)
    dp.profile_collect()
    t0 = time.perf_counter()
    for _ in range(reps):
        dp.backproject(g, angles, poses, proj, dp.W_FDK, out=vol, ws=ws)
    torch.cuda.synchronize()
    t_bp = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        dp.backproject_grad_pose(g, angles, poses, proj, e, dp.W_FDK, out=gp, ws=ws)
    torch.cuda.synchronize()
    t_bpg = (time.perf_counter() - t0) / reps
    kern = dp.profile_collect()
    dp.profile_enable(False)
    upd = float(g.nx) * g.ny * g.nz * V
    # per call (the views are processed in chunks: several launches per call)
    per_kernel = {k: round(v[0] / reps, 4) for k, v in kern.items()}
    launches = {k: v[1] // reps for k, v in kern.items()}
    log(f"[bench] BP {t_bp * 1e3:.2f} ms, BP-grad {t_bpg * 1e3:.2f} ms; kernels {per_kernel}")
    # The config's chain as written: the FDK pre-filter of the projections,
    # then per motion-compensation iteration the FDK back-projection, the
    # gradient-entropy loss and its gradient on the 512^3 volume, the
    # back-projection pose gradient and an Adam step on the 360 x 6 poses.
    from paper_2508_13304_amd import moco
    del vol, e
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q = moco.prefilter(g, proj)
    torch.cuda.synchronize()
    t_filter = time.perf_counter() - t0
    moco.estimate_motion(g, angles, q, iters=1)  # warm-up
    n_it = 3
    r = moco.estimate_motion(g, angles, q, iters=n_it)
    t_iter = r.seconds / n_it
    log(f"[bench] motion compensation: pre-filter {t_filter * 1e3:.2f} ms, "
        f"{t_iter * 1e3:.2f} ms per iteration")
    return {"workload": "512^3 recon at 0.375 mm, 360 views 512x384 at 0.776 mm, FDK weight, "
                        "sinusoidal motion 3 mm / 2 deg",
            "voxel_view_updates": upd,
            "backproject_updates_per_s": upd / t_bp,
            "backproject_grad_updates_per_s": upd / t_bpg,
            "backproject_ms": round(t_bp * 1e3, 3), "backproject_grad_ms": round(t_bpg * 1e3, 3),
            "kernels_ms": per_kernel, "launches_per_call": launches,
            "moco_chain": {"prefilter_ms": round(t_filter * 1e3, 3),
                           "iteration_ms": round(t_iter * 1e3, 3),
                           "iteration": "FDK back-projection + gradient-entropy loss and gradient "
                                        "+ back-projection pose gradient + Adam step (360 x 6)"}}


def run_registration(args, dp, torch, fw):
    """Registrations/s at 0.1 mm / 0.1 deg on the registration-scale workload:
    64 single-view targets rendered at the 64 candidate poses, each registered
    from the identity in one batched launch per iteration; Levenberg-Marquardt
    (analytic gradient + Gauss-Newton matrix) and BFGS with the default and
    with the autotuned kernel variants, LM also with a stopping step of one
    tenth of the target accuracy (on the accepted step, or on the
    Gauss-Newton step proposed at the accepted pose) and coarse to fine on a
    one- and a two-level resolution pyramid, and the Adam driver at the same
    batch.
    Success is always checked against the true poses."""
    from paper_2508_13304_amd import registration as reg
    dev = torch.device("cuda:0")
    c = fw["inputs"]
    g = c["geom"]
    T = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)  # noqa: E731
    vol = T(c["vol"], torch.float32)
    truth = T(c["poses"], torch.float64)
    angles = T(c["angles"], torch.float64)
    B = truth.shape[0]
    targets = dp.project_fwd(g, angles, truth, vol)
    init = torch.zeros_like(truth)
    out = {"workload": f"{B} single-view registrations, 256^3 phantom at 0.8 mm, 512x512 at 0.6 mm, "
                       "truth offsets +-10 mm/+-10 deg, start at identity, SSD loss"}

    def record(name, res):
        ok = reg.success(res.poses, truth)
        et, er = reg.pose_errors(res.poses, truth)
        out[name] = {"registrations_per_s": round(B / res.seconds, 3),
                     "successful_per_s": round(int(ok.sum()) / res.seconds, 3),
                     "success_rate": int(ok.sum()) / B, "seconds": round(res.seconds, 3),
                     "launch_pairs": res.launches,
                     "mean_iterations": float(res.iterations.double().mean()),
                     "median_err_mm": float(et.median()), "median_err_deg": float(er.median()),
                     "max_err_mm": float(et.max()), "max_err_deg": float(er.max())}
        if res.level_launches is not None and len(res.level_launches) > 1:
            out[name]["launches_per_level_finest_first"] = res.level_launches
        log(f"[bench] registration {name}: {out[name]}")

    reg.register_bfgs(g, vol, angles[:4], targets[:4], init[:4], iters=3)  # warm-up
    reg.register_lm(g, vol, angles[:4], targets[:4], init[:4], iters=3)
    record("lm_default_variants", reg.register_lm(g, vol, angles, targets, init))
    record("bfgs_default_variants", reg.register_bfgs(g, vol, angles, targets, init))
    out["autotuned_variants"] = {str(k): v for k, v in
                                 reg.autotune_registration(g, vol, angles, truth, targets).items()}
    record("lm_autotuned", reg.register_lm(g, vol, angles, targets, init))
    # stop once an accepted step is below one tenth of the target accuracy
    # (0.01 mm / 0.01 deg) instead of the library default 1e-4
    record("lm_autotuned_tol_0.01", reg.register_lm(g, vol, angles, targets, init, tol=1e-2))
    # ... and stopping once the undamped Gauss-Newton step at the accepted
    # pose is below that, which skips the evaluation that only confirms it
    record("lm_autotuned_newton_tol_0.01",
           reg.register_lm(g, vol, angles, targets, init, tol=1e-2, rule="newton"))
    # coarse to fine: the same rule, first on the volume averaged 2x2x2 and
    # the targets binned 2x2 (one level: 128^3 / 256^2 / 1 mm steps; two:
    # down to 64^3 / 128^2 / 2 mm), coarse levels stopping at 0.1 mm / 0.1 deg
    reg.register_lm(g, vol, angles[:4], targets[:4], init[:4], iters=3, levels=2)  # warm-up
    for lv in (1, 2):
        record(f"lm_pyramid{lv}_newton_tol_0.01",
               reg.register_lm(g, vol, angles, targets, init, tol=1e-2, rule="newton", levels=lv,
                               coarse_tol=0.1))
    record("bfgs_autotuned", reg.register_bfgs(g, vol, angles, targets, init))
    record("adam", reg.register(g, vol, angles, targets, init, iters=300, lr_t=3.0, lr_r_deg=2.0,
                                decay=0.99))
    return out


def run_registration_paper(args, dp, torch, fw):
    """Registration under the paper's imaging conditions (Sec. III-B): the
    registration-scale workload (64 single-view registrations, truth offsets
    +-10 mm / +-10 deg, start at the identity) with targets carrying Poisson
    noise of a transmission measurement at 1e5 photons per pixel.  Drivers:
    Levenberg-Marquardt on the SSD of the noisy line integrals, Adam on NCC
    with the paper's stopping rule (loss change < 1e-5 or NCC > 0.999; NCC <
    0.99 at the end is the paper's failure), and BFGS on NCC.  Reported per
    driver: success at 0.1 mm / 0.1 deg (and at 0.5 / 1 mm and deg for
    context), registrations/s and the mean absolute error per pose parameter."""
    from paper_2508_13304_amd import proposal as pr
    from paper_2508_13304_amd import registration as reg
    dev = torch.device("cuda:0")
    c = fw["inputs"]
    g = c["geom"]
    T = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)  # noqa: E731
    vol = T(c["vol"], torch.float32)
    truth = T(c["poses"], torch.float64)
    angles = T(c["angles"], torch.float64)
    B = truth.shape[0]
    photons = 1e5
    gen = torch.Generator(device=dev).manual_seed(13304)
    clean = dp.project_fwd(g, angles, truth, vol)
    # The synthetic phantom's line integrals reach far above a head's (the
    # detector would see no photons behind its densest rays at 1e5 photons):
    # the transmission model sees the attenuation scaled so that the largest
    # line integral of the targets is 5 (e^-5 of the photons get through, the
    # order of the paper's head data); the noisy values are returned in the
    # DRRs' own units.
    scale = 5.0 / float(clean.max())
    targets = synth.poisson_log_noise(clean, photons, gen, scale)
    del clean
    init = torch.zeros_like(truth)
    out = {"workload": f"{B} single-view registrations, 256^3 phantom at 0.8 mm, 512x512 at 0.6 mm, "
                       "truth offsets +-10 mm/+-10 deg, start at identity, targets with Poisson noise "
                       f"at {photons:.0e} photons per pixel (attenuation scaled so the largest line "
                       "integral is 5)", "photons": photons, "attenuation_scale": scale}

    def record(name, res):
        row = {"registrations_per_s": round(B / res.seconds, 3), "seconds": round(res.seconds, 3),
               "mean_iterations": float(res.iterations.double().mean()),
               "mae_tx_ty_tz_mm_gx_gy_gz_deg": pr.pose_mae(res.poses, truth)}
        for t in (0.1, 0.5, 1.0):
            ok = reg.success(res.poses, truth, t, t)
            row[f"success_{t:g}"] = int(ok.sum()) / B
        row["successful_per_s"] = round(row["success_0.1"] * B / res.seconds, 3)
        if res.failed is not None:
            row["paper_success_ncc_0.99"] = 1.0 - float(res.failed.double().mean())
        out[name] = row
        log(f"[bench] noisy registration {name}: {row}")

    reg.register_lm(g, vol, angles[:4], targets[:4], init[:4], iters=3)  # warm-up
    record("lm_ssd", reg.register_lm(g, vol, angles, targets, init))
    record("lm_ssd_pyramid2_newton_tol_0.01",
           reg.register_lm(g, vol, angles, targets, init, tol=1e-2, rule="newton", levels=2,
                           coarse_tol=0.1))
    record("adam_ncc_paper_stop", reg.register(g, vol, angles, targets, init, loss="ncc",
                                               stop="paper", iters=300, lr_t=3.0, lr_r_deg=2.0,
                                               decay=0.99))
    record("bfgs_ncc", reg.register_bfgs(g, vol, angles, targets, init, loss="ncc"))
    return out


def run_calibration_batch(args, dp, torch):
    """Uneven batched geometry calibration: 16 independent problems (cubic
    phantoms of 128^3-384^3 voxels spanning ~200 mm, 1-8 views each on
    256^2-768^2 detectors, every view's pose perturbed by +-5 mm/+-3 deg)
    registered by Levenberg-Marquardt on the SSD, entirely on the device.
    One iteration = the single-pass SSD / pose-gradient / Gauss-Newton launch
    for every view of all 16 problems + the FP64 update kernel.  Three ways
    to run it: one SSD launch per problem, the batched launch (variant
    chosen by timing each compiled variant on this batch), and the batched
    iteration captured once in a HIP graph and replayed; then the full
    calibration from the perturbed poses by graph replays."""
    from paper_2508_13304_amd.registration import BatchLM, pose_errors
    dev = torch.device("cuda:0")
    probs, truth = [], []
    n_samples = 0
    for q in synth.config4_problems(dev):
        g, angles, vol, tp = q["geom"], q["angles"], q["vol"], q["truth"]
        probs.append(dict(geom=g, angles=angles, vol=vol, target=dp.project_fwd(g, angles, tp, vol)))
        truth.append(tp)
        n_samples += count_ray_samples(g, angles.cpu().numpy(), np.zeros((len(angles), 6)))
    truth = torch.cat(truth)
    init = torch.zeros_like(truth)
    total_views = truth.shape[0]
    log(f"[bench] calibration batch: 16 problems, {total_views} views, {n_samples:.3e} samples/iteration")
    ws1 = torch.empty(max(dp.workspace_bytes(q["geom"], q["angles"].numel(), dp.OP_FWD_SSD)
                          for q in probs), dtype=torch.uint8, device=dev)

    def timed(fn, reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    reps = max(3, min(args.steps, 10))
    lm = BatchLM(probs, init)
    lm.step_sequential(ws1)
    lm.reset(init)
    t_seq = timed(lambda: lm.step_sequential(ws1), reps)
    # batch autotuning: time each compiled variant of the batched launch
    ms = {}
    for var in range(dp.N_VARIANTS):
        lm.variant = var
        lm.reset(init)
        lm.step()
        lm.reset(init)
        ms[var] = timed(lm.step, reps)
    lm.variant = min(ms, key=ms.get)
    lm.reset(init)
    t_batch = timed(lm.step, reps)
    lm.reset(init)
    lm.capture()
    t_graph = timed(lambda: lm.run(1), reps)
    def converge(max_iters=60):
        """Graph replays from the perturbed poses until every view has
        converged (one host check per iteration), at most max_iters."""
        lm.reset(init)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = 0
        while n < max_iters:
            lm.run(1)
            n += 1
            if bool(lm.state["done"].bool().all()):
                break
        torch.cuda.synchronize()
        return n, time.perf_counter() - t0

    # the calibration itself
    iters, t_cal = converge()
    pose, conv, _ = lm.result()
    te, re = pose_errors(pose, truth)
    ok = (te <= 0.1) & (re <= 0.1)

    # the same calibration stopping once an accepted step is below one tenth
    # of the target accuracy (the update kernel takes tol as an argument, so
    # the iteration is captured again)
    lm.tol = 1e-2
    lm.reset(init)
    lm.capture()
    iters2, t_cal2 = converge()
    pose2, conv2, _ = lm.result()
    te2, re2 = pose_errors(pose2, truth)
    ok2 = (te2 <= 0.1) & (re2 <= 0.1)
    res = {"workload": "16 problems, 128^3-384^3 phantoms (~200 mm), 1-8 views each on 256^2-768^2 "
                       "detectors, every view's pose perturbed +-5 mm/+-3 deg; Levenberg-Marquardt on "
                       "the SSD; one iteration = single-pass SSD + pose gradient + Gauss-Newton "
                       "launch for all views + FP64 update kernel",
           "views": total_views, "samples_per_iteration": n_samples,
           "sequential_ms": round(t_seq * 1e3, 3), "batched_ms": round(t_batch * 1e3, 3),
           "graph_ms": round(t_graph * 1e3, 3),
           "graph_samples_per_s": n_samples / t_graph,
           "sequential_samples_per_s": n_samples / t_seq,
           "batch_variant": lm.variant,
           "variant_ms": {str(k): round(v * 1e3, 3) for k, v in ms.items()},
           "calibration": {"iterations": iters, "seconds": round(t_cal, 4),
                           "views_within_0.1mm_0.1deg": int(ok.sum()),
                           "success_rate": int(ok.sum()) / ok.numel(),
                           "converged": int(conv.sum()),
                           "max_err_mm": float(te.max()), "max_err_deg": float(re.max())},
           "calibration_tol_0.01": {"iterations": iters2, "seconds": round(t_cal2, 4),
                                    "views_within_0.1mm_0.1deg": int(ok2.sum()),
                                    "success_rate": int(ok2.sum()) / ok2.numel(),
                                    "converged": int(conv2.sum()),
                                    "max_err_mm": float(te2.max()), "max_err_deg": float(re2.max())}}
    log(f"[bench] calibration batch: {res}")
    return res


def run_learned(args, dp, torch):
    """Learned proposal + refinement against the plain registration from the
    identity on unseen 192^3 phantoms (offsets +-30 mm / +-20 deg)."""
    from paper_2508_13304_amd import proposal as pr
    if not os.path.exists(pr.WEIGHTS):
        log("[bench] no trained proposal weights; learned leg skipped")
        return None
    net = pr.ProposalNet.load(pr.WEIGHTS)
    res = pr.evaluate(net, synth.geom_c5(), n_phantoms=4, per_phantom=16, log=log)
    res["workload"] = ("4 unseen 192^3 phantoms at 1 mm x 16 offsets (+-30 mm/+-20 deg), one 256x256 "
                       "view at 1.2 mm, SSD loss; both refined by Levenberg-Marquardt; plain = from identity")
    noisy = pr.evaluate(net, synth.geom_c5(), n_phantoms=4, per_phantom=16, log=log, photons=1e5)
    noisy["workload"] = res["workload"] + "; targets with Poisson noise at 1e5 photons per pixel"
    res["noisy"] = noisy
    return res


BF16_PEAK_TFLOPS = 2500.0  # dense BF16 MFMA, MI355X


def proposal_train_flops(net, batch):
    """Algorithmic FLOPs of one training step (FMA counted as 2): per
    convolution, 2 M K Co for the forward product and again for the weight
    gradient and (all but the first layer) the input gradient, with
    M = batch Ho Wo and K = 9 Ci; the same three for the linear head."""
    total, hw = 0, net.size
    for li, (W, _, s) in enumerate(net.convs):
        hw = (hw - 1) // s + 1
        f = 2 * batch * hw * hw * W.shape[1] * W.shape[0]
        total += f * (2 if li == 0 else 3)
    return total + 3 * 2 * batch * net.Wfc.shape[1] * net.Wfc.shape[0]


def run_proposal_training(args, dp, torch, steps=10, batch=256):
    """One training step of the pose-proposal CNN at batch 256 (256x256 pair
    images, forward + backward + Adam, every product on the BF16 MFMA GEMM),
    on seeded synthetic inputs and labels; time per step against the dense
    BF16 peak."""
    from paper_2508_13304_amd import proposal as pr
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev).manual_seed(11)
    net = pr.ProposalNet(size=256, device=dev, seed=1)
    x = torch.rand((batch, net.size, net.size, 2), generator=gen, device=dev).to(torch.bfloat16)
    y = torch.rand((batch, 6), generator=gen, device=dev) * 2 - 1

    def step():
        out, cache = net.forward(x, keep=True)
        d = out - y
        grads, head = net.backward(cache, (2.0 / d.numel()) * d)
        net.adam_step(grads, head, lr=1e-4)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    flops = proposal_train_flops(net, batch)
    tf = flops / (ms * 1e-3) / 1e12
    res = {"batch": batch, "ms_per_step": round(ms, 3), "flops_per_step": flops,
           "tflops": round(tf, 2), "bf16_peak_tflops": BF16_PEAK_TFLOPS,
           "frac": round(tf / BF16_PEAK_TFLOPS, 4),
           "what": "ProposalNet(256x256x2, channels 32-64-128-256-256-256, stride 2) forward + backward + Adam"}
    log(f"[bench] proposal training step: {res}")
    return res


PAPER_LADDER = [(128, 192), (256, 384), (384, 572), (512, 768)]
# The paper's own cost tables (RTX 4090; context, not targets): seconds for
# 100 iterations of a differentiable forward projection of 1 view, and for
# one differentiable back-projection of 256 views.
PAPER_FWD_S = {"rd": [1.25, 2.44, 6.24, 12.70], "dd": [1.27, 3.84, 11.02, 23.58],
               "sf": [1.41, 5.03, 14.49, 32.53]}
PAPER_BP_S = {"vd": [0.17, 1.21, 3.99, 9.50], "dd": [0.65, 4.99, 16.72, 39.52],
              "sf": [1.12, 8.45, 28.55, 69.72]}


def run_paper_ladder(args, dp, torch):
    """Every projector type at the paper's cost-table shapes: (128n)^3
    volumes at 256/(128n) mm, (192n)^2 detectors (572 at n = 3) at
    384/(192n) mm.  Forward: one view, time of 100 iterations of projection +
    pose gradient (RD: the single-pass SSD kernel, with the default and with
    the autotuned variant; SF, DD: projection then gradient).  Back-projection: 256 views over 360 deg, one back-projection
    + pose gradient.  Peak device memory per case and projector type (GB,
    torch's allocator peak over the projector's own step: inputs, outputs and
    the library workspace)."""
    dev = torch.device("cuda:0")
    out = {"fwd": {}, "bp": {}, "paper_fwd_s": PAPER_FWD_S, "paper_bp_s": PAPER_BP_S,
           "note": "paper figures are RTX 4090 timings from its cost tables; context only"}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    for n, (nv_, nd) in enumerate(PAPER_LADDER, start=1):
        h = 256.0 / nv_
        du = 384.0 / nd
        g = synth.Geom(nv_, nv_, nv_, h, h, h, nd, nd, du, du)
        rng = synth.rng_for(5, n)
        vol = synth.ellipsoid_phantom_torch(nv_, h, 20, rng, dev, shell=True)
        key = f"{nv_}^3/{nd}^2"
        # forward, 1 view
        a1 = torch.zeros(1, dtype=torch.float64, device=dev)
        p1 = torch.tensor(synth.random_poses(1, 5.0, 5.0, rng), dtype=torch.float64, device=dev)
        y1 = dp.project_fwd(g, a1, torch.zeros_like(p1), vol)
        res = {}
        peak = {}

        def reset():
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            torch.cuda.reset_peak_memory_stats(dev)

        def peak_gb():
            torch.cuda.synchronize()
            return round(torch.cuda.max_memory_allocated(dev) / 1e9, 3)

        reset()
        res["rd"] = timed(lambda: dp.project_fwd_ssd_grad_pose(g, a1, p1, vol, y1), 10) * 100
        peak["rd"] = peak_gb()
        # the same step with the variant (tile shape x chunk class) the
        # autotuner picks for this shape (it keeps it for later calls)
        res["rd_variant"], _ = dp.autotune(dp.OP_FWD_SSD, g, a1, p1, vol, torch.empty_like(y1),
                                           grad_proj=y1, reps=3)
        res["rd_autotuned"] = timed(lambda: dp.project_fwd_ssd_grad_pose(g, a1, p1, vol, y1),
                                    10) * 100
        for kind in ("sf", "dd"):
            def step(kind=kind):
                l = dp.fp_project(g, a1, p1, vol, kind)
                dp.fp_project_grad_pose(g, a1, p1, vol, 2.0 * (l - y1), kind)
            reset()
            res[kind] = timed(step, 3) * 100
            peak[kind] = peak_gb()
        res["peak_gb"] = peak
        out["fwd"][key] = {k: round(v, 4) if isinstance(v, float) else v for k, v in res.items()}
        # back-projection, 256 views
        V = 256
        ang = torch.tensor(np.arange(V) * 2 * math.pi / V, dtype=torch.float64, device=dev)
        pos = torch.tensor(synth.random_poses(V, 2.0, 1.0, rng), dtype=torch.float64, device=dev)
        gen = torch.Generator(device=dev).manual_seed(n)
        proj = torch.rand((V, nd, nd), device=dev, generator=gen)
        e = torch.randn(vol.shape, device=dev, generator=gen)
        res = {}
        peak = {}
        def vd_step():
            dp.backproject(g, ang, pos, proj, dp.W_NONE)
            dp.backproject_grad_pose(g, ang, pos, proj, e, dp.W_NONE)
        reset()
        res["vd"] = timed(vd_step, 2)
        peak["vd"] = peak_gb()
        for kind in ("sf", "dd"):
            def bstep(kind=kind):
                dp.fp_backproject(g, ang, pos, proj, kind)
                dp.fp_backproject_grad_pose(g, ang, pos, proj, e, kind)
            reset()
            res[kind] = timed(bstep, 1)
            peak[kind] = peak_gb()
        res["peak_gb"] = peak
        out["bp"][key] = {k: round(v, 4) if isinstance(v, float) else v for k, v in res.items()}
        log(f"[bench] ladder {key}: fwd(100 it) {out['fwd'][key]} s; bp(256 views) {out['bp'][key]} s")
        del vol, proj, e
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a bounded sample of the same workload
# ---------------------------------------------------------------------------

def _host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def run_cpu_baseline(fw, n_poses=16, n_bp_views=8):
    """The plain FP64 oracle on the host cores (not a tuned CPU projector):
    forward + SSD pose gradient on a sample of the registration-scale poses
    with all threads and with one, and the back-projector and its pose
    gradient on a sample of the reconstruction-scale views."""
    import oracle
    c = fw["inputs"]
    g = c["geom"]
    host = _host_cpu()
    threads = oracle.num_threads()
    angles, poses = c["angles"][:n_poses], c["poses"][:n_poses]
    y = oracle.project_fwd(g, [0.0], c["target_pose"], c["vol"])

    def fwd_grad(geom, a, p, target):
        t0 = time.perf_counter()
        l = oracle.project_fwd(geom, a, p, c["vol"])
        oracle.project_fwd_grad_pose(geom, a, p, c["vol"], 2.0 * (l - target))
        return time.perf_counter() - t0

    n = count_ray_samples(g, angles, poses)
    dt = fwd_grad(g, angles, poses, y)
    log(f"[bench] oracle: {n_poses} poses in {dt:.2f} s ({threads} threads; {host})")
    # one thread, first pose, the detector's central 128 rows (the same rays as
    # those rows of the full detector: the row centre stays on the axis)
    gband = g.replace(nv=128)
    yband = y[:, (g.nv - 128) // 2:(g.nv + 128) // 2]
    n1 = count_ray_samples(gband, angles[:1], poses[:1])
    oracle.set_num_threads(1)
    try:
        dt1 = fwd_grad(gband, angles[:1], poses[:1], yband)
    finally:
        oracle.set_num_threads(threads)
    log(f"[bench] oracle: central 128 rows of 1 pose in {dt1:.2f} s (1 thread)")
    # back-projection sample: the first views of the 360-view motion at 512^3
    gb = synth.geom_c3_recon()
    m = synth.config3_motion()
    rng = np.random.default_rng(3)
    proj = synth.smooth_images(n_bp_views, gb.nv, gb.nu, rng, n_blobs=4, signed=True).astype(np.float64)
    a_b, p_b = m["angles"][:n_bp_views], m["poses"][:n_bp_views]
    t0 = time.perf_counter()
    oracle.backproject(gb, a_b, p_b, proj, oracle.W_FDK)
    t_bp = time.perf_counter() - t0
    e = np.random.default_rng(5).standard_normal((gb.nz, gb.ny, gb.nx))
    t0 = time.perf_counter()
    oracle.backproject_grad_pose(gb, a_b, p_b, proj, e, oracle.W_FDK)
    t_bpg = time.perf_counter() - t0
    upd = gb.nx * gb.ny * gb.nz * n_bp_views
    log(f"[bench] oracle: back-projection {n_bp_views} views in {t_bp:.2f} s, gradient {t_bpg:.2f} s")
    return {"value": n / dt, "unit": "ray-samples/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_poses} of 64 poses, all 512x512 rays, forward + SSD pose gradient "
                      f"({n:.3e} samples, {dt:.1f} s); plain FP64 oracle, not a tuned CPU projector",
            "host": host,
            "one_thread": {"value": n1 / dt1, "unit": "ray-samples/s", "cores": 1,
                           "sample": f"first pose, central 128 of 512 detector rows, forward + SSD pose "
                                     f"gradient ({n1:.3e} samples, {dt1:.1f} s)"},
            "backprojector": {"backproject_updates_per_s": upd / t_bp,
                              "backproject_grad_updates_per_s": upd / t_bpg, "cores": threads,
                              "sample": f"first {n_bp_views} of 360 views at 512^3 with the FDK weight "
                                        f"({upd:.3e} voxel-view updates; {t_bp:.1f} s back-projection, "
                                        f"{t_bpg:.1f} s gradient); the full 360 views take 45x as long"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-bp", action="store_true", help="skip the back-projector leg")
    ap.add_argument("--no-fwd", action="store_true", help="skip the forward leg (profiling runs)")
    ap.add_argument("--no-reg", action="store_true", help="skip the registration legs")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch calibration leg")
    ap.add_argument("--no-ladder", action="store_true",
                    help="skip the projector-type comparison at the paper's cost-table shapes")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration) and exit")
    ap.add_argument("--probe-calib", action="store_true",
                    help="only run one L2 and one HBM read-probe launch (L2 counter calibration) and exit")
    ap.add_argument("--no-probe", action="store_true", help="skip the L2 / HBM read-bandwidth probe")
    ap.add_argument("--no-train", action="store_true", help="skip the proposal-network training step")
    ap.add_argument("--train-only", action="store_true",
                    help="only time the proposal-network training step (profiling runs) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the projector shards by view / voxel slab across GPUs, see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}), flush=True)
        return
    import paper_2508_13304_amd as dp
    dp.load()
    if args.probe_calib:
        dev = torch.device("cuda:0")
        l2 = torch.ones(1 << 19, dtype=torch.float32, device=dev)   # 2 MiB footprint
        hbm = torch.ones(1 << 29, dtype=torch.float32, device=dev)  # 2 GiB
        torch.cuda.synchronize()
        dp.read_probe(l2, 32, True, 2048)    # 2048 blocks x 32 passes x 2 MiB = 128 GiB requested
        dp.read_probe(hbm, 1, False, 4096)   # every element of 2 GiB once
        torch.cuda.synchronize()
        print(json.dumps({"l2_probe_bytes": 2048 * 32 * l2.numel() * 4,
                          "hbm_probe_bytes": hbm.numel() * 4}), flush=True)
        return
    if args.train_only:
        print(json.dumps({"proposal_training": run_proposal_training(args, dp, torch)}), flush=True)
        return
    if args.no_fwd:
        bp = run_backproject(args, dp, torch)
        print(json.dumps({"backprojector": bp}), flush=True)
        return
    fw = run_forward(args, dp, torch)
    probe = None if args.no_probe else run_cache_probe(dp, torch)
    bp = None if args.no_bp else run_backproject(args, dp, torch)
    regr = None if args.no_reg else run_registration(args, dp, torch, fw)
    regr_noisy = None if args.no_reg else run_registration_paper(args, dp, torch, fw)
    learned = None if args.no_reg else run_learned(args, dp, torch)
    calib = None if args.no_batch else run_calibration_batch(args, dp, torch)
    training = None if args.no_train else run_proposal_training(args, dp, torch)
    ladder = None if args.no_ladder else run_paper_ladder(args, dp, torch)
    cpu = None if args.no_cpu else run_cpu_baseline(fw)
    value = fw["n_samples"] / (fw["ms_step"] * 1e-3)
    reg_rate = reg_method = None
    if regr:
        best = max(((k, v) for k, v in regr.items() if isinstance(v, dict)
                    and "registrations_per_s" in v and v.get("success_rate", 0) >= 1.0),
                   key=lambda kv: kv[1]["registrations_per_s"], default=None)
        reg_rate = best[1]["registrations_per_s"] if best else None
        reg_method = best[0] if best else None
    rec = {
        "metric": "fwd+pose-grad ray-samples/s; 6-DoF registrations/s at <0.1mm/0.1° error",
        "value": value,
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fw["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "registration scale: 256^3 ellipsoid+shell phantom at 0.8 mm, 64 candidate poses "
                               "(+-10 mm/+-10 deg) x one 512x512 view at 0.6 mm, SAD/SDD 1000/1500 mm, "
                               "0.5 mm trilinear march; forward + SSD loss + 64x6 pose gradient in one fused launch",
                   "samples_per_step": fw["n_samples"], "views": fw["V"]},
        "registrations_per_s": reg_rate,
        "registrations_unit": "registrations/s at <0.1 mm / 0.1 deg (64 single-view targets, "
                              "+-10 mm / +-10 deg, best method with every registration successful)",
        "registrations_method": reg_method,
        "roofline": fw["roofline"],
        "gather_roofline": gather_roofline(fw, probe) if probe else None,
        "cpu_baseline": cpu,
        "kernels_ms": fw["per_kernel"],
        "two_call_step": {"ms_per_step": round(fw["two_call_ms"], 4),
                          "value": fw["n_samples"] / (fw["two_call_ms"] * 1e-3),
                          "kernels_ms": fw["two_call_kernels"]},
        "autograd_step": {"ms_per_step": round(fw["autograd_ms"], 4),
                          "value": fw["n_samples"] / (fw["autograd_ms"] * 1e-3),
                          "kernels_ms": fw["autograd_kernels"],
                          "what": "ProjectFwd.apply + torch SSD + loss.backward() for the 64 poses"},
        "backprojector": dict(bp, rooflines=vd_rooflines(bp, probe)) if bp and probe else bp,
        "registration": regr,
        "registration_noisy": regr_noisy,
        "learned_proposal": learned,
        "proposal_training": training,
        "calibration_batch": calib,
        "projector_ladder": ladder,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
