"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/*.h, and rejects invalid arguments before any launch."""
import ctypes as C
import glob
import os
import re
import subprocess

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(dp_\w+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    import paper_2508_13304_amd as m
    return m.load()


def test_library_exports_every_declared_symbol(lib):
    import paper_2508_13304_amd as m
    declared = _declared_functions()
    assert len(declared) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", m.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(dp_\w+)", out))
    missing = [n for n in declared if n not in exported]
    assert not missing, missing
    assert set(m.EXPORTS) <= set(declared)
    for n in declared:
        assert hasattr(lib, n)


def test_struct_layout_matches_header(lib):
    import paper_2508_13304_amd as m
    # int32 x3, double x3, int32 x2, double x7 with natural alignment
    assert C.sizeof(m.DPGeom) == 4 * 3 + 4 + 8 * 3 + 4 * 2 + 8 * 7
    assert lib.dp_version() == 10000


def test_workspace_query(lib):
    import paper_2508_13304_amd as m
    g = synth.geom_c1()
    for op in range(9):  # DP_OP_FWD .. DP_OP_SF_BP_GRAD
        assert m.workspace_bytes(g, 1, op) > 0
        assert m.workspace_bytes(g, 1, op) % 256 == 0
    assert m.workspace_bytes(g, 0, 0) == 0
    assert m.workspace_bytes(g, 1, 9) == 0
    assert m.workspace_bytes(g, 1, -1) == 0
    assert m.workspace_bytes(g.replace(sdd=900.0), 1, 0) == 0
    # grows with the number of views for the image-sized buffers
    assert m.workspace_bytes(g, 8, m.OP_BP) > m.workspace_bytes(g, 1, m.OP_BP)


def _call_fwd(lib, g, V=1, ws_bytes=None, ptr=1 << 20, ws=None):
    import paper_2508_13304_amd as m
    gs = m.geom_struct(g)
    wsb = ws_bytes if ws_bytes is not None else m.workspace_bytes(g, max(V, 1), 0)
    wsp = C.c_void_p(ws if ws is not None else 1 << 24)
    p = C.c_void_p(ptr) if ptr else None
    return lib.dp_project_fwd(C.byref(gs), V, p, p, p, p, wsp, wsb, None)


def test_invalid_arguments_rejected_before_launch(lib):
    import paper_2508_13304_amd as m
    g = synth.geom_c1()
    assert lib.dp_project_fwd(None, 1, None, None, None, None, None, 0, None) == -1
    assert b"NULL" in lib.dp_last_error()
    assert _call_fwd(lib, g.replace(nx=0)) == -1
    assert _call_fwd(lib, g.replace(sdd=1000.0)) == -1
    assert b"sad" in lib.dp_last_error()
    assert _call_fwd(lib, g.replace(step=0.0)) == -1
    assert _call_fwd(lib, g.replace(vx=float("nan"))) == -1
    assert _call_fwd(lib, g, V=0) == -1
    assert _call_fwd(lib, g, V=70000) == -4
    assert _call_fwd(lib, g, ptr=0) == -1
    assert _call_fwd(lib, g, ws_bytes=16) == -2
    assert b"workspace" in lib.dp_last_error()
    assert _call_fwd(lib, g, ws=(1 << 24) + 8) == -1  # misaligned workspace
    big = g.replace(nx=2000, ny=2000, nz=2000)
    assert _call_fwd(lib, big) == -4
    # a long thin volume: fewer than 2^31 padded voxels, but an x extent that
    # 16-bit box origins cannot hold
    assert _call_fwd(lib, g.replace(nx=65532, ny=4, nz=4, vx=0.01)) == -4
    assert b"indexing" in lib.dp_last_error()
    gs = m.geom_struct(g)
    p = C.c_void_p(1 << 20)
    ws = m.workspace_bytes(g, 1, m.OP_BP)
    assert lib.dp_backproject(C.byref(gs), 1, p, p, p, p, 5, p, ws, None) == -1
    assert b"weight_mode" in lib.dp_last_error()
    wsg = m.workspace_bytes(g, 1, m.OP_BP_GRAD)
    assert lib.dp_backproject_grad_pose(C.byref(gs), 1, p, p, p, None, p, 0, C.c_void_p(1 << 24),
                                        wsg, None) == -1
    wsf = m.workspace_bytes(g, 1, m.OP_FWD_GRAD)
    assert lib.dp_project_fwd_grad_pose(C.byref(gs), 1, p, p, p, p, p, C.c_void_p(1 << 24),
                                        wsf - 1, None) == -2


def test_newer_entries_validate_before_launch(lib):
    """Single-pass SSD, footprint, FDK, sharpness, entropy and CNN entries:
    bad arguments return an error code (and a message) before any launch, so
    these run without a GPU."""
    import paper_2508_13304_amd as m
    g = synth.geom_c1()
    gs = m.geom_struct(g)
    p = C.c_void_p(1 << 20)
    ws = C.c_void_p(1 << 24)
    wss = m.workspace_bytes(g, 1, m.OP_FWD_SSD)
    # single-pass SSD: NULL target, short workspace, NULL Hessian
    assert lib.dp_project_fwd_ssd_grad_pose(C.byref(gs), 1, p, p, p, None, p, None, p, ws, wss,
                                            None) == -1
    assert lib.dp_project_fwd_ssd_grad_pose(C.byref(gs), 1, p, p, p, p, p, None, p, ws, wss - 256,
                                            None) == -2
    assert lib.dp_project_fwd_ssd_gauss_newton(C.byref(gs), 1, p, p, p, p, p, None, p, None, ws,
                                               wss, None) == -1
    # footprint pairs: kind, NULLs, workspace
    wf = m.workspace_bytes(g, 1, m.OP_FP_FWD_GRAD)
    assert lib.dp_fp_project_grad_pose(C.byref(gs), 1, p, p, p, p, p, 2, ws, wf, None) == -1
    assert b"kind" in lib.dp_last_error()
    assert lib.dp_fp_project_grad_pose(C.byref(gs), 1, p, p, p, p, None, 0, ws, wf, None) == -1
    assert lib.dp_fp_backproject(C.byref(gs), 1, p, p, None, p, 1, ws,
                                 m.workspace_bytes(g, 1, m.OP_FP_BP), None) == -1
    assert lib.dp_fp_backproject_grad_pose(C.byref(gs), 1, p, p, p, p, p, 1, ws,
                                           m.workspace_bytes(g, 1, m.OP_FP_BP_GRAD) - 256, None) == -2
    # FDK filter: rows too long, non-finite scale
    long_rows = m.geom_struct(g.replace(nu=4001))
    assert lib.dp_fdk_filter(C.byref(long_rows), 1, p, p, 1.0, None) == -4
    assert lib.dp_fdk_filter(C.byref(gs), 1, p, p, float("inf"), None) == -1
    # sharpness / gradient entropy: sizes, workspace, eps
    wsh = lib.dp_sharpness_workspace_bytes(8, 8, 8)
    assert wsh > 0 and wsh % 256 == 0
    assert lib.dp_sharpness(0, 8, 8, p, p, None, ws, wsh, None) == -1
    assert lib.dp_sharpness(8, 8, 8, p, p, None, ws, wsh - 256, None) == -2
    wge = lib.dp_gradient_entropy_workspace_bytes(8, 8, 8)
    assert lib.dp_gradient_entropy(8, 8, 8, p, 0.0, p, None, ws, wge, None) == -1
    assert lib.dp_gradient_entropy(8, 8, 8, p, 1e-12, p, None, C.c_void_p((1 << 24) + 4), wge,
                                   None) == -1  # misaligned workspace
    # kernel variants: every ray-driven op, including the single-pass SSD
    for op in (m.OP_FWD, m.OP_FWD_GRAD, m.OP_FWD_SSD):
        assert lib.dp_get_variant(C.byref(gs), 1, op) in range(m.N_VARIANTS)
        assert lib.dp_set_variant(op, m.N_VARIANTS) == -1
        assert lib.dp_set_variant(op, m.N_VARIANTS - 1) == 0
        assert lib.dp_get_variant(C.byref(gs), 1, op) == m.N_VARIANTS - 1
        assert lib.dp_set_variant(op, -1) == 0
    assert lib.dp_get_variant(C.byref(gs), 1, m.OP_BP) == -1
    assert lib.dp_set_variant(m.OP_BP, 0) == -1
    # implicit-GEMM convolutions: channel multiples of 8, row length, NULL,
    # alignment (all refused before any launch)
    a16 = C.c_void_p(1 << 20)
    assert lib.dp_conv3x3_fwd_bf16(2, 8, 8, 6, 16, 2, a16, a16, 56, a16, 1, 1, a16, None) == -1
    assert lib.dp_conv3x3_fwd_bf16(2, 8, 8, 8, 16, 2, a16, a16, 64, a16, 1, 1, a16, None) == -1
    assert lib.dp_conv3x3_fwd_bf16(2, 8, 8, 8, 16, 2, a16, None, 72, a16, 1, 1, a16, None) == -1
    assert lib.dp_conv3x3_fwd_bf16(2, 8, 8, 8, 16, 2, C.c_void_p((1 << 20) + 8), a16, 72, a16, 1,
                                   1, a16, None) == -1
    assert lib.dp_conv3x3_wgrad_bf16(2, 8, 8, 8, 16, 2, a16, a16, 72, 1, a16, None, 0, None) == -1
    assert lib.dp_conv3x3_wgrad_ws_bytes(2, 8, 8, 8, 16, 2, 72) == 0
    assert lib.dp_conv3x3_dgrad_act_bf16(2, 8, 8, 8, 16, 2, a16, a16, 72, None, 1, a16, None) == -1
    # CNN helpers: 32-bit index spaces
    assert lib.dp_im2col3x3_bf16(512, 256, 256, 64, 1, p, p, None) == -4
    assert lib.dp_col2im3x3(512, 256, 256, 64, 1, p, p, None) == -4
    assert lib.dp_im2col3x3_bf16(0, 8, 8, 8, 1, p, p, None) == -1


def test_batch_ssd_and_lm_update_validate_before_launch(lib):
    """Batched single-pass SSD and the device LM update: the batch workspace
    is the sum of the per-problem ones (so the problem array's layout matches
    the header), and bad arguments are refused before any launch."""
    import paper_2508_13304_amd as m
    g1, g2 = synth.geom_c1(), synth.geom_c1().replace(nx=40, nu=70)
    arr = (m.DPProblem * 2)()
    p = 1 << 20
    for i, (g, V) in enumerate(((g1, 3), (g2, 5))):
        arr[i].geom = m.geom_struct(g)
        arr[i].n_views = V
        arr[i].angles = arr[i].poses = arr[i].vol = arr[i].proj = p
        arr[i].grad_proj = arr[i].grad_pose = arr[i].hess = p
    need = lib.dp_batch_workspace_bytes(arr, 2, m.OP_FWD_SSD)
    assert need == m.workspace_bytes(g1, 3, m.OP_FWD_SSD) + m.workspace_bytes(g2, 5, m.OP_FWD_SSD)
    ws = C.c_void_p(1 << 24)
    assert lib.dp_project_fwd_ssd_gauss_newton_batch(arr, 2, ws, need - 256, -1, None) == -2
    assert lib.dp_project_fwd_ssd_gauss_newton_batch(arr, 2, ws, need, m.N_VARIANTS, None) == -1
    assert lib.dp_project_fwd_ssd_gauss_newton_batch(arr, 17, ws, need, -1, None) == -4
    arr[1].hess = None
    assert lib.dp_project_fwd_ssd_gauss_newton_batch(arr, 2, ws, need, -1, None) == -1
    assert b"problem 1" in lib.dp_last_error()
    q = C.c_void_p(p)
    args = [q] * 10
    assert lib.dp_lm_update(0, *args, 1e-4, None) == -1
    assert lib.dp_lm_update(4, *args, -1.0, None) == -1
    assert lib.dp_lm_update(4, *(args[:9] + [None]), 1e-4, None) == -1
    assert b"NULL" in lib.dp_last_error()


def test_read_probe_argument_validation(lib):
    """The measurement probe rejects bad arguments before any launch."""
    buf, out = C.c_void_p(1 << 20), C.c_void_p(1 << 21)
    assert lib.dp_read_probe(None, 2048, 1, 1, 1, out, None) == -1
    assert lib.dp_read_probe(buf, 2048, 1, 1, 1, None, None) == -1
    assert lib.dp_read_probe(C.c_void_p((1 << 20) + 4), 2048, 1, 1, 1, out, None) == -1
    assert b"aligned" in lib.dp_last_error()
    assert lib.dp_read_probe(buf, 0, 1, 0, 1, out, None) == -1
    assert lib.dp_read_probe(buf, 2048, 0, 1, 1, out, None) == -1
    assert lib.dp_read_probe(buf, 2048, 1, 1, 0, out, None) == -1
    assert lib.dp_read_probe(buf, 3072, 1, 1, 1, out, None) == -1   # not a power of two
    assert lib.dp_read_probe(buf, 1024, 1, 1, 1, out, None) == -1   # below 2048
    assert b"power of two" in lib.dp_last_error()
    assert lib.dp_read_probe(buf, (1 << 32) - 256, 1, 0, 1, out, None) == -4
    assert lib.dp_read_probe(buf, 2048, 1, 0, (1 << 20) + 1, out, None) == -4


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_2508_13304_amd as m
    saved = m._lib
    try:
        m._lib = None
        with pytest.raises(RuntimeError, match="not built"):
            m.load(str(tmp_path / "missing.so"))
    finally:
        m._lib = saved


def test_python_tables_match_the_header():
    """The binding's kernel-name table follows the header's DP_K_* order, and
    its op and footprint-kind constants equal the header's."""
    import paper_2508_13304_amd as m
    src = open(os.path.join(ROOT, "include", "diffproj.h")).read()
    ks = sorted((int(v), n) for n, v in re.findall(r"\bDP_K_(\w+)\s*=\s*(\d+)", src) if n != "COUNT")
    names = {"SETUP": "setup", "VOL_PREP": "vol_prep", "RD_FWD": "rd_fwd", "RD_GRAD": "rd_grad",
             "DET_PREP": "det_prep", "VD_BP": "vd_bp", "VD_GRAD": "vd_grad", "FINALIZE": "finalize",
             "FDK_FILTER": "fdk_filter", "SHARPNESS": "sharpness", "RD_FUSED": "rd_fused",
             "SF": "footprint"}
    assert [names[n] for _, n in ks] == list(m.KERNELS)
    count = int(re.search(r"\bDP_K_COUNT\s*=\s*(\d+)", src).group(1))
    assert count == len(m.KERNELS)
    ops = dict(re.findall(r"\bDP_OP_(\w+)\s*=\s*(\d+)", src))
    for n, v in ops.items():
        assert getattr(m, "OP_" + n) == int(v), n
    kinds = dict(re.findall(r"\bDP_FP_(SF|DD)\s*=\s*(\d+)", src))
    assert m.FP_KINDS == {"sf": int(kinds["SF"]), "dd": int(kinds["DD"])}
