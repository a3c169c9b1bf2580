"""Learned 6-DoF pose proposal for 2D/3D registration.

A 6-layer strided CNN (3x3 kernels, stride 2, channels 32-64-128-256-256-256,
ReLU) reads a pair of DRRs -- the reference rendered at the identity pose and
the target image -- as a 2-channel NHWC image and a linear head regresses the
pose offset (normalised by the training range).  Every layer runs on the
library's BF16 MFMA GEMM with FP32 accumulation (im2col, GEMM, fused
bias/ReLU epilogue; backward via two GEMMs, col2im and a column sum); the
parameters are kept in FP32 and rounded to BF16 for each step.  The
network's proposal initialises the analytic-gradient registration, whose
plain form (started from the identity) is the fallback.
"""
from __future__ import annotations

import argparse
import ctypes as C
import dataclasses
import json
import math
import os
import sys
import time

import torch

from . import _check, _stream, load
from . import project_fwd as _project_fwd

CHANNELS = (32, 64, 128, 256, 256, 256)
# Training range of the pose offset: translations +-30 mm, rotations +-20 deg;
# the network regresses the offset divided by these (order tx ty tz gx gy gz).
T_RANGE_MM = 30.0
R_RANGE_DEG = 20.0
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                       "proposal_192vox_256px.safetensors")


def label_scale(device) -> torch.Tensor:
    return torch.tensor([T_RANGE_MM] * 3 + [math.radians(R_RANGE_DEG)] * 3,
                        dtype=torch.float64, device=device)


def _lib():
    lib = load()
    if not getattr(lib, "_cnn_ready", False):
        vp, i32, i64, f32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
        lib.dp_gemm_bf16.argtypes = [i32, i32, i32, i32, i32, vp, i32, vp, i32, vp, i32, i32, vp]
        lib.dp_gemm_bf16_ws_bytes.argtypes = [i32, i32, i32]
        lib.dp_gemm_bf16_ws_bytes.restype = sz
        lib.dp_gemm_bf16_ws.argtypes = [i32, i32, i32, i32, i32, vp, i32, vp, i32, vp, i32, i32, vp,
                                        sz, vp]
        lib.dp_gemm_bias_act_bf16.argtypes = [i32, i32, i32, vp, i32, vp, i32, vp, i32, i32, vp, i32, vp]
        lib.dp_im2col3x3_bf16.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp]
        lib.dp_im2col3x3_ld_bf16.argtypes = [i32, i32, i32, i32, i32, vp, vp, i32, i32, vp]
        lib.dp_col2im3x3.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp]
        lib.dp_col2im3x3_act_bf16.argtypes = [i32, i32, i32, i32, i32, vp, vp, i32, vp, vp]
        lib.dp_bias_act_bf16.argtypes = [i64, i32, vp, vp, i32, vp, vp]
        lib.dp_act_bwd_bf16.argtypes = [i64, vp, vp, i32, vp, vp]
        lib.dp_colsum_bf16.argtypes = [i32, i32, vp, vp, vp]
        lib.dp_adam_f32.argtypes = [i64, vp, vp, vp, vp, vp, f32, f32, f32, f32, f32, f32, vp]
        lib.dp_conv3x3_fwd_bf16.argtypes = [i32] * 6 + [vp, vp, i32, vp, i32, i32, vp, vp]
        lib.dp_conv3x3_wgrad_ws_bytes.argtypes = [i32] * 7
        lib.dp_conv3x3_wgrad_ws_bytes.restype = sz
        lib.dp_conv3x3_wgrad_bf16.argtypes = [i32] * 6 + [vp, vp, i32, i32, vp, vp, sz, vp]
        lib.dp_conv3x3_dgrad_act_bf16.argtypes = [i32] * 6 + [vp, vp, i32, vp, i32, vp, vp]
        for f in ("dp_gemm_bf16", "dp_gemm_bf16_ws", "dp_gemm_bias_act_bf16", "dp_im2col3x3_bf16",
                  "dp_im2col3x3_ld_bf16", "dp_col2im3x3", "dp_col2im3x3_act_bf16",
                  "dp_bias_act_bf16", "dp_act_bwd_bf16", "dp_colsum_bf16", "dp_adam_f32",
                  "dp_conv3x3_fwd_bf16", "dp_conv3x3_wgrad_bf16", "dp_conv3x3_dgrad_act_bf16"):
            getattr(lib, f).restype = C.c_int
        lib._cnn_ready = True
    return lib


def _p(t):
    return C.c_void_p(t.data_ptr())


def _ld(t):
    """Row stride of a 2-D tensor whose rows are contiguous."""
    assert t.dim() == 2 and (t.stride(1) == 1 or t.shape[1] == 1)
    return t.stride(0)


_WS = {}


def _workspace(device, nbytes):
    """Split-K workspace, one per device, grown on demand (calls on one
    stream use it in turn)."""
    ws = _WS.get(device)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=device)
        _WS[device] = ws
    return ws


def gemm(a, b, ta=False, tb=False, out=None, accumulate=False):
    """FP32 out = op(a) @ op(b) with BF16 operands (2-D, rows contiguous;
    split-K partials in a workspace, so the result is repeatable)."""
    M, K = (a.shape[1], a.shape[0]) if ta else (a.shape[0], a.shape[1])
    N = b.shape[0] if tb else b.shape[1]
    assert a.dtype == torch.bfloat16 and b.dtype == torch.bfloat16
    assert (b.shape[1] if tb else b.shape[0]) == K
    if out is None:
        out = torch.empty((M, N), dtype=torch.float32, device=a.device)
    lib = _lib()
    need = lib.dp_gemm_bf16_ws_bytes(M, N, K)
    ws = _workspace(a.device, need) if need else None
    rc = lib.dp_gemm_bf16_ws(int(ta), int(tb), M, N, K, _p(a), _ld(a), _p(b), _ld(b), _p(out),
                             _ld(out), int(accumulate), _p(ws) if ws is not None else None,
                             ws.numel() if ws is not None else 0, _stream(None))
    _check(rc, "dp_gemm_bf16_ws")
    return out


def gemm_bias_act(a, b, K, bias, relu=True):
    """BF16 act(a[:, :K] @ b[:, :K]^T + bias) with a [M][>=K], b [N][>=K] BF16 and
    bias a 1-D FP32 view of N values (any stride)."""
    M, N = a.shape[0], b.shape[0]
    y = torch.empty((M, N), dtype=torch.bfloat16, device=a.device)
    _check(_lib().dp_gemm_bias_act_bf16(M, N, K, _p(a), _ld(a), _p(b), _ld(b), _p(bias),
                                        bias.stride(0), int(relu), _p(y), N, _stream(None)),
           "dp_gemm_bias_act_bf16")
    return y


def im2col(x, stride, ld=None, ones=False):
    """col [N Ho Wo][ld] BF16: the 9 Ci window values, then (ones) a 1 and zeros."""
    x = x.contiguous()
    N, H, W, Ci = x.shape
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    ld = 9 * Ci if ld is None else ld
    col = torch.empty((N * Ho * Wo, ld), dtype=torch.bfloat16, device=x.device)
    if ld == 9 * Ci and not ones:
        rc = _lib().dp_im2col3x3_bf16(N, H, W, Ci, stride, _p(x), _p(col), _stream(None))
    else:
        rc = _lib().dp_im2col3x3_ld_bf16(N, H, W, Ci, stride, _p(x), _p(col), ld, int(ones),
                                         _stream(None))
    _check(rc, "dp_im2col3x3_bf16")
    return col, Ho, Wo


def col2im(dcol, shape, stride):
    dcol = dcol.contiguous()
    N, H, W, Ci = shape
    dx = torch.empty(shape, dtype=torch.float32, device=dcol.device)
    _check(_lib().dp_col2im3x3(N, H, W, Ci, stride, _p(dcol), _p(dx), _stream(None)),
           "dp_col2im3x3")
    return dx


def col2im_act(dcol, shape, stride, y, relu=True):
    """BF16 dz = col2im(dcol) * (y > 0) for the layer below's BF16 output y."""
    N, H, W, Ci = shape
    dcol, y = dcol.contiguous(), y.contiguous()
    dz = torch.empty(shape, dtype=torch.bfloat16, device=dcol.device)
    _check(_lib().dp_col2im3x3_act_bf16(N, H, W, Ci, stride, _p(dcol), _p(y), int(relu), _p(dz),
                                        _stream(None)), "dp_col2im3x3_act_bf16")
    return dz


def conv_fwd(x, w, stride, bias, relu=True):
    """Implicit-GEMM convolution: BF16 y [N][Ho][Wo][Co] = act(conv3x3(x) +
    bias) for x [N][H][W][Ci] BF16 (Ci a multiple of 8) and weight rows w
    [Co][>= 9 Ci] BF16 ((ky, kx, ci) order); bias a 1-D FP32 view (any stride)."""
    x = x.contiguous()
    N, H, W, Ci = x.shape
    Co = w.shape[0]
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    y = torch.empty((N, Ho, Wo, Co), dtype=torch.bfloat16, device=x.device)
    _check(_lib().dp_conv3x3_fwd_bf16(N, H, W, Ci, Co, stride, _p(x), _p(w), _ld(w), _p(bias),
                                      bias.stride(0), int(relu), _p(y), _stream(None)),
           "dp_conv3x3_fwd_bf16")
    return y


def conv_wgrad(x, dz, stride, out, ones=True):
    """FP32 out [Co][ld] = dz^T . im2col(x) without the im2col matrix (column
    9 Ci: the bias gradient if ones; columns after it zero)."""
    x, dz = x.contiguous(), dz.contiguous()
    N, H, W, Ci = x.shape
    Co, ld = out.shape
    assert out.stride(1) == 1 and out.stride(0) == ld
    lib = _lib()
    need = lib.dp_conv3x3_wgrad_ws_bytes(N, H, W, Ci, Co, stride, ld)
    ws = _workspace(x.device, need) if need else None
    rc = lib.dp_conv3x3_wgrad_bf16(N, H, W, Ci, Co, stride, _p(x), _p(dz), ld, int(ones), _p(out),
                                   _p(ws) if ws is not None else None,
                                   ws.numel() if ws is not None else 0, _stream(None))
    _check(rc, "dp_conv3x3_wgrad_bf16")
    return out


def conv_dgrad_act(dz, w, shape, stride, y=None, relu=True):
    """BF16 input gradient of a 3x3 convolution for dz [N][Ho][Wo][Co], weight
    rows w [Co][>= 9 Ci], times (y > 0) for the layer below's output y if
    relu: computed per parity class of input pixels, no col2im."""
    dz = dz.contiguous()
    N, H, W, Ci = shape
    Co = w.shape[0]
    out = torch.empty(shape, dtype=torch.bfloat16, device=dz.device)
    yp = _p(y.contiguous()) if (relu and y is not None) else None
    _check(_lib().dp_conv3x3_dgrad_act_bf16(N, H, W, Ci, Co, stride, _p(dz), _p(w), _ld(w), yp,
                                            int(relu and y is not None), _p(out), _stream(None)),
           "dp_conv3x3_dgrad_act_bf16")
    return out


def bias_act(z, bias, relu=True):
    z, bias = z.contiguous(), bias.contiguous()
    y = torch.empty(z.shape, dtype=torch.bfloat16, device=z.device)
    _check(_lib().dp_bias_act_bf16(z.shape[0], z.shape[1], _p(z), _p(bias), int(relu), _p(y),
                                   _stream(None)), "dp_bias_act_bf16")
    return y


def act_bwd(dy, y, relu=True):
    dy, y = dy.contiguous(), y.contiguous()
    dz = torch.empty(dy.shape, dtype=torch.bfloat16, device=dy.device)
    _check(_lib().dp_act_bwd_bf16(dy.numel(), _p(dy), _p(y), int(relu), _p(dz), _stream(None)),
           "dp_act_bwd_bf16")
    return dz


def colsum(dz):
    dz = dz.contiguous()
    db = torch.empty(dz.shape[1], dtype=torch.float32, device=dz.device)
    _check(_lib().dp_colsum_bf16(dz.shape[0], dz.shape[1], _p(dz), _p(db), _stream(None)),
           "dp_colsum_bf16")
    return db


def adam(p, g, m, v, pb, lr, betas, eps, c1, c2):
    """One fused Adam step over flat FP32 buffers; pb receives p in BF16."""
    _check(_lib().dp_adam_f32(p.numel(), _p(p), _p(g), _p(m), _p(v), _p(pb), lr, betas[0], betas[1],
                              eps, c1, c2, _stream(None)), "dp_adam_f32")


def _row_len(ci):
    """Row length of a layer's parameter block: 9 Ci weights, the bias, zero
    padding to a multiple of 8 (16-byte rows for the BF16 products)."""
    return (9 * ci + 1 + 7) // 8 * 8


class ProposalNet:
    """Strided CNN + linear head; parameters in FP32, operands in BF16.

    All parameters live in one flat FP32 buffer P (gradients in G of the same
    layout, a BF16 copy in Pb): per conv layer a [Co][row] block whose row
    holds the 9 Ci weights, the bias and zero padding, then the head's
    weights [6][F] and bias [6].  Layers with a multiple of 8 input channels
    run as implicit GEMMs (operand tiles gathered from the activations, no
    im2col matrix; the input gradient per parity class of input pixels, no
    col2im), the 2-channel input layer through an explicit im2col.  The
    forward product reads the BF16 weights with the FP32 bias in its
    epilogue; the weight-gradient product (with an implicit or explicit ones
    column) writes the layer's weight and bias gradients straight into its
    block of G; Adam is one launch over P."""

    def __init__(self, size=256, in_ch=2, channels=CHANNELS, device="cuda:0", seed=0):
        self.size = size
        self.device = torch.device(device)
        g = torch.Generator(device="cpu").manual_seed(seed)
        shapes, ci, hw = [], in_ch, size
        for co in channels:
            shapes.append((ci, co, _row_len(ci)))
            ci, hw = co, (hw - 1) // 2 + 1
        self.feat_hw, self.feat_c = hw, ci
        F = hw * hw * ci
        n = sum(co * r for _, co, r in shapes) + 6 * F + 6
        self.P = torch.zeros(n, device=self.device)
        self.G = torch.zeros(n, device=self.device)
        self.Pb = torch.zeros(n, dtype=torch.bfloat16, device=self.device)
        self.blocks, self.gblocks, self.bblocks, self.convs = [], [], [], []
        off = 0
        for ci, co, r in shapes:
            blk = self.P[off:off + co * r].view(co, r)
            std = math.sqrt(2.0 / (9 * ci))
            blk[:, :9 * ci] = (torch.randn(co, 9 * ci, generator=g) * std).to(self.device)
            self.blocks.append(blk)
            self.gblocks.append(self.G[off:off + co * r].view(co, r))
            self.bblocks.append(self.Pb[off:off + co * r].view(co, r))
            self.convs.append([blk[:, :9 * ci], blk[:, 9 * ci], 2])
            off += co * r
        self.Wfc = self.P[off:off + 6 * F].view(6, F)
        self.Wfc.copy_((torch.randn(6, F, generator=g) * math.sqrt(1.0 / F)).to(self.device))
        self.gWfc = self.G[off:off + 6 * F].view(6, F)
        self.Wfc_b = self.Pb[off:off + 6 * F].view(6, F)
        off += 6 * F
        self.bfc = self.P[off:off + 6]
        self.gbfc = self.G[off:off + 6]
        self.sync_bf16()
        self._adam = None

    def sync_bf16(self):
        """Refresh the BF16 copy after the FP32 parameters were changed."""
        self.Pb.copy_(self.P)

    def params(self):
        ps = []
        for W, b, _ in self.convs:
            ps += [W, b]
        return ps + [self.Wfc, self.bfc]

    def forward(self, x, keep=False):
        """x: [N][H][W][2] BF16 (NHWC).  Returns FP32 [N][6] (and the cache)."""
        cache = []
        h = x.contiguous()
        for li, (W, b, s) in enumerate(self.convs):
            K = W.shape[1]
            if h.shape[3] % 8 == 0:
                # implicit GEMM: the products gather their operand tiles from h
                y = conv_fwd(h, self.bblocks[li], s, b, relu=True)
                col = None
            else:
                # few input channels (the 2-channel input layer): im2col rows
                # padded to the parameter row, with a ones column for the
                # bias gradient
                col, Ho, Wo = im2col(h, s, ld=self.blocks[li].shape[1], ones=keep)
                y = gemm_bias_act(col, self.bblocks[li], K, b, relu=True)
                y = y.view(h.shape[0], Ho, Wo, W.shape[0])
            if keep:
                cache.append((h, col, y, s))
            h = y
        feat = h.reshape(h.shape[0], -1)
        out = gemm(feat, self.Wfc_b, tb=True) + self.bfc
        return (out, (cache, feat)) if keep else out

    def backward(self, cache, dout):
        """Gradients of sum(dout * forward(x)) for every parameter (FP32),
        written into G; returns views of it: per layer (dW, db), and the head's."""
        convs_cache, feat = cache
        d = dout.to(torch.bfloat16).contiguous()
        gemm(d, feat, ta=True, out=self.gWfc)
        self.gbfc.copy_(d.float().sum(0))
        dh = gemm(d, self.Wfc_b)                                   # [N][F] FP32
        _, _, y_top, _ = convs_cache[-1]
        dz = act_bwd(dh.reshape(y_top.shape).contiguous(), y_top, relu=True)
        grads = [None] * len(self.convs)
        for li in range(len(self.convs) - 1, -1, -1):
            W, b, s = self.convs[li]
            x_in, col, y, _ = convs_cache[li]
            dz = dz.reshape(-1, W.shape[0])
            K = W.shape[1]
            # [Co][row]: dW | db | 0
            if col is None:
                conv_wgrad(x_in, dz, s, out=self.gblocks[li], ones=True)
            else:
                gemm(dz, col, ta=True, out=self.gblocks[li])
            if li > 0:
                y_below = convs_cache[li - 1][2]
                if col is None:
                    dz = conv_dgrad_act(dz, self.bblocks[li], tuple(x_in.shape), s, y_below)
                else:
                    dcol = gemm(dz, self.bblocks[li][:, :K])         # [M][9 Ci]
                    dz = col2im_act(dcol, tuple(x_in.shape), s, y_below, relu=True)
            grads[li] = (self.gblocks[li][:, :K], self.gblocks[li][:, K])
        return grads, (self.gWfc, self.gbfc)

    def adam_step(self, grads, head, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, wd=0.0):
        """One Adam step on every parameter; `grads` and `head` must be the
        views of G that backward() returned (the step reads G as a whole)."""
        assert head[0].data_ptr() == self.gWfc.data_ptr()
        if self._adam is None:
            self._adam = (torch.zeros_like(self.P), torch.zeros_like(self.P))
            self._t = 0
        self._t += 1
        if wd:
            self.G.add_(self.P, alpha=wd)
        m, v = self._adam
        adam(self.P, self.G, m, v, self.Pb, lr, betas, eps, 1 - betas[0] ** self._t,
             1 - betas[1] ** self._t)

    def tensors(self) -> dict:
        """Flat name -> FP32 CPU tensor map (safetensors layout)."""
        out = {}
        for i, (W, b, s) in enumerate(self.convs):
            out[f"conv{i}.weight"] = W.detach().cpu().contiguous()
            out[f"conv{i}.bias"] = b.detach().cpu().contiguous()
        out["fc.weight"] = self.Wfc.detach().cpu().contiguous()
        out["fc.bias"] = self.bfc.detach().cpu().contiguous()
        return out

    def save(self, path: str, meta: dict | None = None):
        from safetensors.torch import save_file
        info = {"size": str(self.size), "channels": ",".join(str(W.shape[0]) for W, _, _ in self.convs)}
        info.update({k: str(v) for k, v in (meta or {}).items()})
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        save_file(self.tensors(), path, metadata=info)

    @classmethod
    def load(cls, path: str, device="cuda:0") -> "ProposalNet":
        from safetensors import safe_open
        with safe_open(path, framework="pt") as fh:
            meta = fh.metadata()
            t = {k: fh.get_tensor(k) for k in fh.keys()}
        chans = tuple(int(c) for c in meta["channels"].split(","))
        net = cls(size=int(meta["size"]), channels=chans, device=device)
        for i, conv in enumerate(net.convs):
            conv[0].copy_(t[f"conv{i}.weight"].to(net.device))
            conv[1].copy_(t[f"conv{i}.bias"].to(net.device))
        net.Wfc.copy_(t["fc.weight"].to(net.device))
        net.bfc.copy_(t["fc.bias"].to(net.device))
        net.sync_bf16()
        net.meta = meta
        return net

    def predict(self, x, batch=256) -> torch.Tensor:
        """Pose offsets [N][6] (FP64, mm and rad) for NHWC BF16 pair images."""
        outs = [self.forward(x[i:i + batch]) for i in range(0, x.shape[0], batch)]
        return torch.cat(outs).to(torch.float64) * label_scale(x.device)


def pair_input(ref, target, size):
    """Stack reference and target DRRs ([N][nv][nu] FP32) into the network's
    NHWC BF16 input at size x size (area resampling), each image normalised
    by the reference's maximum."""
    x = torch.stack([ref, target], dim=1)
    if x.shape[-1] != size or x.shape[-2] != size:
        x = torch.nn.functional.adaptive_avg_pool2d(x, (size, size))
    scale = x[:, :1].amax(dim=(1, 2, 3), keepdim=True).clamp_min(1e-6)
    return (x / scale).permute(0, 2, 3, 1).contiguous().to(torch.bfloat16)


# ---------------------------------------------------------------------------
# Training set: DRR pairs rendered by the library's own forward projector
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class DRRSet:
    """Reference DRRs (identity pose) per phantom and target DRRs at random
    pose offsets, both divided by the reference's maximum and stored BF16."""
    ref: torch.Tensor      # [P][nv][nu] bf16
    tgt: torch.Tensor      # [S][nv][nu] bf16
    pid: torch.Tensor      # [S] int64 phantom of each target
    poses: torch.Tensor    # [S][6] f64 pose offsets (mm, rad)

    def __len__(self):
        return self.tgt.shape[0]

    def inputs(self, idx) -> torch.Tensor:
        return torch.stack([self.ref[self.pid[idx]], self.tgt[idx]], dim=-1).contiguous()

    def labels(self, idx) -> torch.Tensor:
        return (self.poses[idx] / label_scale(self.poses.device)).to(torch.float32)


def phantom(geom, rng, device):
    """One training/evaluation phantom: 10-40 random ellipsoids, half of them
    inside a high-attenuation shell, sigma = 1 voxel smoothing."""
    import synth
    n_ell = int(rng.integers(10, 41))
    shell = bool(rng.uniform() < 0.5)
    return synth.ellipsoid_phantom_torch(geom.nx, geom.vx, n_ell, rng, device, shell=shell)


def render_set(geom, n_phantoms, per_phantom, salt, device="cuda:0", log=None) -> DRRSet:
    """Render per_phantom targets at uniform random offsets (+-30 mm, +-20 deg)
    and one identity reference for each of n_phantoms phantoms, gantry angle 0."""
    import synth
    dev = torch.device(device)
    S = n_phantoms * per_phantom
    ref = torch.empty((n_phantoms, geom.nv, geom.nu), dtype=torch.bfloat16, device=dev)
    tgt = torch.empty((S, geom.nv, geom.nu), dtype=torch.bfloat16, device=dev)
    poses = torch.empty((S, 6), dtype=torch.float64, device=dev)
    pid = torch.arange(n_phantoms, device=dev).repeat_interleave(per_phantom)
    zero_angle = torch.zeros(1, dtype=torch.float64, device=dev)
    angles = torch.zeros(per_phantom, dtype=torch.float64, device=dev)
    ident = torch.zeros((1, 6), dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    for i in range(n_phantoms):
        rng = synth.rng_for(4, salt * 1_000_003 + i)
        vol = phantom(geom, rng, dev)
        th = torch.tensor(synth.random_poses(per_phantom, T_RANGE_MM, R_RANGE_DEG, rng),
                          dtype=torch.float64, device=dev)
        r = _project_fwd(geom, zero_angle, ident, vol)[0]
        scale = 1.0 / r.max().clamp_min(1e-6)
        ref[i] = (r * scale).to(torch.bfloat16)
        sl = slice(i * per_phantom, (i + 1) * per_phantom)
        tgt[sl] = (_project_fwd(geom, angles, th, vol) * scale).to(torch.bfloat16)
        poses[sl] = th
        if log and ((i + 1) % max(1, n_phantoms // 10) == 0 or i + 1 == n_phantoms):
            torch.cuda.synchronize(dev)
            log(f"rendered {i + 1}/{n_phantoms} phantoms ({(i + 1) * per_phantom} DRRs) "
                f"in {time.perf_counter() - t0:.1f} s")
    return DRRSet(ref, tgt, pid, poses)


def pose_mae(est, truth):
    """Mean absolute error per pose parameter: tx, ty, tz (mm), gx, gy, gz (deg)."""
    d = (est - truth).abs()
    d[:, 3:] = torch.rad2deg(d[:, 3:])
    return [round(float(x), 6) for x in d.mean(dim=0)]


def pose_error_stats(pred, truth):
    """Median and 90th-percentile |error| per component (mm, deg)."""
    d = (pred - truth).abs()
    d[:, 3:] = torch.rad2deg(d[:, 3:])
    return d.median(dim=0).values, d.quantile(0.9, dim=0)


def train(net, data: DRRSet, val: DRRSet | None = None, epochs=8, batch=256, lr=1e-3,
          lr_min=2e-5, seed=0, log=print):
    """Minimise the mean squared error of the normalised pose offset with Adam
    (cosine learning-rate schedule); every layer's forward and backward runs
    on the library's BF16 MFMA kernels."""
    dev = data.tgt.device
    gen = torch.Generator(device=dev).manual_seed(seed)
    steps_per_epoch = len(data) // batch
    total = epochs * steps_per_epoch
    step = 0
    t0 = time.perf_counter()
    history = []
    for ep in range(epochs):
        perm = torch.randperm(len(data), generator=gen, device=dev)
        acc, cnt = torch.zeros((), device=dev), 0
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            x, y = data.inputs(idx), data.labels(idx)
            out, cache = net.forward(x, keep=True)
            d = out - y
            acc += (d * d).mean().detach()
            cnt += 1
            grads, head = net.backward(cache, (2.0 / d.numel()) * d)
            a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / max(1, total)))
            net.adam_step(grads, head, lr=a)
            step += 1
        msg = f"epoch {ep + 1}/{epochs}: train mse {float(acc) / max(cnt, 1):.5f}"
        if val is not None:
            pred = net.predict(val.inputs(torch.arange(len(val), device=dev)))
            med, p90 = pose_error_stats(pred, val.poses)
            msg += (f"; val median |err| t {med[:3].cpu().numpy().round(2)} mm, "
                    f"r {med[3:].cpu().numpy().round(2)} deg; p90 t {p90[:3].cpu().numpy().round(2)}"
                    f" r {p90[3:].cpu().numpy().round(2)}")
        torch.cuda.synchronize(dev)
        msg += f" ({time.perf_counter() - t0:.1f} s)"
        history.append(msg)
        log(msg)
    return history


# ---------------------------------------------------------------------------
# Registration with the learned proposal
# ---------------------------------------------------------------------------

def _refine(method):
    from .registration import register_bfgs, register_lm
    return {"lm": register_lm, "bfgs": register_bfgs}[method]


def transmission_noise_ssd(targets, photons, scale):
    """Expected SSD that Poisson counting noise leaves at the true pose, per
    target: with counts of mean photons * exp(-scale * l), the log-transformed
    measurement has variance exp(scale * l) / (photons * scale^2) to first
    order; the noisy target stands in for l, so no knowledge of the truth
    enters.  targets: [B][nv][nu]; returns FP64 [B]."""
    y = targets.to(torch.float64)
    return (torch.exp(scale * y) / (photons * scale * scale)).reshape(y.shape[0], -1).sum(1)


def register_learned(net, geom, vol, angles, targets, ref, fallback=True, rel_tol=1e-6,
                     method="lm", noise_ssd=None, **kw):
    """Propose theta0 with the network from (reference DRR, target), refine
    with the analytic-gradient registration (`method`), and fall back to the
    plain registration from the identity for every registration whose refined
    loss stays above rel_tol * |target|^2, plus 1.1 x noise_ssd (the SSD the
    target's noise leaves at the true pose, [B], for noisy targets), keeping
    the lower loss.

    The network was trained at gantry angle 0, so `angles` must be zero;
    `ref` is the [nv][nu] DRR of `vol` at the identity pose.
    Returns (RegistrationResult, theta0, number of fallbacks).
    """
    from .registration import RegistrationResult
    refine = _refine(method)
    if bool((angles != 0).any()):
        raise ValueError("the proposal network is trained for gantry angle 0")
    t0 = time.perf_counter()
    B = targets.shape[0]
    x = pair_input(ref.expand(B, -1, -1), targets, net.size)
    theta0 = net.predict(x)
    res = refine(geom, vol, angles, targets, theta0, **kw)
    poses, its, conv, fl = res.poses.clone(), res.iterations.clone(), res.converged.clone(), \
        res.final_loss.clone()
    launches = res.launches
    n_fb = 0
    if fallback:
        energy = (targets.to(torch.float64) ** 2).reshape(B, -1).sum(1)
        limit = rel_tol * energy
        if noise_ssd is not None:
            limit = limit + 1.1 * noise_ssd.to(device=fl.device, dtype=torch.float64)
        bad = torch.nonzero(fl > limit).flatten()
        n_fb = int(bad.numel())
        if n_fb:
            r2 = refine(geom, vol, angles[bad], targets[bad], torch.zeros_like(theta0[bad]), **kw)
            better = r2.final_loss < fl[bad]
            sel = bad[better]
            poses[sel] = r2.poses[better]
            fl[sel] = r2.final_loss[better]
            conv[sel] = r2.converged[better]
            its[bad] += r2.iterations
            launches += r2.launches
    torch.cuda.synchronize(targets.device)
    out = RegistrationResult(poses=poses, iterations=its, converged=conv, final_loss=fl,
                             seconds=time.perf_counter() - t0, launches=launches)
    return out, theta0, n_fb


def evaluate(net, geom, n_phantoms=8, per_phantom=16, salt=3, device="cuda:0", log=None,
             method="lm", photons=None, **kw):
    """Plain (identity start) versus learned-proposal registration on unseen
    phantoms with offsets drawn like the training set.  Returns success
    rates at 0.1 mm / 0.1 deg, registrations per second and error stats
    (the proposal's median / 90th-percentile error and each pipeline's mean
    absolute error per pose parameter, mm and deg).  `method` is the
    refinement ("lm" Levenberg-Marquardt or "bfgs"), the same for both
    pipelines.  photons: if given, the targets carry Poisson noise of a
    transmission measurement with that many unattenuated photons per pixel,
    the attenuation scaled so that the largest line integral is 5."""
    import synth
    from .registration import success
    refine = _refine(method)
    dev = torch.device(device)
    stats = {"plain_ok": 0, "learned_ok": 0, "n": 0, "plain_s": 0.0, "learned_s": 0.0,
             "fallbacks": 0, "plain_iters": 0, "learned_iters": 0}
    prop_err, truths, plain_est, learned_est = [], [], [], []
    gen = torch.Generator(device=dev).manual_seed(salt)
    for i in range(n_phantoms):
        rng = synth.rng_for(4, salt * 1_000_003 + i)
        vol = phantom(geom, rng, dev)
        truth = torch.tensor(synth.random_poses(per_phantom, T_RANGE_MM, R_RANGE_DEG, rng),
                             dtype=torch.float64, device=dev)
        angles = torch.zeros(per_phantom, dtype=torch.float64, device=dev)
        targets = _project_fwd(geom, angles, truth, vol)
        noise_ssd = None
        if photons:
            # attenuation scaled so the largest line integral is 5 (head-like counts)
            scale = 5.0 / float(targets.max())
            targets = synth.poisson_log_noise(targets, photons, gen, scale)
            noise_ssd = transmission_noise_ssd(targets, photons, scale)
        ref = _project_fwd(geom, angles[:1], torch.zeros_like(truth[:1]), vol)[0]
        torch.cuda.synchronize(dev)
        if i == 0:  # warm-up (library load, workspace, first launches) outside the timing
            refine(geom, vol, angles[:2], targets[:2], torch.zeros_like(truth[:2]), iters=2)
            net.predict(pair_input(ref.expand(2, -1, -1), targets[:2], net.size))
        plain = refine(geom, vol, angles, targets, torch.zeros_like(truth), **kw)
        learned, theta0, nfb = register_learned(net, geom, vol, angles, targets, ref, method=method,
                                                noise_ssd=noise_ssd, **kw)
        stats["plain_ok"] += int(success(plain.poses, truth).sum())
        stats["learned_ok"] += int(success(learned.poses, truth).sum())
        stats["n"] += per_phantom
        stats["plain_s"] += plain.seconds
        stats["learned_s"] += learned.seconds
        stats["fallbacks"] += nfb
        stats["plain_iters"] += int(plain.iterations.sum())
        stats["learned_iters"] += int(learned.iterations.sum())
        prop_err.append(theta0)
        truths.append(truth)
        plain_est.append(plain.poses)
        learned_est.append(learned.poses)
        if log:
            log(f"phantom {i + 1}/{n_phantoms}: plain {stats['plain_ok']}/{stats['n']} "
                f"learned {stats['learned_ok']}/{stats['n']} fallbacks {stats['fallbacks']}")
    truth_all = torch.cat(truths)
    med, p90 = pose_error_stats(torch.cat(prop_err), truth_all)
    n = stats["n"]
    return {
        "registrations": n,
        "plain_success": stats["plain_ok"] / n,
        "learned_success": stats["learned_ok"] / n,
        "plain_registrations_per_s": n / stats["plain_s"],
        "learned_registrations_per_s": n / stats["learned_s"],
        "plain_successful_per_s": stats["plain_ok"] / stats["plain_s"],
        "learned_successful_per_s": stats["learned_ok"] / stats["learned_s"],
        "plain_mean_iterations": stats["plain_iters"] / n,
        "learned_mean_iterations": stats["learned_iters"] / n,
        "fallbacks": stats["fallbacks"],
        "proposal_median_err": med.cpu().tolist(),
        "proposal_p90_err": p90.cpu().tolist(),
        "plain_mae": pose_mae(torch.cat(plain_est), truth_all),
        "learned_mae": pose_mae(torch.cat(learned_est), truth_all),
        "photons": photons,
    }


def _main(argv=None):
    ap = argparse.ArgumentParser(description="Render the DRR training set with the forward "
                                 "projector and train the pose-proposal network on the GPU.")
    ap.add_argument("--phantoms", type=int, default=2000)
    ap.add_argument("--per-phantom", type=int, default=100)
    ap.add_argument("--val-phantoms", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-phantoms", type=int, default=4)
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args(argv)
    import synth

    def log(m):
        print(m, flush=True)

    geom = synth.geom_c5()
    data = render_set(geom, a.phantoms, a.per_phantom, salt=1, log=log)
    val = render_set(geom, a.val_phantoms, a.per_phantom, salt=2, log=log)
    net = ProposalNet(size=geom.nu, seed=0)
    hist = train(net, data, val, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
    net.save(a.out, {"phantoms": a.phantoms, "per_phantom": a.per_phantom, "epochs": a.epochs,
                     "batch": a.batch, "lr": a.lr, "final": hist[-1]})
    log(f"saved {a.out}")
    del data
    if a.eval_phantoms:
        res = evaluate(net, geom, n_phantoms=a.eval_phantoms, per_phantom=16, log=log)
        log(json.dumps(res))


if __name__ == "__main__":
    sys.exit(_main())
