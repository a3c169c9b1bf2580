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

import ctypes as C
import math

import torch

from . import _check, _stream, load

CHANNELS = (32, 64, 128, 256, 256, 256)


def _lib():
    lib = load()
    if not getattr(lib, "_cnn_ready", False):
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        lib.dp_gemm_bf16.argtypes = [i32, i32, i32, i32, i32, vp, i32, vp, i32, vp, i32, i32, vp]
        lib.dp_im2col3x3_bf16.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp]
        lib.dp_col2im3x3.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp]
        lib.dp_bias_act_bf16.argtypes = [i64, i32, vp, vp, i32, vp, vp]
        lib.dp_act_bwd_bf16.argtypes = [i64, vp, vp, i32, vp, vp]
        lib.dp_colsum_bf16.argtypes = [i32, i32, vp, vp, vp]
        for f in ("dp_gemm_bf16", "dp_im2col3x3_bf16", "dp_col2im3x3", "dp_bias_act_bf16",
                  "dp_act_bwd_bf16", "dp_colsum_bf16"):
            getattr(lib, f).restype = C.c_int
        lib._cnn_ready = True
    return lib


def _p(t):
    return C.c_void_p(t.data_ptr())


def gemm(a, b, ta=False, tb=False, out=None, accumulate=False):
    """FP32 out = op(a) @ op(b) with BF16 operands (2-D, contiguous)."""
    M, K = (a.shape[1], a.shape[0]) if ta else (a.shape[0], a.shape[1])
    N = b.shape[0] if tb else b.shape[1]
    assert a.dtype == torch.bfloat16 and b.dtype == torch.bfloat16
    assert (b.shape[1] if tb else b.shape[0]) == K
    if out is None:
        out = torch.empty((M, N), dtype=torch.float32, device=a.device)
    rc = _lib().dp_gemm_bf16(int(ta), int(tb), M, N, K, _p(a), a.shape[1], _p(b), b.shape[1],
                             _p(out), out.shape[1], int(accumulate), _stream(None))
    _check(rc, "dp_gemm_bf16")
    return out


def im2col(x, stride):
    N, H, W, Ci = x.shape
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    col = torch.empty((N * Ho * Wo, 9 * Ci), dtype=torch.bfloat16, device=x.device)
    _check(_lib().dp_im2col3x3_bf16(N, H, W, Ci, stride, _p(x), _p(col), _stream(None)),
           "dp_im2col3x3_bf16")
    return col, Ho, Wo


def col2im(dcol, shape, stride):
    N, H, W, Ci = shape
    dx = torch.empty(shape, dtype=torch.float32, device=dcol.device)
    _check(_lib().dp_col2im3x3(N, H, W, Ci, stride, _p(dcol), _p(dx), _stream(None)),
           "dp_col2im3x3")
    return dx


def bias_act(z, bias, relu=True):
    y = torch.empty(z.shape, dtype=torch.bfloat16, device=z.device)
    _check(_lib().dp_bias_act_bf16(z.shape[0], z.shape[1], _p(z), _p(bias), int(relu), _p(y),
                                   _stream(None)), "dp_bias_act_bf16")
    return y


def act_bwd(dy, y, relu=True):
    dz = torch.empty(dy.shape, dtype=torch.bfloat16, device=dy.device)
    _check(_lib().dp_act_bwd_bf16(dy.numel(), _p(dy), _p(y), int(relu), _p(dz), _stream(None)),
           "dp_act_bwd_bf16")
    return dz


def colsum(dz):
    db = torch.empty(dz.shape[1], dtype=torch.float32, device=dz.device)
    _check(_lib().dp_colsum_bf16(dz.shape[0], dz.shape[1], _p(dz), _p(db), _stream(None)),
           "dp_colsum_bf16")
    return db


class ProposalNet:
    """Strided CNN + linear head; parameters in FP32, operands in BF16."""

    def __init__(self, size=256, in_ch=2, channels=CHANNELS, device="cuda:0", seed=0):
        self.size = size
        self.device = torch.device(device)
        g = torch.Generator(device="cpu").manual_seed(seed)
        self.convs = []   # (W [Co][9 Ci], b [Co], stride)
        ci, hw = in_ch, size
        for co in channels:
            std = math.sqrt(2.0 / (9 * ci))
            W = (torch.randn(co, 9 * ci, generator=g) * std).to(self.device)
            self.convs.append([W, torch.zeros(co, device=self.device), 2])
            ci, hw = co, (hw - 1) // 2 + 1
        self.feat_hw, self.feat_c = hw, ci
        F = hw * hw * ci
        self.Wfc = (torch.randn(6, F, generator=g) * math.sqrt(1.0 / F)).to(self.device)
        self.bfc = torch.zeros(6, device=self.device)
        self._adam = None

    def params(self):
        ps = []
        for W, b, _ in self.convs:
            ps += [W, b]
        return ps + [self.Wfc, self.bfc]

    def forward(self, x, keep=False):
        """x: [N][H][W][2] BF16 (NHWC).  Returns FP32 [N][6] (and the cache)."""
        cache = []
        h = x.contiguous()
        for W, b, s in self.convs:
            col, Ho, Wo = im2col(h, s)
            z = gemm(col, W.to(torch.bfloat16).contiguous(), tb=True)
            y = bias_act(z, b, relu=True)
            if keep:
                cache.append((h.shape, col, y, s))
            h = y.view(h.shape[0], Ho, Wo, W.shape[0])
        feat = h.reshape(h.shape[0], -1)
        out = gemm(feat, self.Wfc.to(torch.bfloat16).contiguous(), tb=True) + self.bfc
        return (out, (cache, feat)) if keep else out

    def backward(self, cache, dout):
        """Gradients of sum(dout * forward(x)) for every parameter (FP32)."""
        convs_cache, feat = cache
        d = dout.to(torch.bfloat16).contiguous()
        dWfc = gemm(d, feat, ta=True)
        dbfc = dout.to(torch.bfloat16).float().sum(0)
        dh = gemm(d, self.Wfc.to(torch.bfloat16).contiguous())   # [N][F] FP32
        grads = [None] * len(self.convs)
        for li in range(len(self.convs) - 1, -1, -1):
            W, b, s = self.convs[li]
            xshape, col, y, _ = convs_cache[li]
            dz = act_bwd(dh.reshape(y.shape).contiguous(), y, relu=True)
            dW = gemm(dz, col, ta=True)                          # [Co][9 Ci]
            db = colsum(dz)
            if li > 0:
                dcol = gemm(dz, W.to(torch.bfloat16).contiguous())  # [M][9 Ci]
                dh = col2im(dcol, xshape, s)
            grads[li] = (dW, db)
        return grads, (dWfc, dbfc)

    def adam_step(self, grads, head, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, wd=0.0):
        flat = []
        for dW, db in grads:
            flat += [dW, db]
        flat += list(head)
        ps = self.params()
        if self._adam is None:
            self._adam = [(torch.zeros_like(p), torch.zeros_like(p)) for p in ps]
            self._t = 0
        self._t += 1
        c1, c2 = 1 - betas[0] ** self._t, 1 - betas[1] ** self._t
        for p, g, (m, v) in zip(ps, flat, self._adam):
            if wd:
                g = g + wd * p
            m.mul_(betas[0]).add_(g, alpha=1 - betas[0])
            v.mul_(betas[1]).addcmul_(g, g, value=1 - betas[1])
            p.sub_(lr * (m / c1) / ((v / c2).sqrt() + eps))

    def state_dict(self):
        return {"convs": [(W.cpu(), b.cpu(), s) for W, b, s in self.convs],
                "Wfc": self.Wfc.cpu(), "bfc": self.bfc.cpu(), "size": self.size}

    def load_state_dict(self, st):
        self.convs = [[W.to(self.device), b.to(self.device), s] for W, b, s in st["convs"]]
        self.Wfc, self.bfc = st["Wfc"].to(self.device), st["bfc"].to(self.device)


def pair_input(ref, target, size):
    """Stack reference and target DRRs ([N][nv][nu] FP32) into the network's
    NHWC BF16 input at size x size (area resampling), each image normalised
    by the reference's maximum."""
    x = torch.stack([ref, target], dim=1)
    if x.shape[-1] != size or x.shape[-2] != size:
        x = torch.nn.functional.adaptive_avg_pool2d(x, (size, size))
    scale = x[:, :1].amax(dim=(1, 2, 3), keepdim=True).clamp_min(1e-6)
    return (x / scale).permute(0, 2, 3, 1).contiguous().to(torch.bfloat16)
