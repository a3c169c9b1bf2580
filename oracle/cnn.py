"""FP64 CPU oracle of the learned-proposal CNN -- TEST INFRASTRUCTURE ONLY.

Plain numpy, written from the definitions (no im2col, no GEMM blocking):
  z[n, yo, xo, co] = b[co] + sum_{ky, kx, ci} W[co, ky, kx, ci] xp[n, s yo + ky, s xo + kx, ci]
with xp the input zero-padded by one pixel (3x3 kernel, stride s), NHWC
layout; ReLU; a fully connected head on the flattened NHWC features; the
mean squared error of the 6 outputs.  Gradients are the adjoints of those
sums.  `bf16` rounds to bfloat16 (round-to-nearest-even), the storage
precision the GPU path uses for operands.
"""
from __future__ import annotations

import numpy as np


def bf16(a) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3_forward(x, W, b, stride):
    """x [N][H][W][Ci], W [Co][3][3][Ci], b [Co] -> z [N][Ho][Wo][Co] (pre-activation)."""
    N, H, Wd, Ci = x.shape
    Co = W.shape[0]
    Ho, Wo = (H - 1) // stride + 1, (Wd - 1) // stride + 1
    xp = np.zeros((N, H + 2, Wd + 2, Ci))
    xp[:, 1:-1, 1:-1, :] = x
    z = np.zeros((N, Ho, Wo, Co)) + b
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :]
            z += np.einsum("nhwc,oc->nhwo", patch, W[:, ky, kx, :])
    return z


def conv3x3_backward(x, W, dz, stride):
    """Gradients (dx, dW, db) of sum(dz * conv3x3_forward(x, W, b, stride))."""
    N, H, Wd, Ci = x.shape
    _, Ho, Wo, Co = dz.shape
    xp = np.zeros((N, H + 2, Wd + 2, Ci))
    xp[:, 1:-1, 1:-1, :] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W, dtype=np.float64)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(ky, ky + stride * (Ho - 1) + 1, stride),
                  slice(kx, kx + stride * (Wo - 1) + 1, stride), slice(None))
            dW[:, ky, kx, :] = np.einsum("nhwo,nhwc->oc", dz, xp[sl])
            dxp[sl] += np.einsum("nhwo,oc->nhwc", dz, W[:, ky, kx, :])
    return dxp[:, 1:-1, 1:-1, :], dW, dz.sum(axis=(0, 1, 2))


def relu(z):
    return np.maximum(z, 0.0)


def network_forward(x, params, round_bf16=True):
    """Conv layers (ReLU) + linear head.  params: list of (W, b, stride) and
    (Wfc [6][F], bfc [6]).  Returns the output [N][6] and the activations."""
    convs, (Wfc, bfc) = params
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    acts = [r(x)]
    h = acts[0]
    for W, b, s in convs:
        h = r(relu(conv3x3_forward(h, r(W), b, s)))
        acts.append(h)
    feat = h.reshape(h.shape[0], -1)
    out = feat @ r(Wfc).T + bfc
    return out, acts


def network_backward(params, acts, dout, round_bf16=True):
    """Gradients of sum(dout * out) with respect to every parameter, with the
    upstream gradients rounded to bf16 where the GPU path stores them."""
    convs, (Wfc, bfc) = params
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    feat = acts[-1].reshape(acts[-1].shape[0], -1)
    d = r(dout)
    dWfc = d.T @ feat
    dbfc = d.sum(0)
    dh = (d @ r(Wfc)).reshape(acts[-1].shape)
    grads = []
    for li in range(len(convs) - 1, -1, -1):
        W, b, s = convs[li]
        y = acts[li + 1]
        dz = r(np.where(y > 0, dh, 0.0))
        dx, dW, db = conv3x3_backward(acts[li], r(W), dz, s)
        grads.append((dW, db))
        dh = dx
    return list(reversed(grads)), (dWfc, dbfc)
