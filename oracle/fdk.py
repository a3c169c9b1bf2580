"""FP64 CPU oracle of the FDK pre-filter and the image-sharpness loss -- TEST
INFRASTRUCTURE ONLY (imported by tests, the smoke check and the bench's CPU
baseline; never by the library).

FDK pre-filter (Feldkamp, Davis and Kress; the filtered back-projection the
paper's motion-compensated reconstruction task builds on, Sec. III-B): the
projections are moved to a virtual detector through the isocentre
(coordinates scaled by SAD/SDD), multiplied by the cosine weight
SAD / sqrt(SAD^2 + u'^2 + v'^2), and every detector row is convolved with the
band-limited (Ram-Lak) ramp kernel sampled at the virtual pixel pitch tau:
    h[0] = 1 / (4 tau^2),  h[k] = 0 for even k != 0,  h[k] = -1 / (pi^2 k^2 tau^2) for odd k,
    q[a] = scale * tau * sum_n p_w[n] h[a - n]
(a row of nu samples is zero outside the detector).  With scale = pi / V for
V views over a full circle, back-projecting q with the FDK distance weight
(SAD/U)^2 gives the FDK reconstruction (Delta beta / 2 = pi / V).

Sharpness (Sec. III-B, motion-compensated reconstruction): negative sum of
squared forward differences of the volume along x, y and z, counted where
both voxels exist:
    S(mu) = - sum_axes sum_i (mu[i + e_axis] - mu[i])^2,
and its gradient dS/dmu.

Gradient entropy (the sharpness criterion of the paper's motion-compensated
FBP experiment, Sec. III-B): with the same forward differences (zero where
the neighbour is outside the grid), g_j = sqrt(dx_j^2 + dy_j^2 + dz_j^2 + eps),
p_j = g_j / sum_k g_k and GE = -sum_j p_j log p_j (lower = sharper).
"""
from __future__ import annotations

import math

import numpy as np


def ramlak(n: int, tau: float) -> np.ndarray:
    """Kernel values h[k] for k = -(n-1) .. n-1 (index k + n - 1)."""
    k = np.arange(-(n - 1), n, dtype=np.float64)
    h = np.zeros_like(k)
    odd = (np.abs(k) % 2) == 1
    h[odd] = -1.0 / (math.pi ** 2 * k[odd] ** 2 * tau ** 2)
    h[k == 0] = 1.0 / (4.0 * tau ** 2)
    return h


def fdk_filter(geom, proj, scale: float) -> np.ndarray:
    """Cosine-weighted, ramp-filtered projections [V][nv][nu] (float64)."""
    p = np.asarray(proj, dtype=np.float64)
    V, nv, nu = p.shape
    mag = geom.sad / geom.sdd
    cu, cv = (nu - 1) / 2.0 + geom.off_u, (nv - 1) / 2.0 + geom.off_v
    u = (np.arange(nu) - cu) * geom.du * mag
    v = (np.arange(nv) - cv) * geom.dv * mag
    cosw = geom.sad / np.sqrt(geom.sad ** 2 + u[None, :] ** 2 + v[:, None] ** 2)
    tau = geom.du * mag
    h = ramlak(nu, tau)
    out = np.empty_like(p)
    for vi in range(V):
        pw = p[vi] * cosw
        for b in range(nv):
            # full linear convolution, then the nu outputs aligned with the row
            out[vi, b] = np.convolve(pw[b], h)[nu - 1:2 * nu - 1]
    return out * (scale * tau)


def sharpness(vol) -> float:
    m = np.asarray(vol, dtype=np.float64)
    s = 0.0
    for ax in range(3):
        d = np.diff(m, axis=ax)
        s -= float(np.sum(d * d))
    return s


def sharpness_grad(vol) -> np.ndarray:
    """dS/dmu: each forward difference d = mu[i+e] - mu[i] contributes
    -2 d to mu[i+e] and +2 d to mu[i]."""
    m = np.asarray(vol, dtype=np.float64)
    g = np.zeros_like(m)
    for ax in range(3):
        d = np.diff(m, axis=ax)
        n = m.shape[ax]
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[ax] = slice(1, n)
        lo[ax] = slice(0, n - 1)
        g[tuple(hi)] -= 2.0 * d
        g[tuple(lo)] += 2.0 * d
    return g


def _forward_diffs(m):
    out = []
    for ax in range(3):
        d = np.zeros_like(m)
        n = m.shape[ax]
        lo = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        d[tuple(lo)] = np.diff(m, axis=ax)
        out.append(d)
    return out


def gradient_entropy(vol, eps: float = 1e-12) -> float:
    m = np.asarray(vol, dtype=np.float64)
    dx, dy, dz = _forward_diffs(m)
    g = np.sqrt(dx * dx + dy * dy + dz * dz + eps)
    p = g / g.sum()
    return float(-np.sum(p * np.log(p)))


def gradient_entropy_grad(vol, eps: float = 1e-12) -> np.ndarray:
    """dGE/dmu.  dGE/dg_j = -(log p_j + GE) / Z (Z = sum g), dg_j/dd = d / g_j,
    and each difference d_j = mu[j + e] - mu[j] feeds +1 into mu[j + e] and
    -1 into mu[j]."""
    m = np.asarray(vol, dtype=np.float64)
    diffs = _forward_diffs(m)
    g = np.sqrt(sum(d * d for d in diffs) + eps)
    Z = g.sum()
    p = g / Z
    ge = -np.sum(p * np.log(p))
    c = -(np.log(p) + ge) / (Z * g)
    out = np.zeros_like(m)
    for ax, d in enumerate(diffs):
        t = c * d
        n = m.shape[ax]
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[ax] = slice(1, n)
        lo[ax] = slice(0, n - 1)
        out -= t
        out[tuple(hi)] += t[tuple(lo)]
    return out
