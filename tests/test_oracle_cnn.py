"""Pins for the CNN oracle (oracle/cnn.py): library correlation, finite
differences and an independent bfloat16 conversion."""
import numpy as np
import torch
from scipy.signal import correlate2d

from oracle import cnn


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(0).standard_normal(10000) * 10 ** np.random.default_rng(1).uniform(-5, 5, 10000)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(x), ref)


def test_conv_forward_matches_scipy_correlation():
    rng = np.random.default_rng(2)
    for stride in (1, 2):
        x = rng.standard_normal((2, 9, 7, 3))
        W = rng.standard_normal((4, 3, 3, 3))
        b = rng.standard_normal(4)
        z = cnn.conv3x3_forward(x, W, b, stride)
        for n in range(2):
            for co in range(4):
                full = sum(correlate2d(np.pad(x[n, :, :, ci], 1), W[co, :, :, ci], mode="valid")
                           for ci in range(3)) + b[co]
                np.testing.assert_allclose(z[n, :, :, co], full[::stride, ::stride], atol=1e-12)


def test_conv_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 6, 5, 2))
    W = rng.standard_normal((3, 3, 3, 2))
    b = rng.standard_normal(3)
    for stride in (1, 2):
        dz = rng.standard_normal(cnn.conv3x3_forward(x, W, b, stride).shape)
        dx, dW, db = cnn.conv3x3_backward(x, W, dz, stride)
        f = lambda x_, W_, b_: np.sum(dz * cnn.conv3x3_forward(x_, W_, b_, stride))  # noqa: E731
        h = 1e-6
        for arr, grad in ((x, dx), (W, dW), (b, db)):
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
                e = np.zeros_like(arr)
                e[idx] = h
                args = [x, W, b]
                pos = [a is arr for a in args].index(True)
                ap, am = list(args), list(args)
                ap[pos], am[pos] = arr + e, arr - e
                fd = (f(*ap) - f(*am)) / (2 * h)
                assert abs(fd - grad[idx]) < 1e-6 * (1 + abs(fd))


def test_network_gradients_match_finite_differences():
    rng = np.random.default_rng(4)
    convs = [(rng.standard_normal((4, 3, 3, 2)) * 0.5, rng.standard_normal(4) * 0.1, 2),
             (rng.standard_normal((5, 3, 3, 4)) * 0.5, rng.standard_normal(5) * 0.1, 2)]
    x = rng.standard_normal((3, 8, 8, 2))
    Wfc = rng.standard_normal((6, 2 * 2 * 5)) * 0.3
    bfc = rng.standard_normal(6) * 0.1
    params = (convs, (Wfc, bfc))
    dout = rng.standard_normal((3, 6))
    out, acts = cnn.network_forward(x, params, round_bf16=False)
    grads, (dWfc, dbfc) = cnn.network_backward(params, acts, dout, round_bf16=False)
    f = lambda p: np.sum(dout * cnn.network_forward(x, p, round_bf16=False)[0])  # noqa: E731
    h = 1e-6
    W0 = convs[0][0]
    for idx in [(0, 1, 1, 0), (3, 2, 0, 1), (1, 0, 2, 1)]:
        e = np.zeros_like(W0)
        e[idx] = h
        pp = ([(W0 + e, convs[0][1], 2), convs[1]], (Wfc, bfc))
        pm = ([(W0 - e, convs[0][1], 2), convs[1]], (Wfc, bfc))
        fd = (f(pp) - f(pm)) / (2 * h)
        assert abs(fd - grads[0][0][idx]) < 1e-5 * (1 + abs(fd))
    e = np.zeros_like(Wfc)
    e[2, 7] = h
    fd = (f((convs, (Wfc + e, bfc))) - f((convs, (Wfc - e, bfc)))) / (2 * h)
    assert abs(fd - dWfc[2, 7]) < 1e-5 * (1 + abs(fd))
