"""BF16 MFMA CNN primitives and the proposal network against the FP64 oracle.

Operands are BF16 on both sides (the oracle rounds the same values with
round-to-nearest-even), so the GEMM differs only by FP32 accumulation order:
|C_gpu - C_ref| <= 1e-5 * (|A| |B|)_ij elementwise.  For whole-network
outputs and gradients, intermediate BF16 roundings may fall on the other
side of a rounding boundary; the normwise bar is 2e-2 (about 8 BF16 ulps).
"""
import numpy as np
import pytest
import torch

from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def bf(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV).to(torch.bfloat16)


@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (70, 45, 33), (128, 64, 96), (5, 300, 129)])
def test_gemm_all_layouts(dp, ta, tb, M, N, K):
    from paper_2508_13304_amd import proposal as pr
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = ocnn.bf16(rng.standard_normal((K, M) if ta else (M, K)))
    B = ocnn.bf16(rng.standard_normal((N, K) if tb else (K, N)))
    C = pr.gemm(bf(A), bf(B), ta=ta, tb=tb).cpu().numpy()
    Aop, Bop = (A.T if ta else A), (B.T if tb else B)
    ref = Aop @ Bop
    bound = np.abs(Aop) @ np.abs(Bop)
    assert np.all(np.abs(C - ref) <= 1e-5 * bound + 1e-30)


def test_gemm_split_k_and_accumulate(dp):
    from paper_2508_13304_amd import proposal as pr
    rng = np.random.default_rng(7)
    M, N, K = 18, 32, 70000  # few output tiles, long reduction: split over K
    A = ocnn.bf16(rng.standard_normal((K, M)))
    B = ocnn.bf16(rng.standard_normal((K, N)))
    C = pr.gemm(bf(A), bf(B), ta=True).cpu().numpy()
    ref = A.T @ B
    bound = np.abs(A.T) @ np.abs(B)
    assert np.all(np.abs(C - ref) <= 1e-5 * bound)
    C0 = torch.full((M, N), 2.0, device=DEV)
    pr.gemm(bf(A), bf(B), ta=True, out=C0, accumulate=True)
    assert np.all(np.abs(C0.cpu().numpy() - (ref + 2.0)) <= 1e-5 * bound + 1e-6)


@pytest.mark.parametrize("stride,Ci,Co", [(1, 5, 7), (2, 5, 7), (2, 16, 300), (1, 8, 32)])
def test_conv_layer_forward_backward(dp, stride, Ci, Co):
    """One conv layer through the library (im2col, GEMMs, col2im, column
    sums) against the oracle; channel counts that take the 16-byte im2col /
    float4 col2im paths (Ci multiple of 8 / 4) and the element paths, and a
    column sum wider than one 256-column strip."""
    from paper_2508_13304_amd import proposal as pr
    rng = np.random.default_rng(11 + stride + Ci)
    N, H, W = 2, 13, 10
    x = ocnn.bf16(rng.standard_normal((N, H, W, Ci)))
    Wt = ocnn.bf16(rng.standard_normal((Co, 3, 3, Ci)))
    b = rng.standard_normal(Co).astype(np.float32).astype(np.float64)
    col, Ho, Wo = pr.im2col(bf(x), stride)
    z = pr.gemm(col, bf(Wt.reshape(Co, -1)), tb=True).cpu().numpy().reshape(N, Ho, Wo, Co) + b
    zref = ocnn.conv3x3_forward(x, Wt, b, stride)
    assert np.abs(z - zref).max() <= 1e-5 * np.abs(zref).max()
    dz = ocnn.bf16(rng.standard_normal(zref.shape))
    dzt = bf(dz.reshape(-1, Co))
    dW = pr.gemm(dzt, col, ta=True).cpu().numpy().reshape(Co, 3, 3, Ci)
    dcol = pr.gemm(dzt, bf(Wt.reshape(Co, -1)))
    dx = pr.col2im(dcol, (N, H, W, Ci), stride).cpu().numpy()
    db = pr.colsum(dzt).cpu().numpy()
    dx_r, dW_r, db_r = ocnn.conv3x3_backward(x, Wt, dz, stride)
    for got, ref in ((dx, dx_r), (dW, dW_r), (db, db_r)):
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


def test_network_forward_backward_against_oracle(dp):
    from paper_2508_13304_amd import proposal as pr
    net = pr.ProposalNet(size=64, channels=(8, 16, 16, 32), seed=3)
    rng = np.random.default_rng(5)
    x = ocnn.bf16(rng.uniform(0, 1, (3, 64, 64, 2)))
    out, cache = net.forward(bf(x), keep=True)
    convs = [(W.cpu().numpy().astype(np.float64).reshape(W.shape[0], 3, 3, -1), b.cpu().numpy(), s)
             for W, b, s in net.convs]
    params = (convs, (net.Wfc.cpu().numpy().astype(np.float64), net.bfc.cpu().numpy()))
    ref, acts = ocnn.network_forward(x, params)
    got = out.cpu().numpy()
    assert np.linalg.norm(got - ref) <= 2e-2 * np.linalg.norm(ref)
    dout = rng.standard_normal((3, 6))
    grads, (dWfc, dbfc) = net.backward(cache, torch.tensor(dout, dtype=torch.float32, device=DEV))
    rgrads, (rWfc, rbfc) = ocnn.network_backward(params, acts, dout)
    assert np.linalg.norm(dWfc.cpu().numpy() - rWfc) <= 2e-2 * np.linalg.norm(rWfc)
    for (dW, db), (rW, rb) in zip(grads, rgrads):
        rW = rW.reshape(rW.shape[0], -1)
        assert np.linalg.norm(dW.cpu().numpy() - rW) <= 2e-2 * np.linalg.norm(rW)
        assert np.linalg.norm(db.cpu().numpy() - rb) <= 2e-2 * np.linalg.norm(rb) + 1e-12


def test_training_reduces_loss_on_a_fixed_batch(dp):
    from paper_2508_13304_amd import proposal as pr
    torch.manual_seed(0)
    net = pr.ProposalNet(size=32, channels=(16, 32, 32), seed=1)
    x = torch.rand((16, 32, 32, 2), device=DEV).to(torch.bfloat16)
    y = torch.randn((16, 6), device=DEV) * 0.5
    losses = []
    for _ in range(60):
        out, cache = net.forward(x, keep=True)
        d = out - y
        losses.append(float((d * d).mean()))
        grads, head = net.backward(cache, 2.0 * d / d.numel())
        net.adam_step(grads, head, lr=3e-3)
    assert losses[-1] < 0.2 * losses[0], losses[::10]


def test_full_size_trained_network_against_oracle(dp):
    """The committed proposal network at its real size (256^2 two-channel
    input, channels 32-64-128-256-256-256, batch 2, the batched layer shapes
    the training and inference launch) against the FP64 oracle network with
    the same BF16 rounding points: output and every parameter gradient within
    2e-2 in norm (BF16 roundings may fall on different sides once FP32 sums
    differ in order)."""
    import os
    from paper_2508_13304_amd import proposal as pr
    if not os.path.exists(pr.WEIGHTS):
        pytest.skip("no trained proposal weights committed")
    net = pr.ProposalNet.load(pr.WEIGHTS)
    rng = np.random.default_rng(7)
    x = ocnn.bf16(rng.uniform(0, 1, (2, net.size, net.size, 2)))
    out, cache = net.forward(bf(x), keep=True)
    convs = [(W.cpu().numpy().astype(np.float64).reshape(W.shape[0], 3, 3, -1), b.cpu().numpy(), s)
             for W, b, s in net.convs]
    params = (convs, (net.Wfc.cpu().numpy().astype(np.float64), net.bfc.cpu().numpy()))
    ref, acts = ocnn.network_forward(x, params)
    got = out.cpu().numpy()
    assert np.linalg.norm(got - ref) <= 2e-2 * np.linalg.norm(ref)
    dout = rng.standard_normal((2, 6))
    grads, (dWfc, dbfc) = net.backward(cache, torch.tensor(dout, dtype=torch.float32, device=DEV))
    rgrads, (rWfc, rbfc) = ocnn.network_backward(params, acts, dout)
    assert np.linalg.norm(dWfc.cpu().numpy() - rWfc) <= 2e-2 * np.linalg.norm(rWfc)
    for (dW, db), (rW, rb) in zip(grads, rgrads):
        rW = rW.reshape(rW.shape[0], -1)
        assert np.linalg.norm(dW.cpu().numpy() - rW) <= 2e-2 * np.linalg.norm(rW)
        assert np.linalg.norm(db.cpu().numpy() - rb) <= 2e-2 * np.linalg.norm(rb) + 1e-12


@pytest.mark.parametrize("relu", [True, False])
def test_bias_activation_and_its_backward_are_exact(dp, relu):
    """bias + ReLU to BF16 and the ReLU backward to BF16, element by element:
    FP32 arithmetic then round-to-nearest-even, bit-equal to torch's
    conversion of the same FP32 values (ragged column count, rows not a
    multiple of any block size)."""
    from paper_2508_13304_amd import proposal as pr
    g = torch.Generator(device=DEV).manual_seed(21)
    M, C = 1037, 37
    z = torch.randn((M, C), device=DEV, generator=g) * 3
    b = torch.randn(C, device=DEV, generator=g)
    y = pr.bias_act(z, b, relu=relu)
    ref = z + b
    if relu:
        ref = ref.clamp_min(0.0)
    assert torch.equal(y, ref.to(torch.bfloat16))
    dy = torch.randn((M, C), device=DEV, generator=g)
    dz = pr.act_bwd(dy, y, relu=relu)
    ref_dz = torch.where(y.float() > 0, dy, torch.zeros_like(dy)) if relu else dy
    assert torch.equal(dz, ref_dz.to(torch.bfloat16))


def _bf16_ulp(a):
    """Spacing of bfloat16 values at |a| (8 significant bits); 0 for a == 0."""
    a = np.abs(np.asarray(a, np.float64))
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a > 0, np.exp2(e - 7), 0.0)


def _layerwise_check(net, x):
    """Teacher-forced, element by element: every conv layer of the library is
    fed the oracle's own BF16 input activation of that layer, and its BF16
    output must equal the oracle's within one BF16 spacing plus the FP32
    accumulation bound 1e-5 (|W| |x| + |b|) of each element (identical
    operands, so the FP32 sums differ only in order, and a rounding to BF16
    can land on the neighbouring value only where the pre-activation lies
    within that bound of a rounding boundary); the head, fed the oracle's
    features, within 1e-5 (|W| |f| + |b|) per sample and output.  Then the
    end-to-end output, per sample and output, within 2^-4 of the output's
    magnitude scale (|W| |f| + |b|): a few BF16 flips compounded over the
    layers stay far below that, a wrong element does not."""
    from paper_2508_13304_amd import proposal as pr
    convs = [(W.cpu().numpy().astype(np.float64).reshape(W.shape[0], 3, 3, -1), b.cpu().numpy().astype(np.float64), s)
             for W, b, s in net.convs]
    Wfc = net.Wfc.cpu().numpy().astype(np.float64)
    bfc = net.bfc.cpu().numpy().astype(np.float64)
    ref, acts = ocnn.network_forward(x, (convs, (Wfc, bfc)))
    worst = 0.0
    for li, ((Wl, bl, s), (Wt, bt, _)) in enumerate(zip(convs, net.convs)):
        h = acts[li]
        col, Ho, Wo = pr.im2col(bf(h), s)
        z = pr.gemm(col, Wt.to(torch.bfloat16).contiguous(), tb=True)
        y = pr.bias_act(z, bt, relu=True).float().cpu().numpy().reshape(acts[li + 1].shape)
        yref = acts[li + 1]
        mag = ocnn.conv3x3_forward(np.abs(h), np.abs(ocnn.bf16(Wl)), np.abs(bl), s)
        tol = _bf16_ulp(np.maximum(np.abs(y), np.abs(yref))) + 1e-5 * mag + 1e-30
        err = np.abs(y - yref)
        assert np.all(err <= tol), (li, float((err / tol).max()))
        worst = max(worst, float((err / tol).max()))
    feat = acts[-1].reshape(acts[-1].shape[0], -1)
    out1 = (pr.gemm(bf(feat), net.Wfc.to(torch.bfloat16).contiguous(), tb=True) + net.bfc).cpu().numpy()
    scale = np.abs(feat) @ np.abs(ocnn.bf16(Wfc)).T + np.abs(bfc)
    assert np.all(np.abs(out1 - ref) <= 1e-5 * scale + 1e-30)
    got = net.forward(bf(x)).cpu().numpy()
    rel = np.abs(got - ref) / scale
    assert np.all(rel <= 2.0 ** -4), float(rel.max())
    return worst, float(rel.max())


def test_network_elementwise_small(dp):
    from paper_2508_13304_amd import proposal as pr
    net = pr.ProposalNet(size=64, channels=(8, 16, 16, 32), seed=3)
    rng = np.random.default_rng(15)
    _layerwise_check(net, ocnn.bf16(rng.uniform(0, 1, (3, 64, 64, 2))))


def test_network_elementwise_full_size(dp):
    import os
    from paper_2508_13304_amd import proposal as pr
    if not os.path.exists(pr.WEIGHTS):
        pytest.skip("no trained proposal weights committed")
    net = pr.ProposalNet.load(pr.WEIGHTS)
    rng = np.random.default_rng(17)
    _layerwise_check(net, ocnn.bf16(rng.uniform(0, 1, (2, net.size, net.size, 2))))


def test_fused_forward_epilogue_equals_separate_passes(dp):
    """The forward product with its bias + ReLU epilogue writes exactly what
    the FP32 product followed by the separate bias / activation pass writes
    (same MFMA accumulation, one rounding to BF16), for a row-padded operand
    with the bias read through a strided view."""
    from paper_2508_13304_amd import proposal as pr
    g = torch.Generator(device=DEV).manual_seed(31)
    M, N, K, row = 1000, 70, 45, 56
    a = (torch.randn((M, row), device=DEV, generator=g)).to(torch.bfloat16)
    blk = torch.randn((N, row), device=DEV, generator=g)
    b = blk[:, K]                       # bias column of the parameter block
    y = pr.gemm_bias_act(a, blk.to(torch.bfloat16), K, b, relu=True)
    z = pr.gemm(a[:, :K].contiguous(), blk[:, :K].to(torch.bfloat16).contiguous(), tb=True)
    assert torch.equal(y, pr.bias_act(z, b.contiguous(), relu=True))


def test_col2im_with_activation_backward_equals_separate_passes(dp):
    from paper_2508_13304_amd import proposal as pr
    g = torch.Generator(device=DEV).manual_seed(32)
    for (N, H, W, C, s) in ((2, 13, 10, 8, 2), (1, 9, 7, 5, 1)):
        Ho, Wo = (H - 1) // s + 1, (W - 1) // s + 1
        dcol = torch.randn((N * Ho * Wo, 9 * C), device=DEV, generator=g)
        y = torch.randn((N, H, W, C), device=DEV, generator=g).to(torch.bfloat16)
        dz = pr.col2im_act(dcol, (N, H, W, C), s, y, relu=True)
        dx = pr.col2im(dcol, (N, H, W, C), s)
        assert torch.equal(dz, pr.act_bwd(dx.reshape(-1, C), y.reshape(-1, C), relu=True).view(N, H, W, C))


def test_im2col_row_stride_and_ones_column(dp):
    from paper_2508_13304_amd import proposal as pr
    g = torch.Generator(device=DEV).manual_seed(33)
    for C, ld in ((2, 24), (8, 80)):
        x = torch.randn((2, 11, 9, C), device=DEV, generator=g).to(torch.bfloat16)
        col, Ho, Wo = pr.im2col(x, 2)
        colp, _, _ = pr.im2col(x, 2, ld=ld, ones=True)
        assert torch.equal(colp[:, :9 * C], col)
        assert torch.all(colp[:, 9 * C] == 1) and torch.all(colp[:, 9 * C + 1:] == 0)


def test_split_k_product_is_repeatable_and_matches_oracle(dp):
    """Weight-gradient shaped product (few output tiles, long reduction):
    split-K partials reduced in split order, so two launches agree bit for
    bit, and the result meets the elementwise FP32-accumulation bound."""
    from paper_2508_13304_amd import proposal as pr
    rng = np.random.default_rng(34)
    M, N, K = 64, 200, 60000
    A = ocnn.bf16(rng.standard_normal((K, M)))
    B = ocnn.bf16(rng.standard_normal((K, N)))
    C1 = pr.gemm(bf(A), bf(B), ta=True)
    C2 = pr.gemm(bf(A), bf(B), ta=True)
    assert torch.equal(C1, C2)
    ref = A.T @ B
    assert np.all(np.abs(C1.cpu().numpy() - ref) <= 1e-5 * (np.abs(A.T) @ np.abs(B)))


def test_fused_adam_matches_the_update_rule(dp):
    from paper_2508_13304_amd import proposal as pr
    g = torch.Generator(device=DEV).manual_seed(35)
    n = 100003
    p = torch.randn(n, device=DEV, generator=g)
    gr = torch.randn(n, device=DEV, generator=g)
    m = torch.randn(n, device=DEV, generator=g) * 0.1
    v = torch.rand(n, device=DEV, generator=g) * 0.01
    pb = torch.empty(n, dtype=torch.bfloat16, device=DEV)
    b1, b2, lr, eps, c1, c2 = 0.9, 0.999, 1e-3, 1e-8, 1 - 0.9 ** 3, 1 - 0.999 ** 3
    # the kernel takes FP32 constants: the reference uses the same values
    f = lambda a: float(np.float32(a))  # noqa: E731
    b1f, b2f, lrf, epsf, c1f, c2f = map(f, (b1, b2, lr, eps, c1, c2))
    m_ref = b1f * m.double() + f(1 - b1f) * gr.double()
    v_ref = b2f * v.double() + f(1 - b2f) * gr.double() ** 2
    p_ref = p.double() - lrf * (m_ref / c1f) / ((v_ref / c2f).sqrt() + epsf)
    mag_m = b1f * m.double().abs() + gr.double().abs() * 0.1
    mag_v = b2f * v.double() + gr.double() ** 2 * 1e-3
    pr.adam(p, gr, m, v, pb, lr, (b1, b2), eps, c1, c2)
    assert torch.all((m.double() - m_ref).abs() <= 4e-7 * mag_m)
    assert torch.all((v.double() - v_ref).abs() <= 4e-7 * mag_v)
    assert torch.allclose(p.double(), p_ref, rtol=1e-6, atol=1e-7)
    assert torch.equal(pb, p.to(torch.bfloat16))


def test_network_training_step_is_repeatable(dp):
    """Two networks from the same seed, one training step each on the same
    batch: bit-identical parameters afterwards (no atomics in any product or
    sum of the step)."""
    from paper_2508_13304_amd import proposal as pr
    x = torch.rand((8, 64, 64, 2), device=DEV, generator=torch.Generator(device=DEV).manual_seed(36))
    x = x.to(torch.bfloat16)
    y = torch.randn((8, 6), device=DEV, generator=torch.Generator(device=DEV).manual_seed(37))
    nets = [pr.ProposalNet(size=64, channels=(8, 16, 32), seed=4) for _ in range(2)]
    for net in nets:
        out, cache = net.forward(x, keep=True)
        grads, head = net.backward(cache, 2.0 * (out - y) / out.numel())
        net.adam_step(grads, head, lr=1e-3)
    assert torch.equal(nets[0].P, nets[1].P)


@pytest.mark.parametrize("N,H,W,Ci,Co,s", [(2, 13, 10, 8, 16, 2), (1, 9, 7, 16, 8, 1),
                                           (2, 16, 16, 32, 64, 2), (3, 7, 11, 64, 24, 2)])
def test_implicit_gemm_convolution_against_oracle(dp, N, H, W, Ci, Co, s):
    """The implicit-GEMM convolution entry points (operand tiles gathered from
    NHWC tensors: no im2col matrix, input gradient per parity class of input
    pixels: no col2im) against the FP64 oracle on ragged and odd sizes, both
    strides.  Forward (BF16 out, before ReLU) and input gradient (BF16 out,
    times the ReLU mask of a layer below): within one BF16 rounding plus the
    FP32 accumulation bound; weight and bias gradients (FP32): 1e-5 of the
    largest entry.  Forward and weight gradient are also bit-equal to the
    explicit im2col products (same MFMA accumulation order)."""
    from paper_2508_13304_amd import proposal as pr
    rng = np.random.default_rng(100 * Ci + Co + s)
    x = ocnn.bf16(rng.standard_normal((N, H, W, Ci)))
    Wt = ocnn.bf16(rng.standard_normal((Co, 3, 3, Ci)))
    b = rng.standard_normal(Co).astype(np.float32).astype(np.float64)
    row = pr._row_len(Ci)
    blk = torch.zeros((Co, row), dtype=torch.float32, device=DEV)
    blk[:, :9 * Ci] = torch.tensor(Wt.reshape(Co, -1), dtype=torch.float32, device=DEV)
    blk[:, 9 * Ci] = torch.tensor(b, dtype=torch.float32, device=DEV)
    wb = blk.to(torch.bfloat16)
    xb = bf(x)
    y = pr.conv_fwd(xb, wb, s, blk[:, 9 * Ci], relu=False)
    zref = ocnn.conv3x3_forward(x, Wt, b, s)
    got = y.float().cpu().numpy()
    tol = 2.0 ** -8 * np.abs(zref) + 1e-5 * np.abs(zref).max()
    assert np.all(np.abs(got - zref) <= tol)
    col, Ho, Wo = pr.im2col(xb, s, ld=row, ones=True)
    assert torch.equal(y.view(-1, Co), pr.gemm_bias_act(col, wb, 9 * Ci, blk[:, 9 * Ci], relu=False))

    dz = ocnn.bf16(rng.standard_normal(zref.shape))
    dzb = bf(dz.reshape(-1, Co))
    dw = torch.empty((Co, row), dtype=torch.float32, device=DEV)
    pr.conv_wgrad(xb, dzb, s, out=dw, ones=True)
    dx_r, dW_r, db_r = ocnn.conv3x3_backward(x, Wt, dz, s)
    dwn = dw.cpu().numpy()
    assert np.abs(dwn[:, :9 * Ci] - dW_r.reshape(Co, -1)).max() <= 1e-5 * np.abs(dW_r).max()
    assert np.abs(dwn[:, 9 * Ci] - db_r).max() <= 1e-5 * np.abs(db_r).max()
    assert np.all(dwn[:, 9 * Ci + 1:] == 0)
    assert torch.equal(dw, pr.gemm(dzb, col, ta=True))

    yb = ocnn.bf16(rng.standard_normal((N, H, W, Ci)))
    out = pr.conv_dgrad_act(dzb, wb, (N, H, W, Ci), s, bf(yb), relu=True)
    ref = dx_r * (yb > 0)
    got = out.float().cpu().numpy()
    tol = 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(dx_r).max()
    assert np.all(np.abs(got - ref) <= tol)
    plain = pr.conv_dgrad_act(dzb, wb, (N, H, W, Ci), s, relu=False).float().cpu().numpy()
    assert np.all(np.abs(plain - dx_r) <= 2.0 ** -8 * np.abs(dx_r) + 1e-5 * np.abs(dx_r).max())
