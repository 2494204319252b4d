"""Pins of the surrogate's FP64 reference against library routines and
exact identities (no GPU)."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import nn_oracle as N


def _rng(seed):
    return np.random.default_rng(seed)


def test_conv3x3_matches_scipy_wrap_correlation():
    r = _rng(1)
    x = r.standard_normal((2, 7, 10, 3))
    w = r.standard_normal((4, 9, 3))
    bias = r.standard_normal(4)
    y = N.conv3x3(x, w, bias)
    for b in range(2):
        for o in range(4):
            want = np.full((7, 10), bias[o])
            for i in range(3):
                k = w[o, :, i].reshape(3, 3)     # k[dy+1, dx+1]
                want += ndi.correlate(x[b, :, :, i], k, mode="wrap")
            np.testing.assert_allclose(y[b, :, :, o], want, rtol=1e-12, atol=1e-12)


def test_conv3x3_adjoints():
    r = _rng(2)
    x = r.standard_normal((2, 6, 8, 5))
    w = r.standard_normal((3, 9, 5))
    g = r.standard_normal((2, 6, 8, 3))
    lhs = np.sum(N.conv3x3(x, w) * g)
    assert abs(lhs - np.sum(x * N.conv3x3_dgrad(g, w))) < 1e-10 * abs(lhs)
    dw, db = N.conv3x3_wgrad(x, g)
    assert abs(lhs - np.sum(w * dw)) < 1e-10 * abs(lhs)
    # bias gradient: d/dbias sum(conv(x, w, bias) * g) = sum of g over pixels
    np.testing.assert_allclose(db, g.reshape(-1, 3).sum(axis=0), rtol=1e-13)


def test_conv3x3_gradients_by_finite_differences():
    r = _rng(3)
    x = r.standard_normal((1, 5, 6, 2))
    w = r.standard_normal((2, 9, 2))
    g = r.standard_normal((1, 5, 6, 2))

    def L(xx, ww):
        return np.sum(N.conv3x3(xx, ww) ** 2 * g)

    y = N.conv3x3(x, w)
    gy = 2 * y * g
    dx = N.conv3x3_dgrad(gy, w)
    dw, _ = N.conv3x3_wgrad(x, gy)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 4, 5, 1), (0, 2, 3, 0)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (L(x + e, w) - L(x - e, w)) / (2 * h)
        assert abs(fd - dx[idx]) < 1e-6 * max(1, abs(fd))
    for idx in [(0, 0, 0), (1, 8, 1), (0, 4, 1)]:
        e = np.zeros_like(w)
        e[idx] = h
        fd = (L(x, w + e) - L(x, w - e)) / (2 * h)
        assert abs(fd - dw[idx]) < 1e-6 * max(1, abs(fd))


def test_pool_and_upsample_adjoints():
    r = _rng(4)
    x = r.standard_normal((2, 8, 6, 3))
    y = r.standard_normal((2, 4, 3, 3))
    assert abs(np.sum(N.avgpool2(x) * y) - np.sum(x * N.avgpool2_bwd(y))) < 1e-12
    z = r.standard_normal((2, 8, 6, 3))
    assert abs(np.sum(N.upsample2(y) * z) - np.sum(y * N.upsample2_bwd(z))) < 1e-12
    np.testing.assert_allclose(N.avgpool2(N.upsample2(y)), y, rtol=1e-15)


def test_rel_l2_gradient_by_finite_differences():
    r = _rng(5)
    p = r.standard_normal((3, 4, 5, 6))
    t = r.standard_normal((3, 4, 5, 6))
    loss, per, g = N.rel_l2(p, t)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (2, 3, 4, 5), (1, 2, 1, 3)]:
        e = np.zeros_like(p)
        e[idx] = h
        fd = (N.rel_l2(p + e, t)[0] - N.rel_l2(p - e, t)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7
    np.testing.assert_allclose(per ** 2, [np.sum((p[b] - t[b]) ** 2) / np.sum(t[b] ** 2) for b in range(3)])


def test_leaky_relu():
    z = np.array([-2.0, -0.5, 0.0, 0.5, 3.0])
    np.testing.assert_array_equal(N.leaky(z), [-0.25, -0.0625, 0.0, 0.5, 3.0])
    np.testing.assert_array_equal(N.leaky_bwd(N.leaky(z), np.ones(5)), [0.125, 0.125, 0.125, 1, 1])


def test_bf16_rounding_matches_torch():
    import torch
    a = _rng(6).standard_normal(10000).astype(np.float32) * 10.0 ** _rng(7).integers(-5, 5, 10000)
    want = torch.tensor(a).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    np.testing.assert_array_equal(N.bf16_round(a), want)


def test_unet_gradient_by_finite_differences():
    """The oracle network's backward against central differences of its
    forward (exact FP64), on a 32 x 32 lattice."""
    layers = N.unet_layers()
    _, n = N.unpack_params(np.zeros(10 ** 7))
    r = _rng(8)
    p = np.zeros(n)
    off = 0
    for name, ci, co, _, _ in layers:
        p[off:off + co * 9 * ci] = r.standard_normal(co * 9 * ci) * np.sqrt(2.0 / (9 * ci))
        p[off + co * 9 * ci:off + co * 9 * ci + co] = 0.01 * r.standard_normal(co)
        off += co * 9 * ci + co
    x = r.standard_normal((1, 32, 32, 48))
    t = r.standard_normal((1, 32, 32, 32))

    def loss(pp):
        out, _ = N.unet_forward(pp, x)
        return 0.5 * np.sum((out - t) ** 2)

    out, act = N.unet_forward(p, x)
    g = N.unet_backward(p, act, out - t)
    h = 1e-5
    picks = [0, 100, 5000, n // 3, n // 2, n - 40, n - 1]
    for i in picks:
        e = np.zeros(n)
        e[i] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(fd)), (i, fd, g[i])
