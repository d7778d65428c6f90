"""Pins of the FP64 warm-start CNN oracle against things other than itself:
scipy's 2D correlation, adjoint identities, central finite differences of
the loss, and Adam's closed-form first step."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def test_conv3x3_is_scipy_correlation_with_zero_padding():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 5, 7))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = cnn.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, c], w[o, :, :, c], mode="same", boundary="fill")
                             for c in range(3))
            np.testing.assert_allclose(out[n, o], ref, rtol=1e-12, atol=1e-12)


def test_pool_and_up_adjoints():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 8, 6))
    y = rng.standard_normal((2, 3, 4, 3))
    assert np.isclose(np.sum(cnn.pool(x) * y), np.sum(x * cnn.pool_backward(y)), rtol=1e-13)
    xs = rng.standard_normal((2, 3, 4, 3))
    ys = rng.standard_normal((2, 3, 8, 6))
    assert np.isclose(np.sum(cnn.up(xs) * ys), np.sum(xs * cnn.up_backward(ys)), rtol=1e-13)
    # pool of a constant is the constant; up then pool is the identity
    assert np.allclose(cnn.pool(np.full((1, 1, 4, 4), 3.0)), 3.0)
    assert np.allclose(cnn.pool(cnn.up(xs)), xs)


def test_conv_backward_is_the_adjoint():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 6, 5))
    w = rng.standard_normal((4, 3, 3, 3))
    dz = rng.standard_normal((2, 4, 6, 5))
    dx, dw, db = cnn.conv3x3_backward(x, w, dz)
    zero = np.zeros(4)
    # linear in x and in w separately
    assert np.isclose(np.sum(cnn.conv3x3(x, w, zero) * dz), np.sum(x * dx), rtol=1e-12)
    assert np.isclose(np.sum(cnn.conv3x3(x, w, zero) * dz), np.sum(w * dw), rtol=1e-12)
    # bias enters every pixel once
    assert np.allclose(db, dz.sum(axis=(0, 2, 3)))


@pytest.mark.parametrize("channels", [(2, 3), (2, 3, 4, 5)])
def test_loss_gradient_matches_central_differences(channels):
    rng = np.random.default_rng(3)
    L = len(channels)
    n = 4 * 2 ** (L - 1)
    p = cnn.init_params(channels, seed=5)
    for k in p:                               # non-zero biases and head terms
        if k.endswith(".b") or k.startswith("head"):
            p[k] = p[k] + 0.1 * rng.standard_normal(p[k].shape)
    u = rng.uniform(0.0, 2.0, (2, n, n))
    target = rng.uniform(0.0, 1.0, (2, n, n))
    scale = 0.7
    loss, g, _ = cnn.loss_and_grads(p, u, target, scale, levels=L)
    assert set(g) == set(p)
    h = 1e-6
    for k in sorted(p):
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(3, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = cnn.loss_and_grads(p, u, target, scale, levels=L)[0]
            flat[idx] = old - h
            lm = cnn.loss_and_grads(p, u, target, scale, levels=L)[0]
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3 * abs(loss)), (k, idx, fd, an)


def test_forward_shapes_and_head_identity():
    """With every conv weight zero the network output is bh + cu * in_scale * u."""
    p = cnn.init_params((2, 3, 4), seed=1)
    for k in p:
        p[k] = np.zeros_like(p[k])
    p["head.b"][:] = 0.25
    p["head.cu"][:] = 2.0
    u = np.random.default_rng(0).standard_normal((3, 16, 16))
    x0, cache = cnn.forward(p, u, 0.5, levels=3)
    assert x0.shape == (3, 16, 16)
    np.testing.assert_allclose(x0, 0.25 + 2.0 * 0.5 * u, rtol=1e-15)
    assert cache["e3b.out"].shape == (3, 4, 4, 4)
    assert cache["d1a.in"].shape == (3, 4, 16, 16)


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(4)
    p = {"a": rng.standard_normal(7)}
    g = {"a": rng.standard_normal(7)}
    m = {"a": np.zeros(7)}
    v = {"a": np.zeros(7)}
    p0 = p["a"].copy()
    cnn.adam_step(p, g, m, v, 1, 1e-3)
    np.testing.assert_allclose(p["a"], p0 - 1e-3 * np.sign(g["a"]), rtol=0, atol=1e-10)
