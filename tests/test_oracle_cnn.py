"""Pins of the FP64 CNN oracle: scipy's periodic correlation, finite-difference
gradients, and Adam's first-step closed form."""

import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn


def test_conv_matches_scipy_periodic_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 7, 6))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = cnn.conv(x, w, b)
    for bi in range(2):
        for co in range(4):
            ref = b[co] + sum(ndimage.correlate(x[bi, ci], w[co, ci], mode="wrap") for ci in range(3))
            assert np.allclose(y[bi, co], ref, atol=1e-12)


def _loss(params, x, t):
    out, _ = cnn.forward(params, x)
    return cnn.mse(out, t)[0]


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    layers = ((3, 5), (5, 4), (4, 3))
    params = cnn.init_params(3, layers)
    params = [(w, rng.standard_normal(b.shape) * 0.1) for w, b in params]
    x = rng.standard_normal((2, 3, 5, 6))
    t = rng.standard_normal((2, 3, 5, 6))
    out, cache = cnn.forward(params, x)
    _, dout = cnn.mse(out, t)
    grads, dx = cnn.backward(params, cache, dout)
    h = 1e-6
    for li, (w, b) in enumerate(params):
        for arr, g in ((w, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gflat = g.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = _loss(params, x, t)
                flat[idx] = old - h
                lm = _loss(params, x, t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gflat[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (li, idx)
    xf = x.reshape(-1)
    for idx in rng.choice(xf.size, size=6, replace=False):
        old = xf[idx]
        xf[idx] = old + h
        lp = _loss(params, x, t)
        xf[idx] = old - h
        lm = _loss(params, x, t)
        xf[idx] = old
        assert abs((lp - lm) / (2 * h) - dx.reshape(-1)[idx]) <= 1e-6


def test_parameter_count():
    params = cnn.init_params(0)
    assert sum(w.size + b.size for w, b in params) == 20259


def test_adam_first_step_is_signed_lr():
    """After one step from zero moments, m_hat = g and v_hat = g^2, so each
    parameter moves by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    params = [(rng.standard_normal((2, 3, 3, 3)), rng.standard_normal(2))]
    grads = [(rng.standard_normal((2, 3, 3, 3)), rng.standard_normal(2))]
    opt = cnn.Adam(params, lr=0.01)
    new = opt.step(params, grads)
    for (p, g, q) in ((params[0][0], grads[0][0], new[0][0]), (params[0][1], grads[0][1], new[0][1])):
        assert np.allclose(q, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    new2 = opt.step(new, grads)  # second step with the same gradient: still ~lr * sign(g)
    assert np.allclose(new2[0][1] - new[0][1], -0.01 * np.sign(grads[0][1]), rtol=1e-6)
