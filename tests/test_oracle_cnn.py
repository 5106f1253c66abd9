"""Pins of the FP64 CNN reference (P12): convolution against brute force and
scipy, backward against central differences, loss gradient closed form, Adam's
first step closed form."""

import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def test_conv_matches_bruteforce_and_scipy():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 6))
    W = rng.standard_normal((3, 2, 3, 3))
    b = rng.standard_normal(3)
    y = cnn.conv3x3(x, W, b)
    for o in range(3):
        for i in range(5):
            for j in range(6):
                s = b[o]
                for c in range(2):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            ii, jj = i + dy, j + dx
                            if 0 <= ii < 5 and 0 <= jj < 6:
                                s += W[o, c, dy + 1, dx + 1] * x[c, ii, jj]
                assert y[o, i, j] == pytest.approx(s, abs=1e-12)
        ref = sum(correlate2d(x[c], W[o, c], mode="same") for c in range(2)) + b[o]
        np.testing.assert_allclose(y[o], ref, atol=1e-12)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    p = cnn.init_params(Q=2, C=3, seed=2)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    x = np.abs(rng.standard_normal((2, 5, 6)))
    t = (rng.random((5, 6)) > 0.6).astype(float)
    pw = 3.0
    prob, cache = cnn.forward(p, x)
    g = cnn.backward(p, cache, t, pw)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = cnn.bce_loss(cnn.forward(p, x)[0], t, pw)
            flat[idx] = old - h
            lm = cnn.bce_loss(cnn.forward(p, x)[0], t, pw)
            flat[idx] = old
            num = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert an == pytest.approx(num, rel=1e-6, abs=1e-10), (k, idx)


def test_bce_gradient_closed_form():
    """dL/da4 = w (sigmoid(a4) - t) / HW: a one-layer check through W4 = 0."""
    rng = np.random.default_rng(3)
    p = cnn.init_params(Q=1, C=2, seed=4)
    p["W4"][:] = 0.0
    p["b4"][:] = 0.3
    x = np.abs(rng.standard_normal((1, 4, 4)))
    t = (rng.random((4, 4)) > 0.5).astype(float)
    prob, cache = cnn.forward(p, x)
    g = cnn.backward(p, cache, t, 2.0)
    w = np.where(t > 0.5, 2.0, 1.0)
    assert g["b4"][0] == pytest.approx(float((w * (cnn.sigmoid(0.3) - t)).sum() / 16), rel=1e-12)


def test_adam_first_step():
    """With bias correction the first step is -lr * g / (|g| + eps)."""
    p = {"a": np.array([1.0, -2.0, 0.5])}
    g = {"a": np.array([0.3, -4.0, 1e-3])}
    opt = cnn.Adam(p, lr=0.01, eps=1e-8)
    opt.step(p, g)
    np.testing.assert_allclose(p["a"], np.array([1.0, -2.0, 0.5]) - 0.01 * g["a"] / (np.abs(g["a"]) + 1e-8))


def test_labels_from_solution():
    z = np.array([0.0, 1.0, 0.0, 0.0])
    act = np.array([[False, False, True, False], [False, True, False, False]])
    np.testing.assert_array_equal(cnn.labels_from_solution(z, act), [1, 0, 0, 1])
