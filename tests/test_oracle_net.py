"""Pins for oracle.net: convolution against scalar loops and a hand-computed
example, GELU against its closed form, gradients against central finite
differences, Adam against the closed-form first step."""

import math

import numpy as np
import pytest

from oracle import net


def test_param_count():
    assert net.param_count() == 28641


def test_conv_hand_example():
    """3x3 image, one channel, kernel with only the centre and right taps:
    z[y, x] = b + 2 a[y, x] + 3 a[y, x+1] (zero beyond the right edge)."""
    a = np.arange(9, dtype=np.float64).reshape(1, 1, 3, 3)
    w = np.zeros((1, 1, 3, 3))
    w[0, 0, 1, 1] = 2.0
    w[0, 0, 1, 2] = 3.0
    z = net.conv3x3(a, w, np.array([0.5]))
    expect = np.array([[0.5 + 0 + 3, 0.5 + 2 + 6, 0.5 + 4 + 0],
                       [0.5 + 6 + 12, 0.5 + 8 + 15, 0.5 + 10 + 0],
                       [0.5 + 12 + 21, 0.5 + 14 + 24, 0.5 + 16 + 0]])
    np.testing.assert_allclose(z[0, 0], expect, rtol=0, atol=1e-14)


def test_conv_matches_scalar_loops():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((2, 3, 5, 6))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(net.conv3x3(a, w, b), net.conv3x3_loops(a, w, b), rtol=1e-12, atol=1e-12)


def test_gelu_closed_form_values():
    x = np.array([-2.0, -0.5, 0.0, 0.5, 2.0])
    phi = 0.5 * (1.0 + np.array([math.erf(t / math.sqrt(2.0)) for t in x]))
    np.testing.assert_allclose(net.gelu(x), x * phi, rtol=1e-15)
    # derivative by central differences
    h = 1e-6
    np.testing.assert_allclose(net.gelu_grad(x), (net.gelu(x + h) - net.gelu(x - h)) / (2 * h), rtol=1e-7, atol=1e-9)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = net.he_init(3)
    f = 40.0 * rng.standard_normal((2, 6, 7))
    x = net.features(f, rng.standard_normal((2, 6, 7)))
    target = rng.standard_normal((2, 6, 7))
    loss, g = net.loss_and_grad(theta, x, target)
    idx = rng.choice(theta.size, size=40, replace=False)
    # include every layer's bias and some first/last-layer weights
    idx = np.concatenate([idx, [0, 300, 580, 608 + 5, theta.size - 1, theta.size - 2]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (net.mse(net.forward(tp, x)[0], target) - net.mse(net.forward(tm, x)[0], target)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_adam_first_step_is_sign_times_lr():
    """At t = 1 with zero moments, m_hat = g and v_hat = g^2, so the step is
    lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    theta, m, v = net.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(theta, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
