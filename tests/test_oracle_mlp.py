"""Pins of the FP64 network reference: central finite differences and Adam by hand."""
import math

import numpy as np

from oracle import mlp_oracle as M


def test_param_count():
    assert M.NPARAM == 6401


def test_gelu_values():
    # exact-erf GELU at a few points: x * Phi(x)
    from scipy.stats import norm
    x = np.array([-3.0, -0.5, 0.0, 0.7, 2.5])
    np.testing.assert_allclose(M.gelu(x), x * norm.cdf(x), rtol=1e-14, atol=1e-300)


def test_gradient_finite_difference():
    rng = np.random.default_rng(0)
    theta = M.init_params(rng)
    X = rng.standard_normal((7, 33))
    y = rng.standard_normal(7)
    _, g = M.loss_and_grad(theta, X, y)
    idx = rng.choice(M.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [M.NPARAM - 1, 0, 2112, 2176, 6336]])
    hstep = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += hstep
        tm = theta.copy(); tm[i] -= hstep
        fd = (M.loss_and_grad(tp, X, y)[0] - M.loss_and_grad(tm, X, y)[0]) / (2 * hstep)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_adam_by_hand():
    theta = np.array([1.0, -2.0])
    grad = np.array([0.5, -0.25])
    m = np.zeros(2); v = np.zeros(2)
    th, m, v = M.adam_step(theta, grad, m, v, 1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2 -> update = lr * sign(g) (eps negligible)
    np.testing.assert_allclose(th, theta - 0.1 * np.sign(grad) * np.abs(grad) / (np.abs(grad) + 1e-8), rtol=1e-15)
    th2, m2, v2 = M.adam_step(th, grad, m, v, 2, lr=0.1)
    mh = (0.9 * m + 0.1 * grad) / (1 - 0.81)
    vh = (0.999 * v + 0.001 * grad ** 2) / (1 - 0.999 ** 2)
    np.testing.assert_allclose(th2, th - 0.1 * mh / (np.sqrt(vh) + 1e-8), rtol=1e-15)


def test_training_reduces_loss():
    rng = np.random.default_rng(1)
    theta = M.init_params(rng)
    X = rng.standard_normal((64, 33))
    w = rng.standard_normal(33) / 6
    y = np.tanh(X @ w)
    m = np.zeros_like(theta); v = np.zeros_like(theta)
    l0 = M.loss_and_grad(theta, X, y)[0]
    for t in range(1, 201):
        _, g = M.loss_and_grad(theta, X, y)
        theta, m, v = M.adam_step(theta, g, m, v, t, lr=3e-3)
    assert M.loss_and_grad(theta, X, y)[0] < 0.2 * l0
