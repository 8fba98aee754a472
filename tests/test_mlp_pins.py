"""Pins of the FP64 surrogate network: gradients against central finite
differences (independent of the analytic backward pass), GELU against the
normal CDF of scipy, and Adam against a hand-worked first step."""
import math

import numpy as np
from scipy import stats

from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 133_633


def test_gelu_is_x_times_normal_cdf():
    x = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(x), x * stats.norm.cdf(x), rtol=1e-13, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(x), fd, rtol=1e-7, atol=1e-9)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    theta = mlp.init_params(5)
    x = rng.standard_normal((7, 6))
    y = (rng.uniform(size=7) < 0.5).astype(np.float64)
    _, g = mlp.loss_and_grad(theta, x, y)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False),
                          [0, 1535, 1536, 1791, mlp.N_PARAMS - 2, mlp.N_PARAMS - 1]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp, _ = mlp.loss_and_grad(tp, x, y)
        lm, _ = mlp.loss_and_grad(tm, x, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bce_matches_definition():
    z = np.array([-30.0, -2.0, 0.0, 1.5, 40.0])
    y = np.array([0.0, 1.0, 1.0, 0.0, 1.0])
    p = 1 / (1 + np.exp(-z))
    want = -np.mean(y * np.log(np.where(y == 1, p, 1)) + (1 - y) * np.log(np.where(y == 0, 1 - p, 1)))
    assert math.isclose(mlp.bce_loss(z, y), want, rel_tol=1e-12)


def test_adam_first_step_moves_by_lr_times_sign():
    """With zero moments, the bias-corrected first step is lr * g / (|g| + eps)."""
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    new, m, v = mlp.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=1e-2)
    assert np.allclose(new, theta - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_reduces_loss_on_a_separable_problem():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((256, 6))
    y = (x[:, 0] + 0.5 * x[:, 1] > 0).astype(np.float64)
    theta = mlp.init_params(11)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0, _ = mlp.loss_and_grad(theta, x, y)
    for t in range(1, 31):
        _, g = mlp.loss_and_grad(theta, x, y)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, lr=3e-3)
    l1, _ = mlp.loss_and_grad(theta, x, y)
    assert l1 < 0.5 * l0
