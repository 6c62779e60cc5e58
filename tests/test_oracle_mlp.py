"""Pins of the reference MLP: central finite differences of the loss, and the
closed-form GELU derivative.  CPU only."""
import math

import numpy as np

from oracle import mlp


def test_gelu_derivative_matches_finite_differences():
    x = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-8
    # GELU(x) = x Phi(x): spot values
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(-1.0) + 0.15865525393145707) < 1e-15


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    sizes = mlp.layer_sizes(4, 7, 3, 5)
    p = mlp.init_params(sizes, rng) + 0.05 * rng.standard_normal(mlp.n_params(sizes))
    X = rng.standard_normal((6, 4))
    T = rng.standard_normal((6, 5))
    loss, g = mlp.loss_and_grad(p, sizes, X, T)
    h = 1e-6
    for idx in rng.choice(p.size, 40, replace=False):
        e = np.zeros_like(p)
        e[idx] = h
        lp, _ = mlp.loss_and_grad(p + e, sizes, X, T)
        lm, _ = mlp.loss_and_grad(p - e, sizes, X, T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(fd)), (idx, fd, g[idx])


def test_adam_first_step_moves_by_lr_times_sign():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 2.0])
    p1, m, v = mlp.adam_step(p, np.zeros(3), np.zeros(3), g, 1, 0.01)
    # bias-corrected first step is lr * g / (|g| + eps)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(1)
    sizes = mlp.layer_sizes(2, 16, 2, 1)
    p = mlp.init_params(sizes, rng)
    X = rng.uniform(-1, 1, (64, 2))
    T = np.sin(2 * X[:, :1]) * np.cos(X[:, 1:])
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0, _ = mlp.loss_and_grad(p, sizes, X, T)
    for t in range(1, 301):
        _, g = mlp.loss_and_grad(p, sizes, X, T)
        p, m, v = mlp.adam_step(p, m, v, g, t, 1e-2)
    l1, _ = mlp.loss_and_grad(p, sizes, X, T)
    assert l1 < 0.05 * l0
