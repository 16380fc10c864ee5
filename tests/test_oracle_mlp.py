"""Pins of the FP64 network reference: finite differences and a closed-form
one-step Adam case."""

import numpy as np

from oracle import mlp


def _shape_params(seed, shape):
    n_in, nh, n_out = shape
    rng = np.random.default_rng(seed)
    P = n_in * nh + nh + nh * nh + nh + nh * n_out + n_out
    return rng.normal(size=P) * 0.3


def test_gradient_matches_finite_differences():
    shape = (7, 5, 3)
    p = _shape_params(0, shape)
    rng = np.random.default_rng(1)
    x, t = rng.normal(size=(6, 7)), rng.normal(size=(6, 3))
    loss, g = mlp.loss_grad(p, x, t, shape)
    h = 1e-6
    for k in range(0, len(p), 3):
        e = np.zeros_like(p)
        e[k] = h
        fd = (mlp.loss_grad(p + e, x, t, shape)[0] - mlp.loss_grad(p - e, x, t, shape)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-8 * max(1.0, abs(fd))


def test_silu_and_its_derivative():
    z = np.linspace(-30, 30, 601)
    assert np.allclose(mlp.silu(z), z * 0.5 * (1 + np.tanh(z / 2)), atol=1e-14)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.silu_grad(z)).max() < 1e-8


def test_first_adam_step_moves_by_lr_times_sign():
    """With zero moments, the bias-corrected first step is lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3])
    p1, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
