"""Pins of the chooser-network oracle: finite differences and Adam's first step.

The paper has no learned component (parity unpinned by the paper); these
checks pin the fp64 oracle by mathematics only.
"""
import numpy as np
import pytest

from oracle import mlp


def batch(seed, B=7):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, 16)), rng.standard_normal((B, 3))


def test_param_count():
    assert mlp.NPARAM == 5443
    p = mlp.init_params(0)
    assert p.shape == (5443,)
    assert np.array_equal(mlp.pack(mlp.unpack(p)), p)


def test_gradient_matches_central_differences():
    p = mlp.init_params(1) + np.random.default_rng(2).normal(0, 0.05, mlp.NPARAM)
    X, T = batch(3)
    shift = np.linspace(-1, 1, 16)
    scale = np.linspace(0.5, 2, 16)
    _, g = mlp.loss_and_grad(p, X, T, shift, scale)
    h = 1e-6
    idx = np.random.default_rng(4).choice(mlp.NPARAM, 300, replace=False)
    idx = np.concatenate([idx, [0, 1023, 1024, 1087, 1088, 5247, 5248, 5439, 5440, 5442]])
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        lp, _ = mlp.loss_and_grad(p + e, X, T, shift, scale)
        lm, _ = mlp.loss_and_grad(p - e, X, T, shift, scale)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, i


def test_forward_consistent_with_loss():
    p = mlp.init_params(5)
    X, T = batch(6)
    y = mlp.forward(p, X)
    loss, _ = mlp.loss_and_grad(p, X, T)
    assert loss == pytest.approx(np.mean((y - T) ** 2))
    # zero weights: output is the last bias
    z = np.zeros(mlp.NPARAM)
    z[-3:] = [1.0, -2.0, 0.5]
    assert np.allclose(mlp.forward(z, X), [1.0, -2.0, 0.5])


def test_adam_first_step_closed_form():
    """With zero moments, step 1 moves every weight by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(8)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr = 1e-3
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr)
    assert np.allclose(p - p1, lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((64, 16))
    T = np.tanh(X[:, :3] * 0.7)
    p = mlp.init_params(10)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0, _ = mlp.loss_and_grad(p, X, T)
    for t in range(1, 201):
        loss, g = mlp.loss_and_grad(p, X, T)
        p, m, v = mlp.adam_step(p, g, m, v, t, 1e-2)
    assert loss < 0.1 * l0
