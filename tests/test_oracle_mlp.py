"""Pins of the oracle surrogate network: backward pass against central
finite differences, Adam's closed-form first step, and a loss that falls on
a smooth regression."""
import numpy as np
import pytest

from oracle import mlp


def tiny(seed=0, n_in=4, hidden=7, n_out=3):
    rng = np.random.default_rng(seed)
    vec = mlp.init_from_normals(rng.standard_normal(mlp.n_params(n_in, hidden, n_out)), n_in, hidden, n_out)
    vec += 0.1 * rng.standard_normal(vec.size)        # non-zero biases too
    X = rng.standard_normal((5, n_in))
    T = rng.standard_normal((5, n_out))
    return vec, X, T, (n_in, hidden, n_out)


def test_backward_matches_central_differences():
    vec, X, T, dims = tiny()
    _, g = mlp.loss_and_grad(vec, X, T, *dims)
    h = 1e-6
    fd = np.zeros_like(vec)
    for i in range(vec.size):
        e = np.zeros_like(vec)
        e[i] = h
        fd[i] = (mlp.loss_and_grad(vec + e, X, T, *dims)[0] - mlp.loss_and_grad(vec - e, X, T, *dims)[0]) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_silu_derivative_closed_form():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    assert np.allclose(mlp.dsilu(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), atol=1e-9)


def test_adam_first_step_is_lr_times_sign():
    vec, X, T, dims = tiny(1)
    _, g = mlp.loss_and_grad(vec, X, T, *dims)
    new, m, v = mlp.adam_step(vec, g, np.zeros_like(vec), np.zeros_like(vec), 1, lr=1e-2, eps=1e-12)
    big = np.abs(g) > 1e-6
    assert np.allclose((vec - new)[big], 1e-2 * np.sign(g[big]), rtol=1e-5)


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    dims = (4, 32, 2)
    vec = mlp.init_from_normals(rng.standard_normal(mlp.n_params(*dims)), *dims)
    X = rng.uniform(-1, 1, (256, 4))
    T = np.stack([np.sin(X[:, 0] + X[:, 1]), X[:, 2] * X[:, 3]], axis=1)
    m = np.zeros_like(vec)
    v = np.zeros_like(vec)
    L0 = mlp.loss_and_grad(vec, X, T, *dims)[0]
    for t in range(1, 301):
        L, g = mlp.loss_and_grad(vec, X, T, *dims)
        vec, m, v = mlp.adam_step(vec, g, m, v, t, lr=1e-2)
    assert L < 0.1 * L0
