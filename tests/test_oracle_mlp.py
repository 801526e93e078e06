"""Pins of the FP64 warm-start network reference: gradients against central
differences, GELU against its definition, the first Adam step."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_matches_definition_and_derivative():
    z = np.linspace(-6, 6, 1001)
    # Phi via the error function's series-free relation to the normal CDF
    from scipy.stats import norm
    np.testing.assert_allclose(mlp.gelu(z), z * norm.cdf(z), rtol=1e-12, atol=1e-14)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    dims = [7, 5, 4, 6]
    params = mlp.init_params(rng, dims)
    params = [p + rng.normal(0, 0.1, p.shape) for p in params]
    X = rng.normal(size=(3, 7))
    T = rng.normal(size=(3, 6))
    loss, grads = mlp.loss_and_grads(params, X, T)
    h = 1e-6
    for k, p in enumerate(params):
        fd = np.zeros_like(p)
        for idx in np.ndindex(p.shape):
            pp = [q.copy() for q in params]
            pp[k][idx] += h
            lp, _ = mlp.loss_and_grads(pp, X, T)
            pp[k][idx] -= 2 * h
            lm, _ = mlp.loss_and_grads(pp, X, T)
            fd[idx] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(grads[k], fd, rtol=1e-6, atol=1e-9)


def test_first_adam_step_is_signed_lr():
    rng = np.random.default_rng(1)
    params = [rng.normal(size=(3, 2)), rng.normal(size=3)]
    grads = [rng.normal(size=(3, 2)), rng.normal(size=3)]
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    new, _, _ = mlp.adam_step(params, grads, m, v, 1, lr=0.01, eps=1e-12)
    for p, q, g in zip(params, new, grads):
        np.testing.assert_allclose(p - q, 0.01 * np.sign(g), rtol=1e-9)


def test_mse_loss_value():
    params = [np.eye(2), np.zeros(2), np.eye(2), np.zeros(2), np.eye(2), np.zeros(2)]
    X = np.array([[0.0, 0.0]])
    T = np.array([[1.0, -1.0]])
    loss, _ = mlp.loss_and_grads(params, X, T)
    assert loss == pytest.approx(1.0)  # Y = 0, mean of (1, 1)
