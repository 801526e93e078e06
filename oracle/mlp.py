"""FP64 reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

Not part of the paper: the learned warm start maps a load vector to initial
multipliers (mu+, mu-, lambda) for the dual ascent (Section 3.3 starts from
lambda = mu = 0).  Architecture: dense layers n_in -> h1 -> h2 -> n_out with
GELU (erf form) after the two hidden layers and a linear output, loss = mean
squared error over all outputs of a batch, Adam (Kingma and Ba, with bias
correction).  Weights are stored [out, in].

Pinned by tests/test_oracle_mlp.py: central-difference gradient checks and
the first Adam step.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) * INV_SQRT_2PI


def forward(params, X):
    """Returns (Y, cache).  params = [W1, b1, W2, b2, W3, b3]."""
    W1, b1, W2, b2, W3, b3 = params
    Z1 = X @ W1.T + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = gelu(Z2)
    Y = H2 @ W3.T + b3
    return Y, (X, Z1, H1, Z2, H2)


def loss_and_grads(params, X, T):
    """Mean squared error over the batch and every output, and its gradient
    with respect to every parameter."""
    W1, b1, W2, b2, W3, b3 = params
    Y, (X, Z1, H1, Z2, H2) = forward(params, X)
    n = Y.size
    R = Y - T
    loss = float(np.sum(R * R) / n)
    dY = 2.0 * R / n
    dW3 = dY.T @ H2
    db3 = dY.sum(0)
    dZ2 = (dY @ W3) * gelu_grad(Z2)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * gelu_grad(Z1)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(0)
    return loss, [dW1, db1, dW2, db2, dW3, db3]


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t = 1 for the first step); returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    c1 = 1.0 - beta1 ** t
    c2 = 1.0 - beta2 ** t
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = beta1 * mm + (1 - beta1) * g
        vv = beta2 * vv + (1 - beta2) * g * g
        out_p.append(p - lr * (mm / c1) / (np.sqrt(vv / c2) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


def init_params(rng, dims):
    """He-style initialisation: W ~ N(0, 2 / fan_in), b = 0."""
    params = []
    for a, b in zip(dims[:-1], dims[1:]):
        params.append(rng.normal(0.0, math.sqrt(2.0 / a), (b, a)))
        params.append(np.zeros(b))
    return params
