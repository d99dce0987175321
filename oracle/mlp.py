"""Oracle of the surrogate network: FP64 multilayer perceptron
x (in) -> H -> H -> out with SiLU activations, mean-squared error, a
hand-derived backward pass (no autograd) and the Adam update (Kingma & Ba,
2015).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Parameter vector layout (shared convention with the library, both written
from this description): W1 [H][in], b1 [H], W2 [H][H], b2 [H], W3 [out][H],
b3 [out], concatenated in that order, weights row-major.  Initialisation from
standard normal deviates z (same layout): W = z / sqrt(fan_in), b = 0.
"""
from __future__ import annotations

import numpy as np


def shapes(n_in: int, hidden: int, n_out: int):
    return [(hidden, n_in), (hidden,), (hidden, hidden), (hidden,), (n_out, hidden), (n_out,)]


def n_params(n_in, hidden, n_out) -> int:
    return sum(int(np.prod(s)) for s in shapes(n_in, hidden, n_out))


def unpack(vec: np.ndarray, n_in, hidden, n_out):
    out, o = [], 0
    for s in shapes(n_in, hidden, n_out):
        k = int(np.prod(s))
        out.append(vec[o:o + k].reshape(s))
        o += k
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def init_from_normals(z: np.ndarray, n_in, hidden, n_out) -> np.ndarray:
    parts = unpack(np.asarray(z, dtype=np.float64), n_in, hidden, n_out)
    W1, _, W2, _, W3, _ = parts
    return pack([W1 / np.sqrt(n_in), np.zeros(hidden), W2 / np.sqrt(hidden), np.zeros(hidden),
                 W3 / np.sqrt(hidden), np.zeros(n_out)])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(vec, X, n_in, hidden, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(vec, n_in, hidden, n_out)
    Z1 = X @ W1.T + b1
    H1 = silu(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = silu(Z2)
    Y = H2 @ W3.T + b3
    return Y, (X, Z1, H1, Z2, H2)


def loss_and_grad(vec, X, T, n_in, hidden, n_out):
    """L = sum (Y - T)^2 / (B * out) and dL/dparams by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unpack(vec, n_in, hidden, n_out)
    Y, (X, Z1, H1, Z2, H2) = forward(vec, X, n_in, hidden, n_out)
    B = X.shape[0]
    R = Y - T
    L = float(np.sum(R * R) / (B * n_out))
    dY = 2.0 * R / (B * n_out)
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * dsilu(Z2)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * dsilu(Z1)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(axis=0)
    return L, pack([dW1, db1, dW2, db2, dW3, db3])


def adam_step(vec, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (vec, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return vec - lr * mhat / (np.sqrt(vhat) + eps), m, v
