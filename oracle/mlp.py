"""Float64 model of the cost-model MLP -- test infrastructure only.

Not part of the paper: the learned tree selection is an addition of this
implementation.  The model, written from its definition:

    x' = (x - mu) / sigma
    h1 = relu(W1 x' + b1),  h2 = relu(W2 h1 + b2),  y = w3 . h2 + b3
    loss = mean over the batch of (y - target)^2

with parameters flat in the order W1 (H x D, row-major), b1, W2 (H x H), b2,
w3 (H), b3.  Gradients by the chain rule, one layer at a time; Adam as
published by Kingma and Ba (bias-corrected moments, beta1 0.9, beta2 0.999,
eps 1e-8).
"""
from __future__ import annotations

import numpy as np


def param_count(D: int, H: int) -> int:
    return H * D + H + H * H + H + H + 1


def unpack(p, D: int, H: int):
    p = np.asarray(p, dtype=np.float64)
    i = 0
    W1 = p[i:i + H * D].reshape(H, D); i += H * D
    b1 = p[i:i + H]; i += H
    W2 = p[i:i + H * H].reshape(H, H); i += H * H
    b2 = p[i:i + H]; i += H
    w3 = p[i:i + H]; i += H
    b3 = p[i]
    return W1, b1, W2, b2, w3, b3


def forward(p, X, mu, sigma, D: int, H: int):
    """Predictions and the intermediate values the gradient needs."""
    W1, b1, W2, b2, w3, b3 = unpack(p, D, H)
    Xn = (np.asarray(X, dtype=np.float64) - mu) / sigma
    z1 = Xn @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    y = a2 @ w3 + b3
    return y, (Xn, z1, a1, z2, a2)


def loss(p, X, t, mu, sigma, D: int, H: int) -> float:
    y, _ = forward(p, X, mu, sigma, D, H)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def loss_grad(p, X, t, mu, sigma, D: int, H: int):
    """(loss, gradient in the flat parameter order)."""
    W1, b1, W2, b2, w3, b3 = unpack(p, D, H)
    y, (Xn, z1, a1, z2, a2) = forward(p, X, mu, sigma, D, H)
    n = y.shape[0]
    r = y - np.asarray(t, dtype=np.float64)
    dy = 2.0 * r / n                       # d loss / d y
    g_w3 = a2.T @ dy
    g_b3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)      # through relu
    g_W2 = dz2.T @ a1
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    g_W1 = dz1.T @ Xn
    g_b1 = dz1.sum(axis=0)
    g = np.concatenate([g_W1.reshape(-1), g_b1, g_W2.reshape(-1), g_b2, g_w3, [g_b3]])
    return float(np.mean(r * r)), g


def adam(p, g, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
