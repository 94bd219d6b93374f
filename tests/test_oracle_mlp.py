"""Pins of the cost-model MLP oracle (oracle.mlp) on the CPU: the chain-rule
gradient against central finite differences, and Adam's first step against
its closed form lr * g / (|g| + eps)."""
import numpy as np

from oracle import mlp as M

D, H = 5, 7


def _setup(seed=0, n=23):
    g = np.random.default_rng(seed)
    p = g.standard_normal(M.param_count(D, H)) * 0.5
    X = g.standard_normal((n, D)) * 3 + 1
    t = g.standard_normal(n)
    mu = X.mean(axis=0)
    sigma = X.std(axis=0) + 0.1
    return p, X, t, mu, sigma


def test_param_count():
    assert M.param_count(12, 32) == 32 * 12 + 32 + 32 * 32 + 32 + 32 + 1


def test_gradient_matches_finite_differences():
    p, X, t, mu, sigma = _setup()
    f0, g = M.loss_grad(p, X, t, mu, sigma, D, H)
    assert abs(f0 - M.loss(p, X, t, mu, sigma, D, H)) < 1e-12
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (M.loss(p + e, X, t, mu, sigma, D, H) - M.loss(p - e, X, t, mu, sigma, D, H)) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-6 * max(1.0, np.max(np.abs(g)))


def test_adam_first_step_closed_form():
    p, X, t, mu, sigma = _setup(1)
    _, g = M.loss_grad(p, X, t, mu, sigma, D, H)
    lr = 1e-2
    p1, m, v = M.adam(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_training_reduces_loss_on_a_smooth_target():
    g = np.random.default_rng(3)
    X = g.uniform(-1, 1, size=(200, D))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2
    p = g.standard_normal(M.param_count(D, H)) * 0.3
    mu, sigma = X.mean(axis=0), X.std(axis=0)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    f0 = M.loss(p, X, t, mu, sigma, D, H)
    for step in range(1, 301):
        _, gr = M.loss_grad(p, X, t, mu, sigma, D, H)
        p, m, v = M.adam(p, gr, m, v, step, 1e-2)
    assert M.loss(p, X, t, mu, sigma, D, H) < 0.1 * f0
