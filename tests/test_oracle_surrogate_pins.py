"""Pins of the surrogate and sampler oracles: analytic backpropagation against
central differences, Adam's first step against its closed form,
delayed acceptance with an exact screen against plain Metropolis-Hastings on
the same random numbers, and the invariance of delayed acceptance with a
biased screen on a 12-D Gaussian."""
import numpy as np
import pytest

from oracle import mcmc as M
from oracle import mlp as L


def test_backprop_matches_central_differences():
    rng = np.random.default_rng(0)
    p = L.init(1)
    x = rng.uniform(-1, 1, size=(7, 12))
    dy = rng.normal(size=7)
    y, cache = L.forward(p, x)
    g = L.backward(p, cache, dy)
    idx = np.concatenate([rng.choice(L.N_PARAM - 257, 40, replace=False), np.arange(L.N_PARAM - 257, L.N_PARAM, 37),
                          [L.N_PARAM - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (np.dot(dy, L.forward(p + e, x)[0]) - np.dot(dy, L.forward(p - e, x)[0])) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    q, m, v = L.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # after bias correction the first step is lr * g / (|g| + eps)
    assert np.allclose(q, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_delayed_acceptance_with_exact_screen_is_mh():
    rng = np.random.default_rng(3)
    logp = lambda t: -0.5 * float(t @ t)  # noqa: E731
    normals = rng.normal(size=(3000, 12))
    unif = rng.uniform(size=(3000, 2))
    chol = 0.4 * np.eye(12)
    a, _ = M.mh(logp, np.zeros(12), chol, normals, unif)
    b, n_eval, _ = M.da_mh(logp, logp, np.zeros(12), chol, normals, unif)
    assert np.array_equal(a, b)


def test_delayed_acceptance_biased_screen_keeps_target():
    """pi = N(0, I_12); screen pi~ = N(0.3, 1.3^2 I): DA chain moments match pi."""
    rng = np.random.default_rng(4)
    logp = lambda t: -0.5 * float(t @ t)  # noqa: E731
    logs = lambda t: -0.5 * float(((t - 0.3) / 1.3) @ ((t - 0.3) / 1.3))  # noqa: E731
    n = 60000
    chain, n_eval, n_s1 = M.da_mh(logp, logs, np.zeros(12), 0.5 * np.eye(12), rng.normal(size=(n, 12)),
                                  rng.uniform(size=(n, 2)))
    burn = chain[5000:]
    # integrated autocorrelation of this random walk is O(50) steps: ~1000 effective samples
    assert np.all(np.abs(burn.mean(0)) < 0.15)
    assert np.all(np.abs(burn.var(0) - 1.0) < 0.25)
    assert n_eval < n  # the screen removed expensive evaluations
