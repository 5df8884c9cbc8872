"""The library's delayed-acceptance sampler (host control flow of
`surrogate.da_mcmc`) against the oracle's delayed-acceptance Metropolis
(Christen & Fox 2005; `oracle/mcmc.py`) driven by the same normals and
uniforms: identical chains and identical counters of expensive evaluations
and stage-1 passes.  The expensive chi^2 and the screen are toy functions on
the host (a quadratic chi^2 and a biased, tilted copy), so no GPU is needed;
the prior is the uniform box of the sampler (outside it both densities are 0).
"""
import numpy as np
import pytest

from oracle import mcmc
from paper_2607_00117_amd import surrogate as S

D = 12
LO, HI = -np.ones(D), 2.0 * np.ones(D)
CENTRE = np.linspace(0.1, 0.9, D)


class ToyBuilder:
    def __init__(self):
        self.calls = 0

    def chi2(self, thetas):
        t = np.atleast_2d(thetas)
        self.calls += len(t)
        return 40.0 * np.sum((t - CENTRE) ** 2, axis=1) + 100.0


class ToySurrogate:
    def predict(self, thetas):
        t = np.atleast_2d(thetas)
        return 30.0 * np.sum((t - CENTRE - 0.15) ** 2, axis=1) + 5.0 * t[:, 0] + 90.0


def _inside(t):
    return bool(np.all((t >= LO) & (t <= HI)))


def _logp(dchi2, f):
    def lp(t):
        return -f(np.asarray(t)[None, :])[0] / dchi2 if _inside(t) else -np.inf
    return lp


@pytest.mark.parametrize("dchi2", [3.0, 25.0])
def test_da_mcmc_matches_oracle_delayed_acceptance(dchi2):
    n_w, n_steps, step_frac = 6, 400, 0.08
    rng = np.random.default_rng(5)
    normals = rng.normal(size=(n_steps, n_w, D))
    uniforms = rng.uniform(size=(n_steps, n_w, 2))
    theta0 = CENTRE + rng.normal(scale=0.2, size=(n_w, D))
    b, s = ToyBuilder(), ToySurrogate()
    res = S.da_mcmc(b, s, theta0, LO, HI, n_steps, dchi2, step_frac=step_frac, use_surrogate=True,
                    normals=normals, uniforms=uniforms)
    chol = np.diag(step_frac * (HI - LO))
    n_eval, n_s1 = 0, 0
    for i in range(n_w):
        chain, ne, ns = mcmc.da_mh(_logp(dchi2, b.chi2), _logp(dchi2, s.predict), theta0[i], chol, normals[:, i],
                                   uniforms[:, i])
        np.testing.assert_array_equal(res["chains"][:, i], chain)
        n_eval += ne
        n_s1 += ns
    assert res["n_full_builds"] == n_eval
    assert res["n_stage1"] == n_s1
    assert 0 < res["n_accepted"] < n_steps * n_w and res["n_stage1"] < n_steps * n_w


def test_plain_chain_matches_oracle_metropolis():
    n_w, n_steps, step_frac, dchi2 = 5, 300, 0.08, 10.0
    rng = np.random.default_rng(6)
    normals = rng.normal(size=(n_steps, n_w, D))
    uniforms = rng.uniform(size=(n_steps, n_w, 2))
    theta0 = CENTRE + rng.normal(scale=0.2, size=(n_w, D))
    b = ToyBuilder()
    res = S.da_mcmc(b, None, theta0, LO, HI, n_steps, dchi2, step_frac=step_frac, use_surrogate=False,
                    normals=normals, uniforms=uniforms)
    chol = np.diag(step_frac * (HI - LO))
    for i in range(n_w):
        chain, _ = mcmc.mh(_logp(dchi2, b.chi2), theta0[i], chol, normals[:, i], uniforms[:, i])
        np.testing.assert_array_equal(res["chains"][:, i], chain)


def test_exact_screen_passes_every_inside_proposal_to_the_full_build():
    """With the screen equal to the full chi^2 the second stage always accepts
    what the first passed: delayed acceptance is then Metropolis with the screen."""
    n_w, n_steps, step_frac, dchi2 = 4, 200, 0.08, 8.0
    rng = np.random.default_rng(7)
    normals = rng.normal(size=(n_steps, n_w, D))
    uniforms = rng.uniform(size=(n_steps, n_w, 2))
    theta0 = CENTRE + rng.normal(scale=0.2, size=(n_w, D))
    b = ToyBuilder()

    class Exact:
        def predict(self, t):
            return b.chi2(t)

    res = S.da_mcmc(b, Exact(), theta0, LO, HI, n_steps, dchi2, step_frac=step_frac, use_surrogate=True,
                    normals=normals, uniforms=uniforms)
    assert res["n_accepted"] == res["n_stage1"]


def test_adapted_screen_then_exact_delayed_acceptance():
    """With the screen refitted during the first adapt_steps steps (here a toy
    refit that changes its bias), the chain after adaptation is the oracle's
    delayed-acceptance chain with the final screen, started from the state
    reached at adapt_steps, on the same random numbers."""
    n_w, n_steps, adapt, step_frac, dchi2 = 4, 300, 100, 0.08, 10.0
    rng = np.random.default_rng(9)
    normals = rng.normal(size=(n_steps, n_w, D))
    uniforms = rng.uniform(size=(n_steps, n_w, 2))
    theta0 = CENTRE + rng.normal(scale=0.2, size=(n_w, D))
    b = ToyBuilder()

    class Adaptive:
        bias = 0.0

        def predict(self, t):
            t = np.atleast_2d(t)
            return 30.0 * np.sum((t - CENTRE - self.bias) ** 2, axis=1) + 90.0

    s = Adaptive()
    calls = []

    def refit(th, chi):
        calls.append(len(chi))
        s.bias = 0.1 / len(calls)

    res = S.da_mcmc(b, s, theta0, LO, HI, n_steps, dchi2, step_frac=step_frac, use_surrogate=True,
                    normals=normals, uniforms=uniforms, refit=refit, refit_every=25, adapt_steps=adapt)
    assert len(calls) == 3 and calls == sorted(calls)
    chol = np.diag(step_frac * (HI - LO))
    start = res["chains"][adapt - 1]
    n_eval, n_s1 = 0, 0
    for i in range(n_w):
        chain, ne, ns = mcmc.da_mh(_logp(dchi2, b.chi2), _logp(dchi2, s.predict), start[i], chol,
                                   normals[adapt:, i], uniforms[adapt:, i])
        np.testing.assert_array_equal(res["chains"][adapt:, i], chain)
        n_eval += ne - 1
        n_s1 += ns
    assert res["n_full_builds_after_adapt"] == n_eval
    assert res["n_stage1_after_adapt"] == n_s1
