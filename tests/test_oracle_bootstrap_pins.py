"""Pins of the bootstrap oracle (Sec. 2.3-2.4, Eq. 6) and the library's host
chi2_model against it.

chi2_model is read as -2 ln of the mean likelihood exp(-chi2_b / 2) over the
realisations.  Its pins: equal values return that value; two values a and
a + 2 ln 3 give a + 2 ln(3/2) (mean of 1 and 1/3 is 2/3); the result lies in
[chi2_min, chi2_min + 2 ln B] and approaches the upper end when one value is
far below the rest; it is symmetric and shifts with a common offset.  The
realisations leave the density block bit-identical and move the observed
maps by exactly sigma * eps.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bootstrap as BS


def test_equal_values_return_the_value():
    for B in (1, 2, 7, 100):
        assert BS.chi2_model([1234.5] * B) == pytest.approx(1234.5, rel=0, abs=1e-12)


def test_two_value_closed_form():
    a = 10.0
    assert BS.chi2_model([a, a + 2 * math.log(3.0)]) == pytest.approx(a + 2 * math.log(1.5), rel=1e-15)
    assert BS.chi2_model([a + 2 * math.log(3.0), a]) == pytest.approx(a + 2 * math.log(1.5), rel=1e-15)


def test_bounds_symmetry_and_shift():
    rng = np.random.default_rng(3)
    for _ in range(50):
        B = int(rng.integers(1, 60))
        x = 500 + 80 * rng.random(B)
        v = BS.chi2_model(x)
        assert x.min() - 1e-9 <= v <= x.min() + 2 * math.log(B) + 1e-9
        assert BS.chi2_model(rng.permutation(x)) == pytest.approx(v, rel=1e-14)
        assert BS.chi2_model(x + 37.25) == pytest.approx(v + 37.25, rel=1e-14)
    # one value far below the others: only it counts, weighted by 1/B
    assert BS.chi2_model([100.0] + [1e4] * 9) == pytest.approx(100.0 + 2 * math.log(10.0), rel=1e-14)


def test_bootstrap_data_moves_only_the_observed_maps():
    rng = np.random.default_rng(4)
    C, cb = 300, 120
    d = rng.random(C) + 0.1
    sig = 0.02 * d
    eps = W.bootstrap_eps(5, C, seed=1)
    out = BS.bootstrap_data(d, sig, eps, cb, C)
    assert out.shape == (5, C)
    assert np.array_equal(out[:, :cb], np.repeat(d[None, :cb], 5, axis=0))
    assert np.allclose((out[:, cb:] - d[None, cb:]) / sig[None, cb:], eps[:, cb:], rtol=1e-9, atol=1e-9)
    assert np.array_equal(BS.bootstrap_data(d, sig, np.zeros((2, C)), cb, C), np.repeat(d[None], 2, axis=0))


def test_library_chi2_model_matches_oracle():
    import paper_2607_00117_amd as P
    rng = np.random.default_rng(5)
    for B in (1, 3, 100):
        x = 6000 + 300 * rng.random(B)
        assert P.chi2_model(x) == pytest.approx(BS.chi2_model(x), rel=1e-14)
    with pytest.raises(P.SchwError):
        P.chi2_model([])
    with pytest.raises(P.SchwError):
        P.chi2_model([1.0, float("nan")])
