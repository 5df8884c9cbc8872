"""Pins of the Gauss-Hermite oracle (Eq. 2) against closed forms of Gaussian
LOSVDs, derived from the definition of the linear moments
g_m = 2 sqrt(pi) int f alpha(w) H_m(w) dv.  For a Gaussian of mean v0 + d s and
width r s, with w = (v - v0)/s:
  shifted (r = 1):  g_0 = exp(-d^2/4), h_1 = g_1/g_0 = d/sqrt(2), h_2 = d^2/(2 sqrt(2))
  scaled  (d = 0):  g_0 = sqrt(2/(1 + r^2)), h_1 = 0, h_2 = (r^2 - 1)/(sqrt(2)(r^2 + 1)), h_3 = 0
and the matched Gaussian (d = 0, r = 1) has g = (1, 0, 0, 0, 0).  Small offsets
reproduce the paper's propagation Delta h_1 = Delta V/(sqrt 2 s),
Delta h_2 = Delta sigma/(sqrt 2 s)."""
import math

import numpy as np
import pytest

from oracle import gh


def gaussian_hist(mu, sig, vlo, vhi, nv):
    """Exact masses of N(mu, sig) in the bins (normal CDF differences)."""
    from scipy.special import ndtr
    e = np.linspace(vlo, vhi, nv + 1)
    return np.diff(ndtr((e - mu) / sig))


def test_hermite_orthonormality():
    x, wq = np.polynomial.hermite.hermgauss(40)  # weight exp(-x^2)
    for m in range(6):
        for n in range(6):
            val = np.sum(wq * gh.hermite(m, x) * gh.hermite(n, x)) / (2 * math.pi)  # int alpha^2 H_m H_n
            assert val == pytest.approx((1.0 if m == n else 0.0) / (2 * math.sqrt(math.pi)), abs=1e-13)


def test_matched_gaussian_has_no_higher_moments():
    g = gh.moments_from_histogram(gaussian_hist(10.0, 80.0, -1000, 1000, 2000), -1000, 1000, 10.0, 80.0)
    assert g[0] == pytest.approx(1.0, abs=1e-5)
    assert np.max(np.abs(g[1:])) < 1e-5


def closed_form(d, r):
    """Moments of N(v0 + d s, r s) about the reference (v0, s): with c = 1 + 1/r^2 and
    mu = d/(r^2 + 1) the Gaussian-weighted w has mean mu and variance 1/c, so
    g_0 = sqrt(2/(1 + r^2)) exp(-d^2/(2(1 + r^2))), h_1 = sqrt(2) mu, h_2 = (2 mu^2 + 2/c - 1)/sqrt(2)."""
    c, mu = 1 + 1 / (r * r), d / (r * r + 1)
    g0 = math.sqrt(2 / (1 + r * r)) * math.exp(-d * d / (2 * (1 + r * r)))
    return g0, math.sqrt(2) * mu, (2 * mu * mu + 2 / c - 1) / math.sqrt(2)


@pytest.mark.parametrize("d", [0.05, 0.4, 1.3])
def test_shifted_gaussian_closed_form(d):
    # bins of s/6700: reading the histogram as uniform within bins costs ~1e-9 here
    s, v0, nv = 60.0, -20.0, 200000
    g = gh.moments_from_histogram(gaussian_hist(v0 + d * s, s, -900, 900, nv), -900, 900, v0, s, nodes=6)
    g0, h1, h2 = closed_form(d, 1.0)
    assert d * d / (2 * math.sqrt(2)) == pytest.approx(h2, rel=1e-14)
    assert g[0] == pytest.approx(g0, rel=1e-8)
    assert g[1] / g[0] == pytest.approx(h1, rel=1e-7)
    assert g[2] / g[0] == pytest.approx(h2, rel=1e-5)


@pytest.mark.parametrize("r", [0.7, 1.05, 1.6])
def test_scaled_gaussian_closed_form(r):
    s, v0, nv = 50.0, 5.0, 200000
    g = gh.moments_from_histogram(gaussian_hist(v0, r * s, -900, 900, nv), -900, 900, v0, s, nodes=6)
    g0, h1, h2 = closed_form(0.0, r)
    assert g[0] == pytest.approx(g0, rel=1e-8)
    assert abs(g[1] / g[0]) < 1e-9 and abs(g[3] / g[0]) < 1e-9
    assert g[2] / g[0] == pytest.approx(h2, rel=1e-5)


def test_small_offset_propagation_matches_paper():
    s = 100.0
    dv, dsig = 5.0, 5.0
    g = gh.moments_from_histogram(gaussian_hist(dv, s, -1500, 1500, 3000), -1500, 1500, 0.0, s)
    assert g[1] / g[0] == pytest.approx(dv / (math.sqrt(2) * s), rel=1e-3)
    g = gh.moments_from_histogram(gaussian_hist(0.0, s + dsig, -1500, 1500, 3000), -1500, 1500, 0.0, s)
    assert g[2] / g[0] == pytest.approx(dsig / (math.sqrt(2) * s), rel=0.05)


def test_moments_are_linear_in_the_histogram():
    rng = np.random.default_rng(3)
    h1, h2 = rng.uniform(size=30), rng.uniform(size=30)
    a = gh.moments_from_histogram(2.0 * h1 + 3.0 * h2, -450, 450, 12.0, 90.0)
    b = 2.0 * gh.moments_from_histogram(h1, -450, 450, 12.0, 90.0) + 3.0 * gh.moments_from_histogram(
        h2, -450, 450, 12.0, 90.0)
    assert np.allclose(a, b, rtol=1e-13, atol=1e-15)


def test_fit_matrix_blocks_and_linearity():
    """The fit matrix of Eq. 3: the density and surface columns are copies of
    the orbit matrix's; the h-block summed over orbits with their weights is the
    h_m of the summed histogram for the observed luminosity: a Gaussian LOSVD
    shifted by d = 0.4 s from the reference, split at random over three orbits,
    gives h_m = exp(-d^2/4) (d/sqrt(2))^m / sqrt(m!) (to the binning error)."""
    from scipy.stats import norm
    n_mass, n_ap, nv = 3, 2, 300
    vlo, vhi, v0, s, d = -600.0, 600.0, 10.0, 80.0, 0.4
    edges = np.linspace(vlo, vhi, nv + 1)
    hist = np.diff(norm.cdf((edges - (v0 + d * s)) / s))  # unit luminosity
    rng = np.random.default_rng(3)
    split = rng.dirichlet(np.ones(3), size=nv).T  # [3 orbits][nv], columns sum to 1
    lum = np.array([2.0, 0.5])
    A = np.zeros((3, n_mass + n_ap * nv + n_ap))
    A[:, :n_mass] = rng.uniform(size=(3, n_mass))
    for a in range(n_ap):
        A[:, n_mass + a * nv:n_mass + (a + 1) * nv] = lum[a] * split * hist
    surf0 = n_mass + n_ap * nv
    A[:, surf0:] = rng.uniform(size=(3, n_ap))
    F = gh.fit_matrix(A, n_mass, n_mass, surf0, n_ap, nv, vlo, vhi, [v0] * n_ap, [s] * n_ap, lum, n_gh=4)
    assert F.shape == (3, n_mass + n_ap + 4 * n_ap)
    np.testing.assert_array_equal(F[:, :n_mass], A[:, :n_mass])
    np.testing.assert_array_equal(F[:, n_mass:n_mass + n_ap], A[:, surf0:])
    h = F[:, n_mass + n_ap:].sum(0).reshape(4, n_ap)
    for m in range(1, 5):
        ref = math.exp(-d * d / 4) * (d / math.sqrt(2)) ** m / math.sqrt(math.factorial(m))
        np.testing.assert_allclose(h[m - 1], ref, atol=2e-4)
    F2 = gh.fit_matrix(A, n_mass, n_mass, None, n_ap, nv, vlo, vhi, [v0] * n_ap, [s] * n_ap, lum, n_gh=2)
    assert F2.shape == (3, n_mass + 2 * n_ap)
    np.testing.assert_allclose(F2[:, n_mass:], F[:, n_mass + n_ap:n_mass + 3 * n_ap], rtol=1e-13)
