"""Pins of the aperture-jackknife oracle (Sec. 2.4; `oracle/jackknife.py`).

* One orbit: the weight problem has the closed-form solution
  w' = max(0, u.y / (u.u + mu)), so every leave-one-aperture-out chi^2 is
  known by hand; the full problem's mu must be the one used.
* Identical apertures: every jackknife problem is the same problem up to a
  relabelling of apertures, so the scatter is zero.
* Relabelling apertures permutes the chi^2 values and keeps the scatter.
* Masked orbits take no part: adding masked orbits changes nothing.
* The scatter of 0, 1, ..., n-1 is sqrt((n - 1)(n^2 - 1)/12).
"""
import math

import numpy as np
import pytest

from oracle import jackknife as J
from oracle import nnls as N


def test_scatter_closed_form():
    for n in (2, 5, 17):
        assert J.jackknife_scatter(np.arange(n, dtype=float)) == pytest.approx(math.sqrt((n - 1) * (n * n - 1) / 12))
    assert J.jackknife_scatter([3.0, 3.0, 3.0]) == 0.0


@pytest.mark.parametrize("surface", [False, True])
def test_one_orbit_closed_form(surface):
    rng = np.random.default_rng(1)
    n_mass, n_ap, nv = 3, 5, 2
    kin0 = n_mass
    surf0 = kin0 + n_ap * nv if surface else None
    nc = n_mass + n_ap * nv + (n_ap if surface else 0)
    A = rng.uniform(0.1, 1.0, size=(1, nc))
    d = rng.uniform(0.1, 1.0, size=nc)
    sig = rng.uniform(0.05, 0.2, size=nc)
    wt = 0.7
    mu = 0.3
    dchi2, chis, ws = J.jackknife(A, d, sig, wt, mu, kin0, n_ap, nv, surf0=surf0)
    u = wt * A[0] / sig
    y = d / sig
    ref = []
    for a in range(n_ap):
        drop = set(range(kin0 + a * nv, kin0 + (a + 1) * nv)) | ({surf0 + a} if surface else set())
        keep = [n for n in range(nc) if n not in drop]
        wp = max(0.0, float(u[keep] @ y[keep]) / (float(u[keep] @ u[keep]) + mu))
        assert ws[a, 0] == pytest.approx(wp * wt, rel=1e-12)
        obs = [n for n in range(kin0, nc) if n not in drop]
        ref.append(sum((u[n] * wp - y[n]) ** 2 for n in obs))
    np.testing.assert_allclose(chis, ref, rtol=1e-12)
    assert dchi2 == pytest.approx(J.jackknife_scatter(ref), rel=1e-10)


def _identical_apertures(n_orb, n_mass, n_ap, nv, seed):
    rng = np.random.default_rng(seed)
    mass = rng.uniform(0, 1, size=(n_orb, n_mass)) * (rng.random((n_orb, n_mass)) < 0.6)
    one = rng.uniform(0, 1, size=(n_orb, nv)) * (rng.random((n_orb, nv)) < 0.6)
    A = np.hstack([mass] + [one] * n_ap)
    w_true = rng.exponential(1.0, n_orb) * (rng.random(n_orb) < 0.5)
    d_one = one.T @ w_true * (1 + 0.05 * rng.normal(size=nv))
    d = np.concatenate([mass.T @ w_true, np.tile(d_one, n_ap)])
    sig = 0.05 * np.maximum(d, 1e-3 * d.max())
    return A, d, sig


def test_identical_apertures_give_zero_scatter():
    n_orb, n_mass, n_ap, nv = 20, 6, 4, 3
    A, d, sig = _identical_apertures(n_orb, n_mass, n_ap, nv, seed=2)
    wt = float(d[:n_mass].sum()) / n_orb
    U, _ = N.scale_problem(A, d, sig, wt)
    mu = N.relative_mu(U, 1e-2)
    dchi2, chis, _ = J.jackknife(A, d, sig, wt, mu, n_mass, n_ap, nv)
    assert np.ptp(chis) <= 1e-9 * chis.max()
    assert dchi2 <= 1e-8 * chis.max()
    assert chis.max() > 0


def test_relabelled_apertures_permute_the_values():
    rng = np.random.default_rng(3)
    n_orb, n_mass, n_ap, nv = 18, 5, 4, 3
    A = rng.uniform(0, 1, size=(n_orb, n_mass + n_ap * nv)) * (rng.random((n_orb, n_mass + n_ap * nv)) < 0.5)
    d = A.T @ rng.exponential(1.0, n_orb) * (1 + 0.05 * rng.normal(size=A.shape[1]))
    sig = 0.05 * np.maximum(d, 1e-3 * d.max())
    wt = float(d[:n_mass].sum()) / n_orb
    mu = N.relative_mu(N.scale_problem(A, d, sig, wt)[0], 1e-2)
    dchi2, chis, _ = J.jackknife(A, d, sig, wt, mu, n_mass, n_ap, nv)
    perm = [2, 0, 3, 1]
    cols = list(range(n_mass)) + [n_mass + p * nv + k for p in perm for k in range(nv)]
    dchi2_p, chis_p, _ = J.jackknife(A[:, cols], d[cols], sig[cols], wt, mu, n_mass, n_ap, nv)
    np.testing.assert_allclose(chis_p, chis[perm], rtol=1e-9)
    assert dchi2_p == pytest.approx(dchi2, rel=1e-9)
    assert dchi2 > 0


def test_masked_orbits_take_no_part():
    rng = np.random.default_rng(4)
    n_orb, n_mass, n_ap, nv = 16, 5, 3, 3
    nc = n_mass + n_ap * nv
    A = rng.uniform(0, 1, size=(n_orb, nc)) * (rng.random((n_orb, nc)) < 0.5)
    d = A.T @ rng.exponential(1.0, n_orb) * (1 + 0.05 * rng.normal(size=nc))
    sig = 0.05 * np.maximum(d, 1e-3 * d.max())
    wt = float(d[:n_mass].sum()) / n_orb
    mu = N.relative_mu(N.scale_problem(A, d, sig, wt)[0], 1e-2)
    base = J.jackknife(A, d, sig, wt, mu, n_mass, n_ap, nv)
    extra = rng.uniform(0, 5, size=(4, nc))
    A2 = np.vstack([A[:7], extra, A[7:]])
    mask = np.zeros(n_orb + 4, dtype=np.uint8)
    mask[7:11] = 1
    out = J.jackknife(A2, d, sig, wt, mu, n_mass, n_ap, nv, mask=mask)
    np.testing.assert_allclose(out[1], base[1], rtol=1e-10)
    assert np.all(out[2][:, 7:11] == 0)
