"""Aperture jackknife of chi^2 (Sec. 2.4), plain NumPy in FP64.

TEST INFRASTRUCTURE ONLY.

Sec. 2.4 sets the likelihood scale Delta chi^2 of Eq. 7 by solving the weights
once per aperture with that aperture's data left out and taking the scatter of
the resulting chi^2 values.  Reading used here:
  * the data of aperture a are its nv line-of-sight-velocity constraints of the
    kinematic block and, when the orbit matrix has the surface-density block,
    its surface-density column; the intrinsic density block is never left out;
  * solve a is the weight problem of Eq. 4 on the remaining constraints, with
    the regularisation strength mu = 2 lambda / N of the full problem held
    fixed, so that leaving data out changes only the data term; masked orbits
    (quality-cut ones) take no part and get weight 0;
  * chi^2_a is Eq. 5 of solve a's weights over the observational constraints
    (kinematic and surface-density columns) that solve a kept;
  * the scatter is the jackknife standard deviation
        Delta chi^2 = sqrt((N_ap - 1) / N_ap * sum_a (chi^2_a - mean chi^2)^2).
Each solve is the exact minimiser `nnls.nnls_oracle`.
"""
import math

import numpy as np

from . import nnls


def aperture_columns(kin0, nv, a, surf0=None):
    """Constraint indices holding aperture a's data."""
    cols = list(range(kin0 + a * nv, kin0 + (a + 1) * nv))
    if surf0 is not None:
        cols.append(surf0 + a)
    return cols


def observational_columns(kin0, n_ap, nv, surf0=None):
    cols = list(range(kin0, kin0 + n_ap * nv))
    if surf0 is not None:
        cols += list(range(surf0, surf0 + n_ap))
    return cols


def jackknife_scatter(chis):
    """sqrt((n - 1)/n sum (x - mean)^2), the jackknife standard deviation."""
    x = np.asarray(chis, dtype=np.float64)
    n = x.size
    m = math.fsum(x.tolist()) / n
    return math.sqrt((n - 1) / n * math.fsum(((x - m) ** 2).tolist()))


def jackknife(A, d, sigma, w_tilde, mu, kin0, n_ap, nv, surf0=None, mask=None):
    """A: orbit matrix [N][C] (orbit-major); d, sigma: [C]; w_tilde: equal
    weight; mu: 2 lambda / N of the full problem (scaled variables).
    Returns (Delta chi^2, chi^2_a [n_ap], weights [n_ap][N] physical)."""
    A = np.asarray(A, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    n_orb, n_con = A.shape
    rows = np.arange(n_orb) if mask is None else np.flatnonzero(np.asarray(mask) == 0)
    obs = observational_columns(kin0, n_ap, nv, surf0)
    chis, ws = [], []
    for a in range(n_ap):
        drop = set(aperture_columns(kin0, nv, a, surf0))
        keep = np.array([n for n in range(n_con) if n not in drop])
        U, y = nnls.scale_problem(A[np.ix_(rows, keep)], d[keep], sigma[keep], w_tilde)
        wp = nnls.nnls_oracle(U, y, mu)
        w = np.zeros(n_orb)
        w[rows] = wp * w_tilde
        kept_obs = [n for n in obs if n not in drop]
        m = A[:, kept_obs].T @ w
        r = (m - d[kept_obs]) / sigma[kept_obs]
        chis.append(math.fsum((r * r).tolist()))
        ws.append(w)
    chis = np.array(chis)
    return jackknife_scatter(chis), chis, np.array(ws)
