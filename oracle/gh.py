"""Gauss-Hermite moments of line-of-sight velocity distributions (Sec. 2.2.4, Eq. 2).

Test infrastructure only: the library computes the same linear moments on the
GPU and is checked against these functions.

Eq. 2 expands an LOSVD about a reference Gaussian of centre v0 and width s,
w = (v - v0)/s, in the modified Hermite polynomials H_m, which are
orthonormal in the sense  int alpha(w)^2 H_m H_n dw = delta_mn / (2 sqrt(pi)),
alpha(w) = exp(-w^2/2)/sqrt(2 pi).  Projecting f onto them gives the linear
moments
    g_m = 2 sqrt(pi) int f(v) alpha(w) H_m(w) dv,
so that for f = (gamma/s) alpha(w) [1 + sum_m h_m H_m(w)] one has g_0 = gamma
and g_m = gamma h_m (m >= 1).  Being linear in f, the g_m of a weighted sum of
orbits is the weighted sum of the orbits' g_m.  A velocity histogram is read
as a density that is uniform inside each bin.
"""
import math

import numpy as np


def hermite(m, w):
    """Modified Hermite polynomial H_m(w), by the three-term recurrence
    H_{m+1} = (sqrt(2) w H_m - sqrt(m) H_{m-1}) / sqrt(m+1), H_0 = 1, H_1 = sqrt(2) w."""
    w = np.asarray(w, dtype=np.float64)
    h_prev, h = np.ones_like(w), math.sqrt(2.0) * w
    if m == 0:
        return h_prev
    for k in range(1, m):
        h_prev, h = h, (math.sqrt(2.0) * w * h - math.sqrt(k) * h_prev) / math.sqrt(k + 1)
    return h


def alpha(w):
    return np.exp(-0.5 * np.asarray(w, dtype=np.float64) ** 2) / math.sqrt(2.0 * math.pi)


def bin_kernel(vlo, vhi, nv, v0, s, n_gh, nodes=64):
    """G[m][k] = 2 sqrt(pi) (1/dv) int_{bin k} alpha(w) H_m(w) dv: the moment of a unit
    mass spread uniformly over velocity bin k.  Gauss-Legendre with `nodes` points per bin."""
    x, wq = np.polynomial.legendre.leggauss(nodes)
    edges = np.linspace(vlo, vhi, nv + 1)
    a, b = edges[:-1, None], edges[1:, None]
    w = (0.5 * (b - a) * x + 0.5 * (a + b) - v0) / s  # [nv][nodes]
    G = np.zeros((n_gh + 1, nv))
    for m in range(n_gh + 1):
        G[m] = 2.0 * math.sqrt(math.pi) * 0.5 * (alpha(w) * hermite(m, w)) @ wq
    return G


def moments_from_histogram(hist, vlo, vhi, v0, s, n_gh=4, nodes=64):
    """Linear moments g_0..g_n_gh of a velocity histogram (masses per bin)."""
    hist = np.asarray(hist, dtype=np.float64)
    G = bin_kernel(vlo, vhi, hist.shape[-1], v0, s, n_gh, nodes)
    return hist @ G.T


def orbit_moments(A_kin, n_ap, nv, vlo, vhi, v0, s, n_gh=4):
    """Per-orbit, per-aperture moments of the kinematic block of an orbit matrix.
    A_kin: [N][n_ap * nv] (aperture-major cells ap * nv + v_bin); v0, s: [n_ap].
    Returns [N][n_ap][n_gh + 1]."""
    A_kin = np.asarray(A_kin, dtype=np.float64).reshape(A_kin.shape[0], n_ap, nv)
    out = np.zeros((A_kin.shape[0], n_ap, n_gh + 1))
    for a in range(n_ap):
        G = bin_kernel(vlo, vhi, nv, v0[a], s[a], n_gh)
        out[:, a, :] = A_kin[:, a, :] @ G.T
    return out


def fit_matrix(A, n_mass, kin0, surf0, n_ap, nv, vlo, vhi, v0, s, gamma, n_gh=4):
    """The stacked orbit matrix of Eq. 3 with Gauss-Hermite kinematics: the
    density block, the surface-density columns (when surf0 is not None) and the
    matrices h_{m,i,n} = g_m(i, n) / gamma_n, m = 1..n_gh (m-major), gamma_n the
    observed luminosity of aperture n (the per-orbit h_m are linear only for a
    fixed normalisation)."""
    A = np.asarray(A, dtype=np.float64)
    g = orbit_moments(A[:, kin0:kin0 + n_ap * nv], n_ap, nv, vlo, vhi, v0, s, n_gh)  # [N][n_ap][n_gh + 1]
    parts = [A[:, :n_mass]]
    if surf0 is not None:
        parts.append(A[:, surf0:surf0 + n_ap])
    gamma = np.asarray(gamma, dtype=np.float64)
    for m in range(1, n_gh + 1):
        parts.append(g[:, :, m] / gamma[None, :])
    return np.hstack(parts)
