"""Regularised NNLS oracle (Eq. 3-4) and chi^2 (Eq. 5), plain NumPy in FP64.

TEST INFRASTRUCTURE ONLY.

The weight problem of Eq. 4 is
    minimise  Q(w) = 1/2 ||U w - y||^2 + (lambda / N) ||w||^2   subject to w >= 0,
i.e. with mu = 2 lambda / N the strictly convex quadratic programme
    minimise  1/2 w^T H w - c^T w,  H = U^T U + mu I,  c = U^T y,  w >= 0.
Because it is strictly convex for mu > 0 its minimiser is unique, so any
exact method defines the answer; the paper's ADMM (Sec. 2.3) is one route to
it.  Here the answer is computed by brute-force support enumeration (tiny
problems) or by the Lawson-Hanson active-set method (Lawson & Hanson 1974,
ch. 23) applied to the normal equations, and certified by the KKT conditions
    w >= 0,  g = H w - c >= 0,  w_i g_i = 0.
"""
import itertools
import math

import numpy as np


def objective(U, y, mu, w):
    r = U @ w - y
    return 0.5 * float(r @ r) + 0.5 * mu * float(w @ w)


def gradient(U, y, mu, w):
    return U.T @ (U @ w - y) + mu * w


def kkt_residual(U, y, mu, w):
    """Natural residual ||min(w, g)||_inf; zero exactly at the optimum."""
    g = gradient(U, y, mu, w)
    return float(np.max(np.abs(np.minimum(w, g)))) if w.size else 0.0


def nnls_bruteforce(U, y, mu):
    """Enumerates every support S: w_S solves the normal equations restricted
    to S, and is accepted when w_S > 0 and the gradient outside S is >= 0."""
    n = U.shape[1]
    H = U.T @ U + mu * np.eye(n)
    c = U.T @ y
    best = None
    for k in range(n + 1):
        for S in itertools.combinations(range(n), k):
            S = list(S)
            w = np.zeros(n)
            if S:
                w[S] = np.linalg.solve(H[np.ix_(S, S)], c[S])
                if np.any(w[S] <= 0):
                    continue
            g = H @ w - c
            out = [j for j in range(n) if j not in S]
            if out and np.any(g[out] < -1e-12 * (1 + np.abs(c).max())):
                continue
            if best is None or objective(U, y, mu, w) < objective(U, y, mu, best):
                best = w
    return best


def nnls_active_set(H, c, max_outer=None, tol=None, start=None):
    """Lawson-Hanson active set for min 1/2 w^T H w - c^T w, w >= 0 (H SPD).

    start: optional initial passive set.  It is first reduced to a feasible
    point (indices whose restricted solution is not positive are dropped), from
    which the standard outer loop continues; the optimum it reaches is the same
    unique minimiser.
    """
    n = H.shape[0]
    if tol is None:
        tol = 1e-13 * max(1.0, float(np.abs(c).max()))
    w = np.zeros(n)
    P = np.zeros(n, dtype=bool)
    if start is not None:
        # feasible warm start: drop indices whose restricted solution is not
        # positive until it is (any feasible w with w_P > 0 may seed the loop)
        P[np.asarray(start, dtype=int)] = True
        for _ in range(n + 1):
            idx = np.flatnonzero(P)
            if idx.size == 0:
                break
            s = np.linalg.solve(H[np.ix_(idx, idx)], c[idx])
            if np.min(s) > 0:
                w[idx] = s
                break
            P[idx[s <= 0]] = False
    max_outer = max_outer or 10 * n + 10
    for _ in range(max_outer):
        g = c - H @ w  # minus the gradient
        Z = ~P
        if not np.any(Z) or np.max(g[Z]) <= tol:
            break
        j = int(np.argmax(np.where(Z, g, -np.inf)))
        P[j] = True
        while True:
            idx = np.flatnonzero(P)
            s = np.zeros(n)
            s[idx] = np.linalg.solve(H[np.ix_(idx, idx)], c[idx])
            if np.min(s[idx]) > 0:
                w = s
                break
            neg = idx[s[idx] <= 0]
            alpha = np.min(w[neg] / (w[neg] - s[neg]))
            w = w + alpha * (s - w)
            P &= w > 0
            w[~P] = 0.0
    return w


def nnls_oracle(U, y, mu):
    """Exact minimiser of Eq. 4 (brute force for n <= 12, else active set
    started from the positive part of the unconstrained ridge solution)."""
    n = U.shape[1]
    if n <= 12:
        return nnls_bruteforce(U, y, mu)
    H = U.T @ U + mu * np.eye(n)
    c = U.T @ y
    ridge = np.linalg.solve(H, c)
    return nnls_active_set(H, c, start=np.flatnonzero(ridge > 0))


def scale_problem(A, d, sigma, w_tilde):
    """Eq. 3 -> Eq. 4: U[n, i] = w_tilde A[i, n] / sigma_n, y_n = d_n / sigma_n,
    solved for the dimensionless w' = w / w_tilde."""
    U = (A * w_tilde).T / sigma[:, None]
    y = d / sigma
    return U, y


def relative_mu(U, nu):
    """Reading of the unspecified regularisation strength: 2 lambda / N =
    nu * mean_i ||U[:, i]||^2."""
    return nu * float(np.mean(np.sum(U * U, axis=0)))


def _square(A):
    return A.multiply(A) if hasattr(A, "multiply") else A * A


def relative_mu_orbit_matrix(A, sigma, w_tilde, nu):
    """relative_mu without forming U, for an orbit-major A[i][n] (dense, or a
    scipy sparse matrix): ||U[:, i]||^2 = w_tilde^2 sum_n A[i][n]^2 / sigma_n^2."""
    col = (w_tilde * w_tilde) * np.asarray(_square(A) @ (1.0 / (sigma * sigma))).ravel()
    return nu * float(np.mean(col))


def kkt_residual_orbit_matrix(A, d, sigma, w_tilde, mu, w):
    """kkt_residual of Eq. 4 relative to ||U^T y||_inf, for the physical weights
    w = w_tilde w' and an orbit-major A[i][n] (dense, or a scipy sparse matrix),
    without forming U: U w' = (A^T w) / sigma and U^T e = w_tilde A (e / sigma)."""
    wp = np.asarray(w, dtype=np.float64) / w_tilde
    e = (np.asarray(A.T @ w).ravel() - d) / sigma
    g = w_tilde * np.asarray(A @ (e / sigma)).ravel() + mu * wp
    q = w_tilde * np.asarray(A @ (d / (sigma * sigma))).ravel()
    return float(np.max(np.abs(np.minimum(wp, g)))) / float(np.max(np.abs(q)))


def sigma_from_data(d, blocks, tol, floor=1e-3):
    """Per-constraint uncertainty: a relative tolerance (1% in Eq. 3) with a
    floor of `floor` times the block maximum for empty cells."""
    s = np.empty_like(d)
    for b0, b1 in blocks:
        blk = d[b0:b1]
        top = float(np.max(blk)) if blk.size else 0.0
        s[b0:b1] = tol * np.maximum(blk, floor * top)
    s[s <= 0] = tol * floor
    return s


def w_tilde_from_data(d, mass_block, n_orb):
    """Equal orbit weight: total target mass in the 3D grid over N_orb."""
    b0, b1 = mass_block
    return float(np.sum(d[b0:b1])) / n_orb


def chi2(A, w, d, sigma, col_begin, col_end):
    """Eq. 5 over constraints [col_begin, col_end): sum ((A^T w - d) / sigma)^2,
    summed with exact rounding (math.fsum)."""
    m = A[:, col_begin:col_end].T @ w
    r = (m - d[col_begin:col_end]) / sigma[col_begin:col_end]
    return math.fsum((r * r).tolist())
