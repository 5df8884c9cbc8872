"""Dithered orbit bundles (Sec. 2.2.1), plain NumPy in FP64.

TEST INFRASTRUCTURE ONLY.

Each initial condition is replaced by n nearby realisations on a small box
centred on it in Cartesian phase space: positions moved by dx times a
deviate, velocities by f_v times the local circular speed v_c times a
deviate (the paper's sizes: 0.1 kpc and 5%); the deviates, uniform on
[-1/2, 1/2), are inputs.  Realisation k of initial condition i is column
i n + k, so a bundle's orbits are consecutive rows of the orbit matrix, and
the bundle enters the fit as one orbit: the mean of its rows.
"""
import numpy as np


def dither(ics, vc, u, dx, fv):
    """ics [6][N], vc [N], u [n][6][N] -> [6][N n]."""
    ics = np.asarray(ics, dtype=np.float64)
    n_d, N = u.shape[0], ics.shape[1]
    out = np.zeros((6, N * n_d))
    for i in range(N):
        for k in range(n_d):
            for c in range(6):
                scale = dx if c < 3 else fv * vc[i]
                out[c, i * n_d + k] = ics[c, i] + u[k, c, i] * scale
    return out


def bundle_rows(A, n_d):
    """Mean of each group of n_d consecutive rows, summed in row order in FP64."""
    A = np.asarray(A, dtype=np.float64)
    nb = A.shape[0] // n_d
    s = A[0::n_d][:nb].copy()
    for k in range(1, n_d):
        s = s + A[k::n_d][:nb]
    return s / n_d
