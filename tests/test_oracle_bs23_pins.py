"""Pins of the oracle's adaptive Bogacki-Shampine 3(2) integrator and its
time-weighted binning (Sec. 2.2.2, Sec. 2.2.4: each sample weighted by its
step over the total time).

Pins: a Kepler orbit against the two-body solution (Kepler's equation); the
error shrinks in proportion to the tolerance; in an axisymmetric potential
seen from a rotating frame the Jacobi energy and L_z are conserved to the
tolerance; the weighted histogram equals a recount of the trajectory's
samples through bin_points, and each block's fractions plus its overflow sum
to one.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

G = O.G


def kepler_solution(GM, r0, v0, t):
    """Position after time t on the two-body orbit from (r0, v0) (f and g
    functions with the eccentric-anomaly change from Kepler's equation)."""
    r = np.linalg.norm(r0)
    a = 1.0 / (2.0 / r - v0 @ v0 / GM)
    n = math.sqrt(GM / a ** 3)
    sig = (r0 @ v0) / math.sqrt(GM)
    M = n * t
    E = M
    for _ in range(100):
        F = E + sig / math.sqrt(a) * (1 - math.cos(E)) - (1 - r / a) * math.sin(E) - M
        dF = 1 + sig / math.sqrt(a) * math.sin(E) - (1 - r / a) * math.cos(E)
        E -= F / dF
    f = 1 - a / r * (1 - math.cos(E))
    g = t + (math.sin(E) - E) / n
    return f * r0 + g * v0


def _kepler_run(rtol, nsteps=3000):
    M = 1e10
    GM = G * M
    pot = O.make_pot([("kepler", (M,))])
    r0 = np.array([8.0, 0.0, 0.5])
    vc = math.sqrt(GM / 8.0)
    v0 = np.array([0.1 * vc, 0.8 * vc, 0.05 * vc])
    traj, dts = O.orbit_bs23(pot, np.concatenate([r0, v0]), 0.01, nsteps, rtol, rtol * 1e-2)
    assert np.all(dts > 0)
    want = kepler_solution(GM, r0, v0, dts.sum())
    return np.linalg.norm(traj[-1, :3] - want) / np.linalg.norm(want), dts.sum() * math.sqrt(GM / 8.0 ** 3) / (2 * math.pi)


def test_kepler_orbit_against_two_body_solution():
    err, periods = _kepler_run(1e-9, nsteps=10000)
    assert periods > 1.0
    assert err < 1e-6


def test_error_proportional_to_tolerance():
    """A fixed count of accepted steps covers less time at a tighter
    tolerance, so the errors are compared per orbital period (the phase
    error of a Kepler orbit grows linearly)."""
    e1, p1 = _kepler_run(1e-7)
    e2, p2 = _kepler_run(1e-9)
    assert 10.0 < (e1 / p1) / (e2 / p2) < 1000.0


def test_rotating_frame_conserves_jacobi_energy_and_lz():
    pot = O.make_pot(W.SMALL["components"], 40.0)
    ic = np.array([4.0, 1.0, 0.3, -30.0, 170.0, 20.0])
    traj, dts = O.orbit_bs23(pot, ic, 0.001, 4000, 1e-10, 1e-12)
    EJ = np.array([O.jacobi(pot, s) for s in traj])
    Lz = traj[:, 0] * traj[:, 4] - traj[:, 1] * traj[:, 3]
    assert np.abs(EJ / EJ[0] - 1).max() < 1e-7
    assert np.abs(Lz / Lz[0] - 1).max() < 1e-7


def test_weighted_histogram_is_a_recount_of_the_samples():
    cfg = W.SMALL
    pot = O.make_pot(cfg["components"], cfg["omega"])
    obs = O.make_obs(dict(cfg["obs"], surface=1, upsilon=2.0), O.euler_matrix(*cfg["euler"]))
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=300)
    ics, dt = ics[:, :5], dt[:5]
    A, ov, _, fl = O.integrate_bs23_and_bin(pot, obs, ics, dt, 300, 1e-7, 1e-9)
    assert np.all(fl == 0)
    nm, nk = obs.nx * obs.ny * obs.nz, obs.n_ap * obs.nv
    for i in range(5):
        traj, dts = O.orbit_bs23(pot, ics[:, i], dt[i], 300, 1e-7, 1e-9)
        mass, kin = O.bin_points(obs, np.ascontiguousarray(traj[1:].T))
        w = np.repeat(dts, 4) / (4 * dts.sum())
        m, k = mass.ravel(), kin.ravel()
        want_m = np.bincount(m[m >= 0], weights=w[m >= 0], minlength=nm)
        want_k = np.bincount(k[(k >= 0) & (k < nk)], weights=w[(k >= 0) & (k < nk)], minlength=nk)
        assert np.allclose(A[i, :nm], want_m, rtol=1e-12, atol=1e-15)
        assert np.allclose(A[i, nm:nm + nk], want_k, rtol=1e-12, atol=1e-15)
        assert A[i, :nm].sum() + ov[i, 0] == pytest.approx(1.0, abs=1e-12)
        assert A[i, nm:nm + nk].sum() + ov[i, 1] == pytest.approx(1.0, abs=1e-12)
