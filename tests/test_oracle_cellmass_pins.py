"""Pins of the oracle's target cell masses m*_n (Sec. 2.2.4: the stellar mass
of the model density in each cell of the self-consistency grid).

The cell integrals use the oracle's densities; the pins use its forces:
Gauss's theorem makes the mass inside a closed surface equal to
-(1 / 4 pi G) times the flux of the acceleration through it, so the sum of
the cells of a grid must equal a surface integral of the force over the
grid's outer boundary (a cylinder, or a box).  The forces are pinned
separately (finite differences of the potential, closed forms), so a dropped
term in a density, a wrong Jacobian or a misplaced cell edge fails here.
Further pins: a grid that encloses the whole Ferrers bar holds its mass M
exactly, its eight octants hold M/8 each, and the sectors of an
axisymmetric model's ring hold equal masses.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O

G = O.G


def _spec(nx, ny, nz, lo, hi, grid):
    return dict(nx=nx, ny=ny, nz=nz, lo=lo, hi=hi, npx=1, npy=1, plo=(-1, -1), phi=(1, 1), nv=1, vlo=-1, vhi=1,
                symmetrize=1, drift_every=0, grid=grid)


def _cyl_flux_mass(pot, Rmax, Z):
    """Mass inside R < Rmax, |z| < Z of an axisymmetric model from the flux
    of its force through the cylinder's side, top and bottom."""
    def gx(x, z):
        return O.accel(pot, np.array([x, 0.0, z]))

    side = integrate.quad(lambda z: gx(Rmax, z)[0], -Z, Z, epsabs=0, epsrel=1e-12, limit=200)[0] * 2 * math.pi * Rmax
    top = integrate.quad(lambda R: gx(R, Z)[2] * R, 0, Rmax, epsabs=0, epsrel=1e-12, limit=200)[0] * 2 * math.pi
    bot = integrate.quad(lambda R: -gx(R, -Z)[2] * R, 0, Rmax, epsabs=0, epsrel=1e-12, limit=200)[0] * 2 * math.pi
    return -(side + top + bot) / (4 * math.pi * G)


def _box_flux_mass(pot, lo, hi, nq=48):
    """Mass inside the box [lo, hi] from the flux through its six faces
    (tensor Gauss-Legendre with nq x nq nodes per face)."""
    t, w = np.polynomial.legendre.leggauss(nq)
    total = 0.0
    for d in range(3):
        e, f = [k for k in range(3) if k != d]
        ue = 0.5 * (hi[e] - lo[e]) * t + 0.5 * (hi[e] + lo[e])
        uf = 0.5 * (hi[f] - lo[f]) * t + 0.5 * (hi[f] + lo[f])
        jac = 0.25 * (hi[e] - lo[e]) * (hi[f] - lo[f])
        for side, sgn in ((hi[d], 1.0), (lo[d], -1.0)):
            s = 0.0
            for i in range(nq):
                for j in range(nq):
                    x = np.zeros(3)
                    x[d], x[e], x[f] = side, ue[i], uf[j]
                    s += w[i] * w[j] * O.accel(pot, x)[d]
            total += sgn * s * jac
    return -total / (4 * math.pi * G)


@pytest.mark.parametrize("comp", [("mn", (5e10, 3.0, 0.3)), ("plummer", (1e10, 0.5)), ("isochrone", (2e10, 1.0)),
                                  ("nfw_q", (1e12, 10.0, 1.0, 70.0))], ids=lambda c: c[0])
def test_cylindrical_grid_total_is_gauss_flux(comp):
    pot = O.make_pot([comp])
    spec = _spec(4, 3, 4, (0.0, -math.pi, -3.0), (10.0, math.pi, 3.0), "cylindrical")
    m = O.cell_masses(pot, O.make_obs(spec, np.eye(3)), rel_tol=1e-8, abs_tol=1e-12 * comp[1][0])
    want = _cyl_flux_mass(pot, 10.0, 3.0)
    assert m.sum() == pytest.approx(want, rel=1e-8)


def test_axisymmetric_sectors_hold_equal_masses():
    pot = O.make_pot([("mn", (5e10, 3.0, 0.3)), ("plummer", (1e10, 0.5))])
    spec = _spec(3, 6, 2, (0.0, -math.pi, -3.0), (9.0, math.pi, 3.0), "cylindrical")
    m = O.cell_masses(pot, O.make_obs(spec, np.eye(3)), rel_tol=1e-10, abs_tol=1e-3).reshape(3, 6, 2)
    assert np.allclose(m, m[:, :1, :], rtol=1e-9, atol=0)
    assert np.allclose(m[:, :, 0], m[:, :, 1], rtol=1e-9, atol=0)  # z-reflection


def test_ferrers_bar_enclosed_mass_and_octants():
    M = 1e10
    pot = O.make_pot([("ferrers2", (M, 4.0, 1.5, 1.0))])
    m = O.cell_masses(pot, O.make_obs(_spec(2, 2, 2, (-4.5, -2.0, -1.5), (4.5, 2.0, 1.5), "cartesian"), np.eye(3)),
                      rel_tol=1e-8, abs_tol=1e-2)
    assert m.sum() == pytest.approx(M, rel=1e-9)
    assert np.allclose(m, M / 8, rtol=1e-9, atol=0)


def test_ferrers_bar_cut_by_the_grid_is_gauss_flux():
    pot = O.make_pot([("ferrers2", (1e10, 4.0, 1.5, 1.0))])
    lo, hi = (-2.5, -1.0, -0.5), (3.0, 2.0, 0.75)
    m = O.cell_masses(pot, O.make_obs(_spec(3, 2, 2, lo, hi, "cartesian"), np.eye(3)), rel_tol=1e-8, abs_tol=1e-2)
    assert m.sum() == pytest.approx(_box_flux_mass(pot, lo, hi), rel=1e-7)


@pytest.mark.parametrize("kind", ["da_t3", "da_v4"])
def test_needle_bar_box_is_gauss_flux(kind):
    pot = O.make_pot([(kind, (1e10, 0.5, 0.4, 3.0, 0.4))])
    lo, hi = (-1.0, -1.0, -0.8), (2.0, 1.5, 1.0)
    m = O.cell_masses(pot, O.make_obs(_spec(1, 1, 1, lo, hi, "cartesian"), np.eye(3)), rel_tol=1e-8, abs_tol=1e-1)
    assert m.sum() == pytest.approx(_box_flux_mass(pot, lo, hi, nq=40), rel=1e-6)


def test_flattened_halo_has_no_closed_form_density():
    """The flattened-potential NFW (q != 1) has no density formula here: the
    oracle returns NaN rather than a wrong mass."""
    pot = O.make_pot([("nfw_q", (1e12, 10.0, 0.9, 70.0))])
    m = O.cell_masses(pot, O.make_obs(_spec(1, 1, 1, (0, -1, -1), (1, 1, 1), "cartesian"), np.eye(3)), rel_tol=1e-6)
    assert np.isnan(m).all()
