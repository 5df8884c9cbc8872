"""Pins of the oracle's Jeans-equation initial conditions (Sec. 2.2.1): the
velocity dispersions and mean rotation at each starting position from the
anisotropic Jeans equations in the azimuth-averaged potential, for the
fiducial tracer density nu ~ exp(-R/h_R - |z|/h_z).

Pins: on the axis of a point mass sigma_z^2 has the closed form
GM [1/z - e^(z/h_z) E1(z/h_z) / h_z]; off the axis the oracle's moments
(built with a Richardson difference in R) match the radial Jeans equation
evaluated with the analytic R-derivative of the point mass's vertical force
under the integral (scipy quadrature); the azimuth average of a barred
model's vertical force matches a 256-point trapezoid rule over the oracle's
force; the moments are invariant under the mirrors of Table 1; the draws
scale the dispersions and rotate prograde.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O

G = O.G
M = 1e10
HR, HZ = 3.5, 1.2


def test_point_mass_on_the_axis_closed_form():
    pot = O.make_pot([("kepler", (M,))])
    z = np.array([0.3, 1.0, 2.5])
    pos = np.stack([np.zeros(3), np.zeros(3), z])
    mom, ics = O.jeans_ics(pot, pos, np.zeros((3, 3)), HR, HZ, b=1.5)
    GM = G * M
    want = GM * (1 / z - np.exp(z / HZ) * special.exp1(z / HZ) / HZ)
    assert np.allclose(mom[2] ** 2, want, rtol=1e-9, atol=0)
    assert np.allclose(mom[0] ** 2, 1.5 * want, rtol=1e-9) and np.array_equal(mom[1], mom[0])
    assert np.all(mom[3] == 0.0)


@pytest.mark.parametrize("R,z,b", [(2.0, 0.5, 1.0), (5.0, 1.5, 2.0), (0.8, 0.1, 0.7)])
def test_point_mass_radial_jeans_equation(R, z, b):
    pot = O.make_pot([("kepler", (M,))])
    GM = G * M

    def fz(zp):
        return GM * zp / (R * R + zp * zp) ** 1.5

    def dfz_dR(zp):
        return -3 * GM * R * zp / (R * R + zp * zp) ** 2.5

    s2 = HZ * integrate.quad(lambda s: math.exp(-s) * fz(z + HZ * s), 0, np.inf, epsabs=0, epsrel=1e-13)[0]
    ds2 = HZ * integrate.quad(lambda s: math.exp(-s) * dfz_dR(z + HZ * s), 0, np.inf, epsabs=0, epsrel=1e-13)[0]
    vphi2 = b * (s2 * (1 - R / HR) + R * ds2) + GM * R * R / (R * R + z * z) ** 1.5
    mean = math.sqrt(max(vphi2 - b * s2, 0.0))
    mom, _ = O.jeans_ics(pot, np.array([[R], [0.0], [z]]), np.zeros((3, 1)), HR, HZ, b=b)
    assert mom[2, 0] ** 2 == pytest.approx(s2, rel=1e-9)
    assert mom[0, 0] ** 2 == pytest.approx(b * s2, rel=1e-9)
    assert mom[3, 0] == pytest.approx(mean, rel=1e-7)
    assert mom[4, 0] == pytest.approx(math.sqrt(GM * R * R / (R * R + z * z) ** 1.5), rel=1e-10)


def test_barred_azimuth_average_matches_trapezoid():
    comps = [("mn", (4e10, 3.0, 0.3)), ("ferrers2", (1e10, 4.0, 1.5, 1.0))]
    pot = O.make_pot(comps)
    R, z = 3.0, 0.4
    ph = np.arange(256) * (2 * math.pi / 256)

    def fz_avg(zp):
        return -np.mean([O.accel(pot, np.array([R * math.cos(p), R * math.sin(p), zp]))[2] for p in ph])

    s2 = HZ * integrate.quad(lambda s: math.exp(-s) * fz_avg(z + HZ * s), 0, 70, epsabs=0, epsrel=1e-10, limit=200)[0]
    mom, _ = O.jeans_ics(pot, np.array([[R * math.cos(0.3)], [R * math.sin(0.3)], [z]]), np.zeros((3, 1)), HR, HZ)
    assert mom[2, 0] ** 2 == pytest.approx(s2, rel=1e-8)


def test_mirror_invariance_and_draws():
    comps = [("mn", (4e10, 3.0, 0.3)), ("ferrers2", (1e10, 4.0, 1.5, 1.0))]
    pot = O.make_pot(comps)
    p = np.array([2.0, -1.0, 0.3])
    pos = np.stack([p, p * [1, 1, -1], -p * [1, 1, -1], -p], axis=1)
    eps = np.array([[0.5] * 4, [-1.0] * 4, [2.0] * 4])
    mom, ics = O.jeans_ics(pot, pos, eps, HR, HZ)
    assert np.allclose(mom, mom[:, :1], rtol=1e-10, atol=0)
    assert np.array_equal(ics[:3], pos)
    x, y = pos[0, 0], pos[1, 0]
    R = math.hypot(x, y)
    vR = (ics[3, 0] * x + ics[4, 0] * y) / R
    vp = (x * ics[4, 0] - y * ics[3, 0]) / R
    assert vR == pytest.approx(0.5 * mom[0, 0], rel=1e-12)
    assert vp == pytest.approx(mom[3, 0] - mom[1, 0], rel=1e-12)
    assert ics[5, 0] == pytest.approx(2.0 * mom[2, 0], rel=1e-12)
    assert mom[3, 0] > 0  # prograde
