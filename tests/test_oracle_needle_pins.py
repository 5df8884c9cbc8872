"""Pins of the Dehnen-Aly needle bars in the oracle (Eq. 12, App. A), beyond
the generic force = -grad Phi and Poisson pins that every component gets.

* A needle shorter than any other scale (L -> 0) leaves the parent
  axisymmetric T3 / V4 pairs, whose potentials are evaluated here in closed
  form from App. A.
* Far from the bar the potential is -GM/r whatever eta (f integrates to 1).
* The bar is symmetric under x -> -x, y -> -y, z -> -z.
* For eta = 0 and a point on the bar's axis beyond its end, I_1 has the
  elementary closed form asinh-type integral of a uniform needle.
"""
import math

import numpy as np
import pytest

import oracle as O

G = O.G


def parent_phi(kind, M, a, b, x):
    R2 = x[0] ** 2 + x[1] ** 2
    zeta = math.sqrt(x[2] ** 2 + b * b)
    Z = a + zeta
    R = math.sqrt(R2 + Z * Z)
    if kind == "da_t3":
        return -G * M * (1 / R + a * (Z - a / 3) / R ** 3 + a * a * Z * Z / R ** 5)
    return -G * M * (1 / R + (a * (Z - 2 * a / 5) + b * b / 2) / R ** 3
                     + 3 * a * (a * Z * (2 * Z - a) / 5 + b * b / 2 * (Z - a / 5)) / R ** 5
                     + a * a * Z * Z * (a * Z + 3 * b * b) / R ** 7 + 7 * a ** 3 * b * b * Z ** 4 / (2 * R ** 9 * zeta))


PTS = [np.array(p) for p in ([1.0, 2.0, 0.3], [0.2, -0.1, 0.05], [5.0, -1.0, 0.8], [0.0, 0.0, 0.0])]


@pytest.mark.parametrize("kind", ["da_t3", "da_v4"])
def test_short_needle_is_the_parent_pair(kind):
    M, a, b = 1e10, 1.2, 0.6
    pot = O.make_pot([(kind, (M, a, b, 1e-6, 0.7))])
    for x in PTS:
        assert O.phi(pot, x) == pytest.approx(parent_phi(kind, M, a, b, x), rel=1e-10)


@pytest.mark.parametrize("kind", ["da_t3", "da_v4"])
@pytest.mark.parametrize("eta", [-1.0, 0.0, 1.0])
def test_far_field_and_symmetry(kind, eta):
    M = 3e9
    pot = O.make_pot([(kind, (M, 1.0, 0.5, 3.0, eta))])
    x = np.array([3e3, -2e3, 1e3])
    r = np.linalg.norm(x)
    assert O.phi(pot, x) == pytest.approx(-G * M / r, rel=2e-3)
    for p in PTS[:3]:
        v = O.phi(pot, p)
        for s in ([-1, 1, 1], [1, -1, 1], [1, 1, -1]):
            assert O.phi(pot, p * np.array(s)) == pytest.approx(v, rel=1e-13)


def test_uniform_needle_on_axis_closed_form():
    """eta = 0, a = 0 (T3 reduces to -GM I_1 plus terms that vanish with a),
    point on the axis (y = 0): I_1 = (1/2L) [asinh((x + L)/Z) - asinh((x - L)/Z)]."""
    M, b, L = 2e9, 0.7, 2.5
    pot = O.make_pot([("da_t3", (M, 0.0, b, L, 0.0))])
    for xv, zv in ((0.3, 0.0), (4.0, 0.5), (-1.7, 1.2)):
        Z = math.sqrt(zv * zv + b * b)
        I1 = (math.asinh((xv + L) / Z) - math.asinh((xv - L) / Z)) / (2 * L)
        assert O.phi(pot, np.array([xv, 0.0, zv])) == pytest.approx(-G * M * I1, rel=1e-12)
