"""Pins of the oracle's cylindrical mass grid (Sec. 2.2.4: 3D bins uniform in
R, phi and z).  Away from the edges the cell is the one a direct computation
of R = sqrt(x^2 + y^2) and phi = atan2(y, x) gives; on an edge the rule is
half-open (the lower edge belongs to the cell), the axis and the edge at
phi = pi go to the last sector; the four mirror copies (Table 1) reach the
cells of (x, y, +-z) and (-x, -y, +-z), so the symmetrised histogram is
invariant under those reflections.
"""
import math

import numpy as np

import oracle as O

SPEC = dict(nx=6, ny=8, nz=5, lo=(0.0, -math.pi, -2.0), hi=(9.0, math.pi, 2.0), npx=4, npy=4, plo=(-8, -8),
            phi=(8, 8), nv=5, vlo=-300, vhi=300, symmetrize=1, drift_every=1, grid="cylindrical")


def direct_cell(x, y, z):
    R = math.hypot(x, y)
    ir = math.floor(R / 1.5)
    isec = math.floor((math.atan2(y, x) + math.pi) / (2 * math.pi / 8))
    iz = math.floor((z + 2.0) / 0.8)
    if not (0 <= ir < 6 and 0 <= iz < 5):
        return -1
    return (ir * 8 + min(isec, 7)) * 5 + iz


def test_random_points_match_direct_computation():
    rng = np.random.default_rng(1)
    n = 4000
    pts = np.stack([rng.uniform(-10, 10, n), rng.uniform(-10, 10, n), rng.uniform(-2.5, 2.5, n),
                    rng.normal(0, 100, n), rng.normal(0, 100, n), rng.normal(0, 100, n)])
    mass, _ = O.bin_points(O.make_obs(SPEC, np.eye(3)), pts, "f64")
    for i in range(n):
        x, y, z = pts[:3, i]
        assert mass[i, 0] == direct_cell(x, y, z)
        assert mass[i, 1] == direct_cell(x, y, -z)
        assert mass[i, 2] == direct_cell(-x, -y, z)
        assert mass[i, 3] == direct_cell(-x, -y, -z)


def test_edges_axis_and_half_open_rule():
    obs = O.make_obs(SPEC, np.eye(3))
    w = 2 * math.pi / 8
    cases = []
    for k in range(8):  # exactly on the lower edge of sector k (as represented): inside k
        ph = -math.pi + 2 * math.pi * k / 8
        cases.append(((3.0 * math.cos(ph) + 1e-12 * math.cos(ph + w / 2), 3.0 * math.sin(ph) + 1e-12 * math.sin(ph + w / 2),
                       0.1), (2 * 8 + k) * 5 + 2))
    cases.append(((0.0, 0.0, 0.1), (0 * 8 + 7) * 5 + 2))       # the axis: last sector
    cases.append(((-3.0, 0.0, 0.1), (2 * 8 + 7) * 5 + 2))      # phi = pi: last sector
    cases.append(((1.5, 1e-9, 0.1), (1 * 8 + 4) * 5 + 2))      # R on the edge 1.5: outer bin
    cases.append(((9.0, 1e-9, 0.1), -1))                       # R on the outer edge: outside
    pts = np.zeros((6, len(cases)))
    for j, (p, _) in enumerate(cases):
        pts[:3, j] = p
    mass, _ = O.bin_points(obs, pts, "f64")
    for j, (_, want) in enumerate(cases):
        assert mass[j, 0] == want, (cases[j], mass[j, 0])


def test_symmetrised_histogram_is_mirror_invariant():
    rng = np.random.default_rng(2)
    n = 3000
    pts = np.stack([rng.uniform(-10, 10, n), rng.uniform(-10, 10, n), rng.uniform(-2.5, 2.5, n),
                    np.zeros(n), np.zeros(n), np.zeros(n)])

    def hist(p):
        m, _ = O.bin_points(O.make_obs(SPEC, np.eye(3)), p, "f64")
        h = np.zeros(6 * 8 * 5)
        for c in m.ravel():
            if c >= 0:
                h[c] += 1
        return h

    h0 = hist(pts)
    for s in ([1, 1, -1], [-1, -1, 1], [-1, -1, -1]):
        q = pts.copy()
        q[:3] *= np.array(s)[:, None]
        assert np.array_equal(hist(q), h0)
