"""GPU parity of the target cell masses m*_n (Sec. 2.2.4; Sec. 3's 600-cell
cylindrical grid, R 0-10 kpc, z +-3 kpc) against the oracle's nested adaptive
Gauss-Kronrod integrals.

Bar: |m_gpu - m_oracle| <= 1e-6 m_oracle + 1e-9 M_sel per cell, M_sel the
total mass of the selected components.  The first term covers the library's
quadrature on smooth densities (Gauss-Legendre 8^3 per box converges to
~1e-11 at two boxes per dimension); the second covers cells cut by the
Ferrers bar's edge, where the density (1 - m^2)^2 has a jump in its second
derivative and the composite rule converges slowly (below 1e-9 M at
n_sub = 8).  The oracle runs to 1e-12 M or better.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_common import lib
from tests.test_oracle_cellmass_pins import _cyl_flux_mass, _spec

pytestmark = pytest.mark.gpu

PAPER_GRID = _spec(10, 6, 10, (0.0, -math.pi, -3.0), (10.0, math.pi, 3.0), "cylindrical")


def gpu_cell_masses(components, spec, mask, n_sub):
    import torch
    P = lib()
    pot = P.build_potential(components, 0.0)
    out = torch.full((spec["nx"] * spec["ny"] * spec["nz"],), float("nan"), dtype=torch.float64, device="cuda:0")
    P.cell_masses(pot, P.obs_spec(spec), mask, n_sub, out)
    return out.cpu().numpy()


def _check(m_g, m_o, M):
    err = np.abs(m_g - m_o)
    bound = 1e-6 * np.abs(m_o) + 1e-9 * M
    print(f"max |err| / M = {err.max() / M:.2e}, worst err/bound = {(err / bound).max():.3f}")
    assert np.all(err <= bound)


def test_paper_grid_disc_and_bar(gpu):
    """Stellar disc + Ferrers bar of the barred model (the halo excluded) on
    the 600-cell cylindrical grid at n_sub = 8: every cell against the
    oracle, and the grid's total against the
    enclosed mass (Gauss's theorem for the disc, M for the bar, which lies
    inside the grid)."""
    comps = W.BARRED["components"]
    m_g = gpu_cell_masses(comps, PAPER_GRID, 0b011, 8)
    assert np.all(np.isfinite(m_g)) and np.all(m_g >= 0)
    stellar = O.make_pot(comps[:2])
    M = comps[0][1][0] + comps[1][1][0]
    m_o = O.cell_masses(stellar, O.make_obs(PAPER_GRID, np.eye(3)), rel_tol=1e-9, abs_tol=1e-3)
    _check(m_g, m_o, M)
    want = _cyl_flux_mass(O.make_pot(comps[:1]), 10.0, 3.0) + comps[1][1][0]
    assert abs(m_g.sum() - want) <= 1e-9 * M
    # the bar is bisymmetric and the disc axisymmetric: sectors k and k + 3 agree
    m6 = m_g.reshape(10, 6, 10)
    assert np.allclose(m6[:, :3], m6[:, 3:], rtol=1e-9, atol=1e-12 * M)


def test_cartesian_grid_plummer_and_disc(gpu):
    """The small model's bulge + disc on its 10 x 10 x 10 Cartesian grid at
    n_sub = 4, every cell against the oracle (a ragged subset of components:
    the disc alone, then both)."""
    comps = W.SMALL["components"]
    spec = dict(W.SMALL["obs"])
    for mask, sel in ((0b10, comps[1:]), (0b11, comps)):
        m_g = gpu_cell_masses(comps, spec, mask, 4)
        m_o = O.cell_masses(O.make_pot(sel), O.make_obs(spec, np.eye(3)), rel_tol=1e-10, abs_tol=1e-3)
        _check(m_g, m_o, sum(c[1][0] for c in sel))


@pytest.mark.parametrize("kind", ["da_t3", "da_v4"])
def test_needle_bar_cells(gpu, kind):
    """A needle bar on a 3 x 1 x 2 Cartesian grid around it at n_sub = 4:
    each cell against the oracle, whose density is itself an adaptive
    needle integral."""
    comps = [("mn", (4e10, 3.0, 0.3)), (kind, (1e10, 0.5, 0.4, 3.0, 0.4))]
    spec = _spec(3, 1, 2, (-1.0, -1.0, -0.8), (2.0, 1.5, 1.0), "cartesian")
    m_g = gpu_cell_masses(comps, spec, 0b10, 4)
    m_o = O.cell_masses(O.make_pot(comps[1:]), O.make_obs(spec, np.eye(3)), rel_tol=1e-8, abs_tol=1e-1)
    _check(m_g, m_o, 1e10)


def test_repeatable_and_timed(gpu):
    """Two calls give identical masses (fixed reduction order); the paper's
    grid at n_sub = 8 and the barred model's 18,000-cell Cartesian grid at
    n_sub = 4 are timed."""
    import torch
    P = lib()
    comps = W.BARRED["components"]
    pot = P.build_potential(comps, 0.0)
    for spec, n_sub in ((PAPER_GRID, 8), (W.BARRED["obs"], 4)):
        o = P.obs_spec(spec)
        n = spec["nx"] * spec["ny"] * spec["nz"]
        a = torch.empty(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        P.cell_masses(pot, o, 0b011, n_sub, a)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        P.cell_masses(pot, o, 0b011, n_sub, b)
        t1.record()
        torch.cuda.synchronize()
        print(f"{n} cells, n_sub {n_sub}: {t0.elapsed_time(t1):.2f} ms")
        assert torch.equal(a, b)
