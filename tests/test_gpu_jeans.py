"""GPU parity of the Jeans-equation initial conditions (Sec. 2.2.1) against the
oracle's adaptive Gauss-Kronrod integrals (the same Richardson step in R).

Bar: dispersions to 1e-6 relative; the mean rotation, which holds a
difference quotient of the dispersion, to 1e-4 km/s plus 1e-6 relative.  The
library's rules (13 graded panels of 8-point Gauss-Legendre in s, a 128-point
trapezoid rule in azimuth) reach ~1e-9 on these potentials, and the
difference quotient multiplies an error that varies with R by R / h = 500 at
most, an error that does not by nothing.
"""
import math

import numpy as np
import pytest
from scipy import special

import oracle as O
import workloads as W
from oracle import ics as I
from tests.gpu_common import lib

pytestmark = pytest.mark.gpu

HR, HZ = 3.5, 1.2


def gpu_jeans(components, pos, eps, b=1.0):
    import torch
    P = lib()
    pot = P.build_potential(components, 0.0)
    dev = torch.device("cuda:0")
    n = pos.shape[1]
    mom = torch.empty((5, n), dtype=torch.float64, device=dev)
    ics = torch.empty((6, n), dtype=torch.float64, device=dev)
    P.jeans_ics(pot, torch.from_numpy(np.ascontiguousarray(pos)).to(dev),
                torch.from_numpy(np.ascontiguousarray(eps)).to(dev), HR, HZ, b, mom, ics)
    return mom.cpu().numpy(), ics.cpu().numpy()


def _check(mom_g, mom_o):
    idx = [0, 1, 2, 4]
    err = np.abs(mom_g[idx] - mom_o[idx])
    rel = err / np.maximum(np.abs(mom_o[idx]), 1e-300)
    dv = np.abs(mom_g[3] - mom_o[3])
    print(f"dispersions and v_c max rel {rel.max():.2e}, mean rotation max abs {dv.max():.2e} km/s")
    assert np.all(err <= 1e-6 * np.abs(mom_o[idx]))
    assert np.all(dv <= 1e-4 + 1e-6 * np.abs(mom_o[3]))


def test_barred_model_matches_oracle(gpu):
    """Disc + Ferrers bar + flattened halo of the barred model at 10 seeded
    positions of the fiducial double-exponential, plus the axis and a point
    near it."""
    comps = W.BARRED["components"]
    pos, eps = W.disc_positions(10, seed=4)
    pos = np.concatenate([pos, [[0.0, 0.05], [0.0, -0.02], [0.7, -0.3]]], axis=1)
    eps = np.concatenate([eps, np.ones((3, 2))], axis=1)
    mom_g, ics_g = gpu_jeans(comps, pos, eps, b=1.3)
    mom_o, ics_o = O.jeans_ics(O.make_pot(comps), pos, eps, HR, HZ, b=1.3)
    _check(mom_g, mom_o)
    assert np.array_equal(ics_g[:3], pos)
    assert np.allclose(ics_g[3:], ics_o[3:], rtol=0, atol=1e-4 + 1e-6 * np.abs(ics_o[3:]).max())


def test_point_mass_axis_closed_form(gpu):
    """sigma_z^2 on the axis of a point mass: GM [1/z - e^(z/h_z) E1(z/h_z) / h_z]."""
    M = 1e10
    z = np.array([0.3, 1.0, 2.5, 6.0])
    pos = np.stack([np.zeros(4), np.zeros(4), z])
    mom, _ = gpu_jeans([("kepler", (M,))], pos, np.zeros((3, 4)))
    want = O.G * M * (1 / z - np.exp(z / HZ) * special.exp1(z / HZ) / HZ)
    assert np.allclose(mom[2] ** 2, want, rtol=1e-8, atol=0)
    assert np.all(mom[3] == 0.0)


def test_needle_bar_and_timing(gpu):
    """A potential with a needle bar takes the needle kernels: 4 positions
    against the oracle; then 30,000 positions (the paper's 7,500 x 4) of the
    barred model timed."""
    import torch
    comps = [("mn", (4e10, 3.0, 0.3)), ("da_t3", (1e10, 0.5, 0.4, 3.0, 0.4))]
    pos, eps = W.disc_positions(4, seed=7)
    mom_g, _ = gpu_jeans(comps, pos, eps)
    mom_o, _ = O.jeans_ics(O.make_pot(comps), pos, eps, HR, HZ)
    _check(mom_g, mom_o)
    P = lib()
    pos, eps = W.disc_positions(30000, seed=8)
    pot = P.build_potential(W.BARRED["components"], 0.0)
    dev = torch.device("cuda:0")
    p_t, e_t = torch.from_numpy(pos).to(dev), torch.from_numpy(eps).to(dev)
    mom = torch.empty((5, 30000), dtype=torch.float64, device=dev)
    ics = torch.empty((6, 30000), dtype=torch.float64, device=dev)
    P.jeans_ics(pot, p_t, e_t, HR, HZ, 1.0, mom, ics)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    P.jeans_ics(pot, p_t, e_t, HR, HZ, 1.0, mom, ics)
    t1.record()
    torch.cuda.synchronize()
    print(f"30000 positions: {t0.elapsed_time(t1):.1f} ms")
    assert torch.isfinite(ics).all() and (mom[:3] > 0).all()


def test_dither_and_bundles_bit_exact(gpu):
    """Four realisations of 333 initial conditions on the paper's box (0.1 kpc,
    5% of v_c) and the bundle means of FP32 and FP64 orbit matrices (ragged
    column count) equal the oracle's bit for bit."""
    import torch
    P = lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    n = 333
    ics = rng.normal(0, 100, (6, n))
    vc = rng.uniform(50, 250, n)
    u = W.dither_deviates(4, n, seed=6)
    out = torch.empty((6, 4 * n), dtype=torch.float64, device=dev)
    P.dither_ics(torch.from_numpy(ics).to(dev), torch.from_numpy(vc).to(dev), torch.from_numpy(u).to(dev), 0.1, 0.05,
                 out)
    assert np.array_equal(out.cpu().numpy(), I.dither(ics, vc, u, 0.1, 0.05))
    for td, nd in ((torch.float32, 4), (torch.float64, 4), (torch.float32, 3)):
        A = torch.rand((nd * 97, 1001), dtype=td, device=dev)
        B = torch.empty((97, 1001), dtype=td, device=dev)
        P.bundle_rows(A, nd, B)
        want = I.bundle_rows(A.cpu().numpy(), nd).astype(np.float32 if td == torch.float32 else np.float64)
        assert np.array_equal(B.cpu().numpy(), want)
