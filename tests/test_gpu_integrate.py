"""GPU parity of integrate_and_bin / bin_points / integrate_orbits against the oracle.

Bar: bin indices are bit-exact on identical inputs (both sides decide in the
same precision); double-precision trajectories of the analytic potentials are
bit-exact (both sides evaluate the same expression order with IEEE sqrt and
division and no FMA contraction), hence counts, drifts and flags are equal;
the single-precision barred path is compared statistically with the FP64
oracle on a seeded subsample.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_common import counts_from_fractions, gpu_integrate, lib, oracle_integrate

pytestmark = pytest.mark.gpu


def edge_points(obs, R, rng, n, dtype):
    """Random states plus states whose coordinates sit on, and one ulp either
    side of, grid edges (in the given precision)."""
    pts = np.stack([rng.uniform(-12, 12, n), rng.uniform(-12, 12, n), rng.uniform(-4, 4, n),
                    rng.normal(0, 200, n), rng.normal(0, 200, n), rng.normal(0, 200, n)]).astype(dtype)
    k = n // 4
    for axis, (lo, hi, nb) in enumerate(zip(obs["lo"], obs["hi"], (obs["nx"], obs["ny"], obs["nz"]))):
        edges = lo + (hi - lo) * rng.integers(0, nb + 1, k) / nb
        e = edges.astype(dtype)
        jitter = rng.integers(-1, 2, k)
        e = np.where(jitter < 0, np.nextafter(e, dtype(-np.inf)), np.where(jitter > 0, np.nextafter(e, dtype(np.inf)), e))
        pts[axis, axis * k:(axis + 1) * k] = e
    return pts


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_bin_points_bit_exact(gpu, dtype):
    import torch
    P = lib()
    cfg = W.BARRED
    npd = np.float64 if dtype == "f64" else np.float32
    rng = np.random.default_rng(11)
    pts = edge_points(cfg["obs"], None, rng, 20000, npd)
    pot = P.build_potential(cfg["components"], cfg["omega"], cfg["euler"])
    o = P.obs_spec(cfg["obs"])
    t = torch.from_numpy(pts).to(gpu)
    mass = torch.empty((pts.shape[1], 4), dtype=torch.int32, device=gpu)
    kin = torch.empty_like(mass)
    P.bin_points(pot, o, t, mass, kin)
    torch.cuda.synchronize()
    om, ok = O.bin_points(O.make_obs(cfg["obs"], O.euler_matrix(*cfg["euler"])), pts, dtype)
    assert np.array_equal(mass.cpu().numpy(), om)
    assert np.array_equal(kin.cpu().numpy(), ok)
    assert (om < 0).any() and (om >= 0).any()


def test_integrate_orbits_fp64_bit_exact(gpu):
    """Plummer + Miyamoto-Nagai, static and rotating frame: final states equal to the last bit."""
    import torch
    P = lib()
    rng = np.random.default_rng(5)
    n = 193
    ics = np.stack([rng.uniform(-8, 8, n), rng.uniform(-8, 8, n), rng.uniform(-1, 1, n),
                    rng.normal(0, 120, n), rng.normal(0, 120, n), rng.normal(0, 40, n)])
    dt = rng.uniform(5e-4, 3e-3, n)
    comps = [("plummer", (1e10, 0.5)), ("mn", (5e10, 3.0, 0.3)), ("kepler", (1e8,)), ("isochrone", (2e9, 1.0))]
    pot = P.build_potential(comps, 0.0, (0.0, 0.0, 0.0))
    out = torch.empty((6, n), dtype=torch.float64, device=gpu)
    P.integrate_orbits(pot, torch.from_numpy(ics).to(gpu), torch.from_numpy(dt).to(gpu), 500, out)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    opot = O.make_pot(comps, 0.0)
    for i in range(n):
        ref = O.orbit(opot, ics[:, i], dt[i], 500)[-1]
        assert np.array_equal(g[:, i], ref), (i, g[:, i] - ref)


def test_small_workload_fp64_counts_identical(gpu):
    """The full Plummer + MN workload (2,000 orbits x 1,000 FP64 steps): integer
    counts, overflow, Jacobi drift and flags identical to the oracle."""
    cfg = W.SMALL
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=cfg["n_steps"])
    A, ov, dr, fl = gpu_integrate(cfg, ics, dt, cfg["n_steps"], "f64")
    c_o, ov_o, dr_o, fl_o = oracle_integrate(cfg, ics, dt, cfg["n_steps"])
    assert np.array_equal(counts_from_fractions(A, cfg["n_steps"]), c_o)
    assert np.array_equal(A, O.time_fractions(c_o, cfg["n_steps"]))
    assert np.array_equal(np.rint(ov * 4 * cfg["n_steps"]).astype(np.int64), ov_o)
    assert np.max(np.abs(dr - dr_o)) <= 1e-5  # parity bar; expected bit-exact
    assert np.array_equal(dr, dr_o)
    assert np.array_equal(fl, fl_o)


@pytest.mark.parametrize("n,n_steps,sym", [(1, 7, 1), (63, 33, 0), (130, 50, 1)])
def test_ragged_shapes_fp64(gpu, n, n_steps, sym):
    cfg = W.SMALL
    rng = np.random.default_rng(n)
    ics = np.stack([rng.uniform(-8, 8, n), rng.uniform(-8, 8, n), rng.uniform(-1, 1, n),
                    rng.normal(0, 150, n), rng.normal(0, 150, n), rng.normal(0, 50, n)])
    dt = rng.uniform(1e-3, 4e-3, n)
    obs = dict(cfg["obs"], symmetrize=sym, drift_every=3)
    A, ov, dr, fl = gpu_integrate(cfg, ics, dt, n_steps, "f64", obs=obs)
    c_o, ov_o, dr_o, fl_o = oracle_integrate(cfg, ics, dt, n_steps, obs=obs)
    ncopy = 4 if sym else 1
    assert np.array_equal(counts_from_fractions(A, n_steps, ncopy), c_o)
    assert np.array_equal(np.rint(ov * ncopy * n_steps).astype(np.int64), ov_o)
    assert np.array_equal(dr, dr_o) and np.array_equal(fl, fl_o)


_ORACLE_CACHE = {}


def _barred_oracle(ic64, dt64, n_steps, f32_state):
    key = f32_state
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle_integrate(W.BARRED, ic64, dt64, n_steps, f32_state=f32_state)
    return _ORACLE_CACHE[key]


@pytest.mark.parametrize("lanes", [1, 2])
def test_barred_fp32_subsample_vs_fp64_oracle(gpu, lanes):
    """Barred model (MN + Ferrers + flattened NFW, 40 km/s/kpc) in FP32 against the
    FP64 oracle on the seeded 1,000-orbit subsample of the 100,000-orbit library,
    full 10,000 steps.  Exact: per-block normalisation of every row.  Jacobi
    drift: median |drift_f32 - drift_f64| <= 1e-5.  Time fractions: chaotic
    orbits of a rotating bar amplify any rounding difference, so the per-orbit
    L1 distance between GPU and oracle rows is compared with the distance
    between the oracle and the oracle whose state is rounded to binary32 after
    every step (the error any FP32 integrator carries): the GPU must not
    decorrelate much faster than that floor.  Run with one and with two lanes
    per orbit."""
    cfg = W.BARRED
    n_steps = cfg["n_steps"]
    table = W.load_table(cfg["table"])
    ics, dt = W.disc_ics(table, cfg["n_orb"], seed=cfg["ic_seed"], n_steps=n_steps)
    sub = W.subsample_draw(cfg["n_orb"], cfg["subsample"]["n"], cfg["subsample"]["seed"])
    ics32, dt32 = ics[:, sub].astype(np.float32), dt[sub].astype(np.float32)
    P = lib()
    P.set_tuning("integrate_lanes_per_orbit", lanes)
    try:
        A, ov, dr, fl = gpu_integrate(cfg, ics32, dt32, n_steps, "f32")
    finally:
        P.set_tuning("integrate_lanes_per_orbit", 1)
    ic64, dt64 = ics32.astype(np.float64), dt32.astype(np.float64)
    c_o, ov_o, dr_o, fl_o = _barred_oracle(ic64, dt64, n_steps, False)
    c_p, *_ = _barred_oracle(ic64, dt64, n_steps, True)
    c_g = counts_from_fractions(A, n_steps)
    nm = 30 * 30 * 20
    ovc = np.rint(ov * 4 * n_steps).astype(np.int64)
    assert np.all(c_g[:, :nm].sum(1) + ovc[:, 0] == 4 * n_steps)
    assert np.all(c_g[:, nm:].sum(1) + ovc[:, 1] == 4 * n_steps)
    A_o, A_p = O.time_fractions(c_o, n_steps), O.time_fractions(c_p, n_steps)
    l1 = np.abs(A.astype(np.float64) - A_o).sum(1) / 2
    l1_ref = np.abs(A_p - A_o).sum(1) / 2
    ddr = np.abs(dr - dr_o)
    print(f"row L1 gpu-vs-oracle median {np.median(l1):.3g} p90 {np.percentile(l1, 90):.3g}; "
          f"oracle-vs-fp32-state-oracle median {np.median(l1_ref):.3g} p90 {np.percentile(l1_ref, 90):.3g}; "
          f"|drift_f32 - drift_f64| median {np.median(ddr):.3g} p90 {np.percentile(ddr, 90):.3g}; "
          f"flagged {np.mean(fl & 1):.4f} vs {np.mean(fl_o & 1):.4f}")
    assert np.median(ddr) <= 1e-5
    assert np.median(l1) <= 2.0 * np.median(l1_ref) + 0.01
    assert np.percentile(l1, 90) <= 2.0 * np.percentile(l1_ref, 90) + 0.02
    assert abs(np.mean(fl & 1) - np.mean(fl_o & 1)) <= 0.01


CYL = dict(nx=10, ny=6, nz=10, lo=(0.0, -math.pi, -3.0), hi=(10.0, math.pi, 3.0), npx=10, npy=5, plo=(-10, -5),
           phi=(10, 5), nv=15, vlo=-450, vhi=450, symmetrize=1, drift_every=1, grid="cylindrical")


def cyl_edge_points(rng, n, dtype):
    """Random states plus states on, and one ulp either side of, the R edges
    (on the x axis, where R^2 = x^2) and on the sector edge directions."""
    pts = np.stack([rng.uniform(-12, 12, n), rng.uniform(-12, 12, n), rng.uniform(-4, 4, n),
                    rng.normal(0, 200, n), rng.normal(0, 200, n), rng.normal(0, 200, n)]).astype(dtype)
    k = n // 3
    e = (CYL["lo"][0] + rng.integers(0, CYL["nx"] + 1, k) * ((CYL["hi"][0] - CYL["lo"][0]) / CYL["nx"])).astype(dtype)
    jit = rng.integers(-1, 2, k)
    e = np.where(jit < 0, np.nextafter(e, dtype(-np.inf)), np.where(jit > 0, np.nextafter(e, dtype(np.inf)), e))
    sgn = np.where(rng.random(k) < 0.5, -1, 1).astype(dtype)
    pts[0, :k] = sgn * e
    pts[1, :k] = 0
    ph = -math.pi + 2.0 * math.pi * rng.integers(0, CYL["ny"] + 1, k) / CYL["ny"]
    r = rng.uniform(0.5, 9.5, k)
    pts[0, k:2 * k] = (r * np.cos(ph).astype(dtype)).astype(dtype)
    pts[1, k:2 * k] = (r * np.sin(ph).astype(dtype)).astype(dtype)
    pts[:3, 2 * k] = 0  # the axis
    return pts


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cylindrical_bin_points_bit_exact(gpu, dtype):
    import torch
    P = lib()
    npd = np.float64 if dtype == "f64" else np.float32
    rng = np.random.default_rng(12)
    pts = cyl_edge_points(rng, 30000, npd)
    euler = (0.7, 1.0, 0.0)
    pot = P.build_potential(W.SMALL["components"], 0.0, euler)
    o = P.obs_spec(CYL)
    t = torch.from_numpy(pts).to(gpu)
    mass = torch.empty((pts.shape[1], 4), dtype=torch.int32, device=gpu)
    kin = torch.empty_like(mass)
    P.bin_points(pot, o, t, mass, kin)
    torch.cuda.synchronize()
    om, ok = O.bin_points(O.make_obs(CYL, O.euler_matrix(*euler)), pts, dtype)
    assert np.array_equal(mass.cpu().numpy(), om)
    assert np.array_equal(kin.cpu().numpy(), ok)
    assert (om < 0).any() and (om >= 0).any()


def test_cylindrical_small_workload_fp64_counts_identical(gpu):
    """The small model (2,000 orbits x 1,000 FP64 steps) on a 10 x 6 x 10 = 600-cell
    cylindrical grid: counts, drifts and flags equal to the oracle's."""
    cfg = W.SMALL
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=1000)
    A, ov, dr, fl = gpu_integrate(cfg, ics, dt, 1000, "f64", obs=CYL)
    c_o, ov_o, dr_o, fl_o = oracle_integrate(cfg, ics, dt, 1000, obs=CYL)
    assert np.array_equal(counts_from_fractions(A, 1000), c_o)
    assert np.array_equal(dr, dr_o) and np.array_equal(fl, fl_o)
    assert c_o[:, :600].sum() > 0


SURF = dict(W.SMALL["obs"], surface=1, upsilon=2.5, vlo=-120.0, vhi=150.0, nv=9)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_surface_bin_points_bit_exact(gpu, dtype):
    """With the surface-density block on, an event in an aperture whose
    velocity is outside the range reports kin = n_ap * nv + aperture."""
    import torch
    P = lib()
    npd = np.float64 if dtype == "f64" else np.float32
    rng = np.random.default_rng(21)
    n = 20000
    pts = np.stack([rng.uniform(-12, 12, n), rng.uniform(-12, 12, n), rng.uniform(-4, 4, n),
                    rng.normal(0, 200, n), rng.normal(0, 200, n), rng.normal(0, 200, n)]).astype(npd)
    euler = W.SMALL["euler"]
    pot = P.build_potential(W.SMALL["components"], 0.0, euler)
    t = torch.from_numpy(pts).to(gpu)
    mass = torch.empty((n, 4), dtype=torch.int32, device=gpu)
    kin = torch.empty_like(mass)
    P.bin_points(pot, P.obs_spec(SURF), t, mass, kin)
    torch.cuda.synchronize()
    om, ok = O.bin_points(O.make_obs(SURF, O.euler_matrix(*euler)), pts, dtype)
    assert np.array_equal(mass.cpu().numpy(), om)
    assert np.array_equal(kin.cpu().numpy(), ok)
    n_kin = 50 * 9
    assert (ok >= n_kin).any() and ((ok >= 0) & (ok < n_kin)).any() and (ok < 0).any()


@pytest.mark.parametrize("n_orb,n_steps", [(2000, 1000), (130, 17000)], ids=["small", "wide-counters"])
def test_surface_block_fp64_identical(gpu, n_orb, n_steps):
    """Small model with the surface block (Upsilon = 2.5, a velocity range
    that leaves some events out): the whole orbit matrix, overflow, drift and
    flags equal the oracle's; the second case has more events per row than a
    16-bit counter holds."""
    cfg = W.SMALL
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=n_steps)
    ics, dt = ics[:, :n_orb], dt[:n_orb]
    A, ov, dr, fl = gpu_integrate(cfg, ics, dt, n_steps, "f64", obs=SURF)
    c_o, ov_o, dr_o, fl_o = oracle_integrate(cfg, ics, dt, n_steps, obs=SURF)
    oobs = O.make_obs(SURF, O.euler_matrix(*cfg["euler"]))
    assert A.shape[1] == 1000 + 450 + 50
    assert np.array_equal(A, O.time_fractions(c_o, n_steps, obs=oobs))
    assert np.array_equal(ov, ov_o / (4.0 * n_steps))
    assert np.array_equal(dr, dr_o) and np.array_equal(fl, fl_o)
    kin = c_o[:, 1000:1450].reshape(n_orb, 50, 9).sum(2)
    assert (c_o[:, 1450:] > kin).any()
