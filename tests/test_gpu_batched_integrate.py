"""GPU parity of the multi-potential integrate_and_bin launch (batched trial
potentials, Sec. 3.2.3's batched chains) and of irregular pixel-to-aperture
maps (Sec. 2.2.4's Voronoi regrouping of pixels) against the oracle.

One launch carries several potentials with ragged orbit counts (one of them
empty); each potential's rows are compared with one oracle run of that
potential alone.  Every launch shape the batched builds use is covered: the
one-wave-per-workgroup grid and the persistent grid (8 waves per CU), both
LDS budgets of the histogram workgroups, Cartesian and cylindrical mass grids,
and a workspace small enough that the orbits run in several chunks whose
boundaries fall inside potentials.

Bar: double-precision orbits of the analytic potentials are bit-exact (counts,
overflow, drift, flags); the single-precision barred family meets the
statistical bar of the single-potential FP32 test (row L1 against the FP64
oracle within twice the FP32-state oracle's floor, drift parity at the median).
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_common import counts_from_fractions, lib

pytestmark = pytest.mark.gpu

DEG = math.pi / 180.0

# four analytic potentials, each with its own viewing angles; offsets ragged, one potential empty
FP64_POTS = [
    ([("plummer", (1e10, 0.5)), ("mn", (5e10, 3.0, 0.3))], (45 * DEG, 60 * DEG, 0.0)),
    ([("plummer", (2e10, 0.8)), ("mn", (3e10, 2.5, 0.4))], (10 * DEG, 30 * DEG, 5 * DEG)),
    ([("isochrone", (8e9, 1.0)), ("mn", (6e10, 3.5, 0.25))], (80 * DEG, 75 * DEG, 0.0)),
    ([("plummer", (1.5e10, 0.6)), ("mn", (4e10, 3.0, 0.5)), ("kepler", (1e8,))], (0.0, 45 * DEG, 20 * DEG)),
]
OFFSETS = [0, 150, 150, 301, 397]

CYL = dict(nx=10, ny=6, nz=10, lo=(0.0, -math.pi, -3.0), hi=(10.0, math.pi, 3.0), npx=10, npy=5, plo=(-10, -5),
           phi=(10, 5), nv=15, vlo=-450, vhi=450, symmetrize=1, drift_every=1, grid="cylindrical")


def _ics(n, seed):
    rng = np.random.default_rng(seed)
    ics = np.stack([rng.uniform(-8, 8, n), rng.uniform(-8, 8, n), rng.uniform(-1, 1, n),
                    rng.normal(0, 150, n), rng.normal(0, 150, n), rng.normal(0, 50, n)])
    return ics, rng.uniform(1e-3, 4e-3, n)


def _gpu_batched(pots, offsets, ics, dt, n_steps, obs, dtype, ws_orbits=None, pix2ap=None):
    """One integrate_and_bin launch over all potentials; ws_orbits caps the
    workspace at that many orbits' event streams (forces chunking)."""
    import torch
    P = lib()
    dev = torch.device("cuda:0")
    td = torch.float64 if dtype == "f64" else torch.float32
    code = P.SW_F64 if dtype == "f64" else P.SW_F32
    p2a = None if pix2ap is None else torch.from_numpy(np.asarray(pix2ap, dtype=np.int32)).to(dev)
    o = P.obs_spec(obs, p2a)
    n = ics.shape[1]
    nc = P.ncon(o)
    A = torch.full((n, nc), float("nan"), dtype=td, device=dev)
    ov = torch.full((n, 2), float("nan"), dtype=torch.float64, device=dev)
    dr = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    fl = torch.full((n,), 255, dtype=torch.uint8, device=dev)
    full = P.integrate_workspace_bytes(o, len(pots), n, n_steps, code)
    nbytes = full
    if ws_orbits is not None:
        nbytes = P.integrate_workspace_bytes(o, len(pots), ws_orbits, n_steps, code) + 4096
        assert nbytes < full
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    P.integrate_and_bin(pots, offsets, torch.from_numpy(np.ascontiguousarray(ics)).to(dev, td),
                        torch.from_numpy(np.ascontiguousarray(dt)).to(dev, td), n_steps, o, A, ov, dr, fl, ws)
    torch.cuda.synchronize()
    return A.cpu().numpy(), ov.cpu().numpy(), dr.cpu().numpy(), fl.cpu().numpy()


def _oracle_one(comps, omega, euler, obs, ics, dt, n_steps, f32_state=False):
    pot = O.make_pot(comps, omega)
    ob = O.make_obs(obs, O.euler_matrix(*euler))
    return O.integrate_and_bin(pot, ob, ics, dt, n_steps, f32_state=f32_state), ob


class _Tuning:
    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        P = lib()
        self.old = {k: P.get_tuning(k) for k in self.kv}
        for k, v in self.kv.items():
            P.set_tuning(k, v)

    def __exit__(self, *a):
        P = lib()
        for k, v in self.old.items():
            P.set_tuning(k, v)


@pytest.mark.parametrize("grid", ["cartesian", "cylindrical"])
@pytest.mark.parametrize("waves", [0, 8])
@pytest.mark.parametrize("lds_kb", [32, 64])
@pytest.mark.parametrize("chunked", [False, True])
def test_batched_fp64_bit_exact_per_potential(gpu, grid, waves, lds_kb, chunked):
    P = lib()
    n_steps = 240
    obs = dict(W.SMALL["obs"], drift_every=3) if grid == "cartesian" else CYL
    ics, dt = _ics(OFFSETS[-1], seed=31)
    pots = [P.build_potential(c, 0.0, e) for c, e in FP64_POTS]
    with _Tuning(integrate_waves_per_cu=waves, hist_lds_kb=lds_kb):
        A, ov, dr, fl = _gpu_batched(pots, OFFSETS, ics, dt, n_steps, obs, "f64", ws_orbits=128 if chunked else None)
    for k, (comps, euler) in enumerate(FP64_POTS):
        a, b = OFFSETS[k], OFFSETS[k + 1]
        if a == b:
            continue
        (c_o, ov_o, dr_o, fl_o), ob = _oracle_one(comps, 0.0, euler, obs, ics[:, a:b], dt[a:b], n_steps)
        assert np.array_equal(A[a:b], O.time_fractions(c_o, n_steps, obs=ob)), (k, grid, waves, lds_kb, chunked)
        assert np.array_equal(ov[a:b], ov_o / (4.0 * n_steps)), k
        assert np.array_equal(dr[a:b], dr_o), k
        assert np.array_equal(fl[a:b], fl_o), k


def test_batched_wide_counters_and_empty_ends(gpu):
    """Potentials with no orbits at both ends of the offsets, and more events per
    row than a 16-bit histogram counter holds (4 x 17,000 steps)."""
    P = lib()
    n_steps = 17000
    obs = dict(W.SMALL["obs"], drift_every=50)
    ics, dt = _ics(70, seed=32)
    offs = [0, 0, 40, 70, 70]
    pots = [P.build_potential(FP64_POTS[i][0], 0.0, FP64_POTS[i][1]) for i in (0, 1, 2, 3)]
    with _Tuning(integrate_waves_per_cu=8, hist_lds_kb=32):
        A, ov, dr, fl = _gpu_batched(pots, offs, ics, dt, n_steps, obs, "f64")
    for k in (1, 2):
        a, b = offs[k], offs[k + 1]
        (c_o, ov_o, dr_o, fl_o), ob = _oracle_one(FP64_POTS[k][0], 0.0, FP64_POTS[k][1], obs, ics[:, a:b], dt[a:b],
                                                  n_steps)
        assert np.array_equal(A[a:b], O.time_fractions(c_o, n_steps, obs=ob)), k
        assert np.array_equal(dr[a:b], dr_o) and np.array_equal(fl[a:b], fl_o), k


def _walker_models(n_pot, seed):
    th = W.walker_thetas(n_pot, seed=seed)
    return [W.theta_to_model(t) for t in th]


@pytest.mark.parametrize("waves,lds_kb,chunked", [(0, 64, False), (8, 32, True)])
def test_batched_fp32_barred_family_vs_fp64_oracle(gpu, waves, lds_kb, chunked):
    """Three trial potentials of the barred family (walker draws: disc, Ferrers bar
    rotating at its own pattern speed, flattened NFW halo, own inclination), 2,000
    FP32 steps over the barred model's observables, in one launch: every row's
    blocks normalised exactly; per potential the row L1 against the FP64 oracle
    within twice the FP32-state oracle's floor, drift parity at the median."""
    P = lib()
    cfg = W.BARRED
    n_steps = 2000
    models = _walker_models(3, seed=41)
    offs = [0, 96, 160, 288]
    table = W.load_table(cfg["table"])
    ics, dt = W.disc_ics(table, offs[-1], seed=42, n_steps=n_steps, periods=10.0)
    ics32, dt32 = ics.astype(np.float32), dt.astype(np.float32)
    pots = [P.build_potential(c, om, eu) for c, om, eu in models]
    obs = dict(cfg["obs"])
    with _Tuning(integrate_waves_per_cu=waves, hist_lds_kb=lds_kb):
        A, ov, dr, fl = _gpu_batched(pots, offs, ics32, dt32, n_steps, obs, "f32", ws_orbits=64 if chunked else None)
    nm = 30 * 30 * 20
    c_g = counts_from_fractions(A, n_steps)
    ovc = np.rint(ov * 4 * n_steps).astype(np.int64)
    assert np.all(c_g[:, :nm].sum(1) + ovc[:, 0] == 4 * n_steps)
    assert np.all(c_g[:, nm:].sum(1) + ovc[:, 1] == 4 * n_steps)
    ic64, dt64 = ics32.astype(np.float64), dt32.astype(np.float64)
    for k, (comps, om, eu) in enumerate(models):
        a, b = offs[k], offs[k + 1]
        (c_o, _, dr_o, fl_o), ob = _oracle_one(comps, om, eu, obs, ic64[:, a:b], dt64[a:b], n_steps)
        (c_p, *_), _ = _oracle_one(comps, om, eu, obs, ic64[:, a:b], dt64[a:b], n_steps, f32_state=True)
        A_o, A_p = O.time_fractions(c_o, n_steps, obs=ob), O.time_fractions(c_p, n_steps, obs=ob)
        l1 = np.abs(A[a:b].astype(np.float64) - A_o).sum(1) / 2
        l1_ref = np.abs(A_p - A_o).sum(1) / 2
        ddr = np.abs(dr[a:b] - dr_o)
        print(f"potential {k}: row L1 median {np.median(l1):.3g} (floor {np.median(l1_ref):.3g}), "
              f"p90 {np.percentile(l1, 90):.3g} (floor {np.percentile(l1_ref, 90):.3g}); "
              f"|d drift| median {np.median(ddr):.3g}")
        assert np.median(ddr) <= 1e-5, k
        assert np.median(l1) <= 2.0 * np.median(l1_ref) + 0.01, k
        assert np.percentile(l1, 90) <= 2.0 * np.percentile(l1_ref, 90) + 0.02, k


def _irregular_map(npx, npy, n_ap, seed):
    """A Voronoi-like regrouping: pixels assigned to the nearest of n_ap seeded
    generators, with a ring of unused (-1) pixels at the corners."""
    rng = np.random.default_rng(seed)
    gx, gy = rng.uniform(0, npx, n_ap), rng.uniform(0, npy, n_ap)
    jx, jy = np.meshgrid(np.arange(npx) + 0.5, np.arange(npy) + 0.5, indexing="ij")
    d2 = (jx[..., None] - gx) ** 2 + (jy[..., None] - gy) ** 2
    m = np.argmin(d2, axis=-1).astype(np.int32)
    r = np.hypot((jx - npx / 2) / (npx / 2), (jy - npy / 2) / (npy / 2))
    m[r > 1.15] = -1
    used = np.unique(m[m >= 0])
    remap = -np.ones(n_ap, dtype=np.int32)
    remap[used] = np.arange(used.size, dtype=np.int32)
    m = np.where(m >= 0, remap[np.maximum(m, 0)], -1).astype(np.int32)
    return m.reshape(-1), int(used.size)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pix2ap_bin_points_bit_exact(gpu, dtype):
    """An irregular pixel -> aperture map with unused pixels: bin indices of random
    points equal the oracle's, and unused pixels report no aperture."""
    import torch
    P = lib()
    npd = np.float64 if dtype == "f64" else np.float32
    pmap, n_ap = _irregular_map(10, 5, 17, seed=3)
    obs = dict(W.SMALL["obs"], pix2ap=pmap, n_ap=n_ap)
    rng = np.random.default_rng(13)
    n = 20000
    pts = np.stack([rng.uniform(-12, 12, n), rng.uniform(-12, 12, n), rng.uniform(-4, 4, n),
                    rng.normal(0, 200, n), rng.normal(0, 200, n), rng.normal(0, 200, n)]).astype(npd)
    euler = W.SMALL["euler"]
    pot = P.build_potential(W.SMALL["components"], 0.0, euler)
    o = P.obs_spec(obs, torch.from_numpy(pmap).to(gpu))
    mass = torch.empty((n, 4), dtype=torch.int32, device=gpu)
    kin = torch.empty_like(mass)
    P.bin_points(pot, o, torch.from_numpy(pts).to(gpu), mass, kin)
    torch.cuda.synchronize()
    om, ok = O.bin_points(O.make_obs(obs, O.euler_matrix(*euler)), pts, dtype)
    assert np.array_equal(mass.cpu().numpy(), om)
    assert np.array_equal(kin.cpu().numpy(), ok)
    assert (ok >= 0).any() and (ok < 0).any() and ok.max() < n_ap * obs["nv"]


@pytest.mark.parametrize("surface", [0, 1])
def test_pix2ap_batched_fp64_identical(gpu, surface):
    """The small model's observables regrouped into 17 irregular apertures (unused
    corner pixels), two potentials in one launch, surface block on and off: the
    whole orbit matrix, overflow, drift and flags equal the oracle's."""
    P = lib()
    n_steps = 300
    pmap, n_ap = _irregular_map(10, 5, 17, seed=3)
    obs = dict(W.SMALL["obs"], pix2ap=pmap, n_ap=n_ap, surface=surface, upsilon=2.0)
    ics, dt = _ics(200, seed=33)
    offs = [0, 90, 200]
    sel = (0, 2)
    pots = [P.build_potential(FP64_POTS[i][0], 0.0, FP64_POTS[i][1]) for i in sel]
    A, ov, dr, fl = _gpu_batched(pots, offs, ics, dt, n_steps, obs, "f64", pix2ap=pmap)
    assert A.shape[1] == 1000 + n_ap * 15 + (n_ap if surface else 0)
    for k, i in enumerate(sel):
        a, b = offs[k], offs[k + 1]
        (c_o, ov_o, dr_o, fl_o), ob = _oracle_one(FP64_POTS[i][0], 0.0, FP64_POTS[i][1], obs, ics[:, a:b], dt[a:b],
                                                  n_steps)
        assert np.array_equal(A[a:b], O.time_fractions(c_o, n_steps, obs=ob)), k
        assert np.array_equal(ov[a:b], ov_o / (4.0 * n_steps)), k
        assert np.array_equal(dr[a:b], dr_o) and np.array_equal(fl[a:b], fl_o), k
    assert ov[:, 1].max() > 0  # unused pixels and the velocity range leave events out
