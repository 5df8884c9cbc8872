"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds configuration data and random draws only: potential
parameters, grid geometry, seeded initial conditions, mock-subset draws and
noise.  It contains none of the method's arithmetic (no potential, force,
integration, projection, binning or solve).  Initial conditions are built
from tabulated circular-speed curves stored in ``tables/*.json``; those tables
are written once by ``oracle/make_tables.py`` from the FP64 oracle.

The paper fits an N-body mock IFU cube that is not available here; these
seeded stand-ins follow the paper's shapes where the configurations are
silent (double-exponential fiducial positions with h_R = 3.5 kpc and
h_z = 1.2 kpc, Sec. 2.2.1 and Sec. 3.2.3; a weighted orbit subset as mock).
"""
import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEG = math.pi / 180.0

# Plummer bulge + Miyamoto-Nagai disc, static, 2,000 orbits x 1,000 FP64 steps.
SMALL = dict(
    name="plummer_mn_2k_orbits_1k_steps_f64",
    components=[("plummer", (1e10, 0.5)), ("mn", (5e10, 3.0, 0.3))],
    omega=0.0,
    euler=(45 * DEG, 60 * DEG, 0.0),
    n_orb=2000, n_steps=1000, periods=50.0, dtype="f64",
    obs=dict(nx=10, ny=10, nz=10, lo=(-10.0, -10.0, -3.0), hi=(10.0, 10.0, 3.0),
             npx=10, npy=5, plo=(-10.0, -5.0), phi=(10.0, 5.0), pix2ap=None,
             nv=15, vlo=-450.0, vhi=450.0, symmetrize=1, drift_every=1),
    ic_seed=1, mock=dict(seed=2, frac=0.1, noise=0.0, tol=0.01),
    table="plummer_mn",
    subsample=dict(seed=9, n=2000),
)

# Barred model: MN disc + rotating Ferrers n=2 bar + flattened NFW halo,
# 100,000 orbits x 10,000 FP32 steps, 48,000 constraints.
BARRED = dict(
    name="mn_ferrers_nfwq_100k_orbits_10k_steps_f32",
    components=[("mn", (4e10, 3.0, 0.3)), ("ferrers2", (1e10, 4.0, 1.5, 1.0)),
                ("nfw_q", (1e12, 10.0, 0.9, 70.0))],
    omega=40.0,
    euler=(45 * DEG, 60 * DEG, 0.0),
    n_orb=100000, n_steps=10000, periods=50.0, dtype="f32",
    obs=dict(nx=30, ny=30, nz=20, lo=(-10.0, -10.0, -3.0), hi=(10.0, 10.0, 3.0),
             npx=40, npy=25, plo=(-10.0, -6.25), phi=(10.0, 6.25), pix2ap=None,
             nv=30, vlo=-450.0, vhi=450.0, symmetrize=1, drift_every=10),
    ic_seed=3, mock=dict(seed=4, frac=0.1, noise=0.02, tol=0.02),
    table="barred",
    subsample=dict(seed=9, n=1000),
)

# The 12 parameters varied per walker: disc M,a,b; bar M,a,b,c,Omega; halo M200,c,q; inclination.
THETA_NAMES = ["disc_M", "disc_a", "disc_b", "bar_M", "bar_a", "bar_b", "bar_c", "omega",
               "halo_M200", "halo_c", "halo_q", "incl"]


def theta_nominal(cfg=BARRED):
    (_, (dM, da, db)), (_, (bM, ba, bb, bc)), (_, (hM, hc, hq, _h0)) = cfg["components"]
    return np.array([dM, da, db, bM, ba, bb, bc, cfg["omega"], hM, hc, hq, cfg["euler"][1]])


def theta_to_model(theta, cfg=BARRED):
    """12-vector -> (components, omega, euler) in the barred family."""
    t = [float(v) for v in theta]
    comps = [("mn", (t[0], t[1], t[2])), ("ferrers2", (t[3], t[4], t[5], t[6])),
             ("nfw_q", (t[8], t[9], t[10], 70.0))]
    return comps, t[7], (cfg["euler"][0], t[11], cfg["euler"][2])


def load_table(name):
    with open(os.path.join(HERE, "tables", name + ".json")) as f:
        t = json.load(f)
    for k in ("R", "Phi", "vc", "Ec"):
        t[k] = np.asarray(t[k], dtype=np.float64)
    return t


def grid_ics(table, n_energy=20, n_eta=10, n_psi=10, seed=1, n_steps=1000, periods=50.0):
    """Uniform energy grid x circularity x start angle (E_c between the
    circular orbits at 0.5 and 10 kpc).  Each orbit starts in the midplane at
    the circular radius of its energy, azimuth drawn from the seed, with
    v_phi = eta v_c and the remaining kinetic energy split between v_R and v_z
    by the start angle.  dt = periods * T_c / n_steps."""
    R, vc, Ec = table["R"], table["vc"], table["Ec"]
    rng = np.random.default_rng(seed)
    E_lo, E_hi = np.interp(0.5, R, Ec), np.interp(10.0, R, Ec)
    n = n_energy * n_eta * n_psi
    phi0 = rng.uniform(0.0, 2 * math.pi, size=n)
    ics = np.zeros((6, n))
    dt = np.zeros(n)
    i = 0
    for j in range(n_energy):
        E = E_lo + (j + 0.5) * (E_hi - E_lo) / n_energy
        Rc = float(np.interp(E, Ec, R))
        v = float(np.interp(Rc, R, vc))
        Tc = 2 * math.pi * Rc / v
        for k in range(n_eta):
            eta = (k + 0.5) / n_eta
            vphi = eta * v
            vrest = math.sqrt(max(0.0, (1 - eta * eta)) * v * v)
            for l in range(n_psi):
                psi = (l + 0.5) / n_psi * (math.pi / 2)
                vR, vz = vrest * math.cos(psi), vrest * math.sin(psi)
                c, s = math.cos(phi0[i]), math.sin(phi0[i])
                ics[:, i] = (Rc * c, Rc * s, 0.0, vR * c - vphi * s, vR * s + vphi * c, vz)
                dt[i] = periods * Tc / n_steps
                i += 1
    return ics, dt


def disc_ics(table, n, seed=3, n_steps=10000, periods=50.0, h_R=3.5, h_z=1.2, R_max=15.0, z_max=5.0):
    """Positions from p(R, z) ~ R exp(-R/h_R) exp(-|z|/h_z) (truncated),
    uniform azimuth; inertial velocities v_phi ~ N(0.9 v_c, 0.25 v_c),
    v_R ~ N(0, 0.25 v_c), v_z ~ N(0, 0.15 v_c) with v_c the azimuth-averaged
    midplane circular speed at the starting radius; dt = periods T_c(R) / n_steps."""
    rng = np.random.default_rng(seed)
    Rs = np.empty(0)
    while Rs.size < n:
        r = rng.gamma(2.0, h_R, size=2 * n)
        Rs = np.concatenate([Rs, r[(r < R_max) & (r > 1e-3)]])
    Rs = Rs[:n]
    zs = np.empty(0)
    while zs.size < n:
        z = rng.laplace(0.0, h_z, size=2 * n)
        zs = np.concatenate([zs, z[np.abs(z) < z_max]])
    zs = zs[:n]
    ph = rng.uniform(0.0, 2 * math.pi, size=n)
    v = np.interp(Rs, table["R"], table["vc"])
    vphi = rng.normal(0.9, 0.25, size=n) * v
    vR = rng.normal(0.0, 0.25, size=n) * v
    vz = rng.normal(0.0, 0.15, size=n) * v
    c, s = np.cos(ph), np.sin(ph)
    ics = np.stack([Rs * c, Rs * s, zs, vR * c - vphi * s, vR * s + vphi * c, vz])
    dt = periods * (2 * math.pi * Rs / v) / n_steps
    return ics, dt


def disc_positions(n, seed=3, h_R=3.5, h_z=1.2, R_max=15.0, z_max=5.0):
    """Starting positions [3][n] from the fiducial p(R, z) ~ R exp(-R/h_R)
    exp(-|z|/h_z) truncated at R_max, z_max, uniform azimuth, and the standard
    normal deviates [3][n] of their velocity draws (v_R, v_phi, v_z)."""
    rng = np.random.default_rng(seed + 500)
    Rs = np.empty(0)
    while Rs.size < n:
        r = rng.gamma(2.0, h_R, size=2 * n)
        Rs = np.concatenate([Rs, r[(r < R_max) & (r > 1e-3)]])
    zs = np.empty(0)
    while zs.size < n:
        z = rng.laplace(0.0, h_z, size=2 * n)
        zs = np.concatenate([zs, z[np.abs(z) < z_max]])
    Rs, zs = Rs[:n], zs[:n]
    ph = rng.uniform(0.0, 2 * math.pi, size=n)
    return np.stack([Rs * np.cos(ph), Rs * np.sin(ph), zs]), rng.standard_normal((3, n))


def dither_deviates(n_dither, n, seed=5):
    """Uniform deviates on [-1/2, 1/2) [n_dither][6][n] placing each initial
    condition's realisations in the box around it."""
    return np.random.default_rng(seed + 700).uniform(-0.5, 0.5, size=(n_dither, 6, n))


def mock_draw(n_orb, seed, frac=0.1):
    """Seeded subset of round(frac N) orbits with weights ~ Exp(1)."""
    rng = np.random.default_rng(seed)
    k = int(round(frac * n_orb))
    idx = np.sort(rng.choice(n_orb, size=k, replace=False))
    w = np.zeros(n_orb)
    w[idx] = rng.exponential(1.0, size=k)
    return w


def noise_draw(n, seed):
    return np.random.default_rng(seed + 1000).normal(size=n)


def bootstrap_eps(n_rhs, n_con, seed=9):
    """Standard normal deviates [n_rhs][n_con] for the bootstrap realisations of the data."""
    return np.random.default_rng(seed + 2000).normal(size=(n_rhs, n_con))


def subsample_draw(n_orb, n, seed):
    return np.sort(np.random.default_rng(seed).choice(n_orb, size=n, replace=False))


def walker_thetas(n=64, seed=5, spread=0.3, cfg=BARRED):
    rng = np.random.default_rng(seed)
    return theta_nominal(cfg)[None, :] * rng.uniform(1 - spread, 1 + spread, size=(n, 12))


def walker_orbit_counts(n=64, seed=5, lo=20000, hi=150000):
    return np.random.default_rng(seed + 1).integers(lo, hi + 1, size=n)


def latin_hypercube(n, d, seed=7):
    """McKay et al. (1979): one point per stratum per dimension, strata
    matched by independent seeded permutations; values in (0, 1)."""
    rng = np.random.default_rng(seed)
    u = (rng.permuted(np.tile(np.arange(n), (d, 1)), axis=1).T + rng.uniform(size=(n, d))) / n
    return u


def sparse_lognormal_matrix(n_orb, blocks, density=0.05, seed=6, dtype=np.float32):
    """Synthetic orbit matrix [n_orb][n_con]: each entry nonzero with
    probability `density`, value LogNormal(0, 1), each orbit's row normalised
    to sum 1 within every block."""
    rng = np.random.default_rng(seed)
    n_con = blocks[-1][1]
    A = np.zeros((n_orb, n_con), dtype=np.float64)
    for b0, b1 in blocks:
        m = rng.random((n_orb, b1 - b0)) < density
        v = np.where(m, rng.lognormal(0.0, 1.0, size=(n_orb, b1 - b0)), 0.0)
        s = v.sum(axis=1, keepdims=True)
        s[s == 0] = 1.0
        A[:, b0:b1] = v / s
    return A.astype(dtype)


def ncon(obs):
    n_ap = obs["n_ap"] if obs.get("pix2ap") is not None else obs["npx"] * obs["npy"]
    return obs["nx"] * obs["ny"] * obs["nz"] + n_ap * obs["nv"]


def blocks(obs):
    nm = obs["nx"] * obs["ny"] * obs["nz"]
    return [(0, nm), (nm, ncon(obs))]


# The paper's own pipeline (Sec. 2.2-2.4, Sec. 3.2.3) on the barred model: 7,500
# Jeans initial conditions x 4 dithers, BS23 (rtol 1e-4) for 5,000 accepted
# steps, a 600-cell cylindrical density grid, ~600 irregular apertures of a
# 60 x 40 pixel grid with 30 velocity bins, the surface-density block, and
# 100 bootstrap realisations of the maps.  rho: the ADMM penalty of the weight
# solves as a multiple of trace(U U^T)/N.
PAPER = dict(
    name="paper_pipeline_barred_7500x4_bs23_5k_steps_f64",
    n_ic=7500, n_dither=4, n_steps=5000, rtol=1e-4, atol=1e-6, h0=2e-3, dx=0.1, fv=0.05, h_R=3.5, h_z=1.2,
    jeans_b=1.0, n_boot=100, n_gh=4, dh=0.02, stellar_mask=0b011, n_sub=4, rho=0.5,
    obs=dict(nx=10, ny=6, nz=10, lo=(0.0, -math.pi, -3.0), hi=(10.0, math.pi, 3.0), grid="cylindrical",
             npx=60, npy=40, plo=(-10.0, -20.0 / 3.0), phi=(10.0, 20.0 / 3.0),
             nv=30, vlo=-450.0, vhi=450.0, symmetrize=1, drift_every=1, surface=1, upsilon=1.0),
    n_gen=880, ap_scale=6.0, ap_seed=23, ic_seed=21, mock=dict(seed=22, frac=0.1, tol=0.01, noise=0.01),
)


def voronoi_map(npx, npy, plo, phi, n_gen, seed, scale=3.0):
    """A stand-in for the paper's Voronoi apertures (its PowerBin binning of an
    IFU field is not available): n_gen seeded generators, denser towards the
    centre (exponential in radius with the given scale, uniform angle), each
    pixel of the npx x npy grid assigned to its nearest generator; generators
    with no pixel are dropped and the rest renumbered in order.  Returns
    (map [npx * npy] int32, pixel (jX, jY) at jX * npy + jY; number of apertures)."""
    rng = np.random.default_rng(seed + 3000)
    r = rng.exponential(scale, size=4 * n_gen)
    t = rng.uniform(0.0, 2 * math.pi, size=4 * n_gen)
    gx, gy = r * np.cos(t), r * np.sin(t)
    keep = (gx >= plo[0]) & (gx < phi[0]) & (gy >= plo[1]) & (gy < phi[1])
    gx, gy = gx[keep][:n_gen], gy[keep][:n_gen]
    px = plo[0] + (np.arange(npx) + 0.5) * (phi[0] - plo[0]) / npx
    py = plo[1] + (np.arange(npy) + 0.5) * (phi[1] - plo[1]) / npy
    X, Y = np.meshgrid(px, py, indexing="ij")
    d2 = (X.reshape(-1, 1) - gx[None, :]) ** 2 + (Y.reshape(-1, 1) - gy[None, :]) ** 2
    near = np.argmin(d2, axis=1)
    used = np.unique(near)
    remap = np.full(gx.size, -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    return remap[near].astype(np.int32), int(used.size)
