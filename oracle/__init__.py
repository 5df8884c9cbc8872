"""FP64 CPU oracle for the Schwarzschild model-build hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg.  The product path never imports it, and it
imports nothing from the product package.

The orbit integration, symmetrisation, projection and binning live in the
plain C library ``schw_oracle.c`` (double precision, no FMA contraction);
this module wraps it with ctypes.  The weight solve, chi^2, Gauss-Hermite
moments, the MLP and the delayed-acceptance sampler are plain NumPy in the
sibling modules.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

KINDS = {"kepler": 1, "isochrone": 2, "plummer": 3, "mn": 4, "nfw_q": 5, "ferrers2": 6, "da_t3": 7, "da_v4": 8}
G = 4.300917270e-6

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        src = os.path.join(_build.HERE, "schw_oracle.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        _lib = C.CDLL(path)
        _declare(_lib)
    return _lib


class _Comp(C.Structure):
    _fields_ = [("kind", C.c_int), ("p", C.c_double * 8)]


class _Pot(C.Structure):
    _fields_ = [("ncomp", C.c_int), ("comp", _Comp * 8), ("omega", C.c_double)]


class _Obs(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("npx", C.c_int), ("npy", C.c_int),
                ("plo", C.c_double * 2), ("phi", C.c_double * 2),
                ("pix2ap", C.POINTER(C.c_int32)), ("n_ap", C.c_int),
                ("nv", C.c_int), ("vlo", C.c_double), ("vhi", C.c_double),
                ("R", C.c_double * 9), ("symmetrize", C.c_int), ("drift_every", C.c_int), ("grid", C.c_int),
                ("surface", C.c_int), ("upsilon", C.c_double)]


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_i32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def _declare(L):
    P, O = C.POINTER(_Pot), C.POINTER(_Obs)
    L.orc_phi.argtypes = [P, _dp]; L.orc_phi.restype = C.c_double
    L.orc_accel.argtypes = [P, _dp, _dp]; L.orc_accel.restype = None
    L.orc_density.argtypes = [P, _dp]; L.orc_density.restype = C.c_double
    L.orc_jeans.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_long, _dp, _dp, _dp, _dp]; L.orc_jeans.restype = None
    L.orc_orbit_bs23.argtypes = [P, _dp, C.c_double, C.c_int, C.c_double, C.c_double, _dp, _dp]
    L.orc_orbit_bs23.restype = None
    L.orc_integrate_bs23_and_bin.argtypes = [P, C.POINTER(_Obs), C.c_long, _dp, _dp, C.c_int, C.c_double, C.c_double,
                                             _dp, _dp, _dp, _u8, C.c_int]
    L.orc_integrate_bs23_and_bin.restype = None
    L.orc_cell_mass.argtypes = [P, C.POINTER(_Obs), C.c_int, C.c_double, C.c_double]; L.orc_cell_mass.restype = C.c_double
    L.orc_jacobi.argtypes = [P, _dp]; L.orc_jacobi.restype = C.c_double
    L.orc_ferrers_lambda.argtypes = [C.c_double, C.c_double, C.c_double, _dp]
    L.orc_ferrers_lambda.restype = C.c_double
    L.orc_set_ferrers_rule.argtypes = [C.c_int]
    L.orc_set_ferrers_rule.restype = C.c_int
    L.orc_nfw_derived.argtypes = [C.c_double, C.c_double, C.c_double, _dp]; L.orc_nfw_derived.restype = None
    L.orc_euler_matrix.argtypes = [C.c_double, C.c_double, C.c_double, _dp]; L.orc_euler_matrix.restype = None
    L.orc_step.argtypes = [P, _dp, C.c_double]; L.orc_step.restype = None
    L.orc_orbit.argtypes = [P, _dp, C.c_double, C.c_int, _dp]; L.orc_orbit.restype = None
    L.orc_ncon.argtypes = [O]; L.orc_ncon.restype = C.c_int
    L.orc_integrate_and_bin.argtypes = [P, O, C.c_long, _dp, _dp, C.c_int, _i32, _i64, _dp, _u8, C.c_int]
    L.orc_integrate_and_bin.restype = None
    L.orc_integrate_and_bin_f32state.argtypes = L.orc_integrate_and_bin.argtypes
    L.orc_integrate_and_bin_f32state.restype = None
    L.orc_bin_points_f64.argtypes = [O, C.c_long, _dp, _i32, _i32]; L.orc_bin_points_f64.restype = None
    L.orc_bin_points_f32.argtypes = [O, C.c_long, _fp, _i32, _i32]; L.orc_bin_points_f32.restype = None


def make_pot(components, omega=0.0):
    """components: list of (kind_name, params tuple) in the kind's slot order."""
    p = _Pot()
    p.ncomp = len(components)
    for i, (kind, params) in enumerate(components):
        p.comp[i].kind = KINDS[kind]
        for j, v in enumerate(params):
            p.comp[i].p[j] = float(v)
    p.omega = float(omega)
    return p


def euler_matrix(alpha, beta, gamma):
    R = np.zeros(9)
    lib().orc_euler_matrix(alpha, beta, gamma, R)
    return R.reshape(3, 3)


def make_obs(spec, R):
    """spec: dict with keys nx, ny, nz, lo, hi, npx, npy, plo, phi, pix2ap (array or None),
    n_ap, nv, vlo, vhi, symmetrize, drift_every.  R: 3x3 projection matrix."""
    o = _Obs()
    o.nx, o.ny, o.nz = spec["nx"], spec["ny"], spec["nz"]
    for i in range(3):
        o.lo[i], o.hi[i] = spec["lo"][i], spec["hi"][i]
    o.npx, o.npy = spec["npx"], spec["npy"]
    for i in range(2):
        o.plo[i], o.phi[i] = spec["plo"][i], spec["phi"][i]
    m = spec.get("pix2ap")
    if m is not None:
        m = np.ascontiguousarray(m, dtype=np.int32)
        o.pix2ap = m.ctypes.data_as(C.POINTER(C.c_int32))
        o._keep = m
        o.n_ap = int(spec["n_ap"])
    else:
        o.pix2ap = C.POINTER(C.c_int32)()
        o.n_ap = spec["npx"] * spec["npy"]
    o.nv, o.vlo, o.vhi = spec["nv"], spec["vlo"], spec["vhi"]
    R = np.asarray(R, dtype=np.float64).reshape(9)
    for i in range(9):
        o.R[i] = R[i]
    o.symmetrize = int(spec.get("symmetrize", 1))
    o.drift_every = int(spec.get("drift_every", 1))
    o.grid = 1 if spec.get("grid", "cartesian") == "cylindrical" else 0
    o.surface = int(spec.get("surface", 0))
    o.upsilon = float(spec.get("upsilon", 1.0))
    return o


def phi(pot, x):
    return lib().orc_phi(C.byref(pot), np.ascontiguousarray(x, dtype=np.float64))


def accel(pot, x):
    g = np.zeros(3)
    lib().orc_accel(C.byref(pot), np.ascontiguousarray(x, dtype=np.float64), g)
    return g


def density(pot, x):
    return lib().orc_density(C.byref(pot), np.ascontiguousarray(x, dtype=np.float64))


def cell_masses(pot, obs, cells=None, rel_tol=1e-10, abs_tol=0.0):
    """Target cell masses m*_n (Sec. 2.2.4): the mass of pot's density (every
    component of pot) in each mass-grid cell of obs, by nested adaptive
    Gauss-Kronrod to rel_tol of each piece or its share of abs_tol [M_sun]
    per cell.  cells: indices to evaluate (default: all)."""
    n = obs.nx * obs.ny * obs.nz
    idx = range(n) if cells is None else cells
    return np.array([lib().orc_cell_mass(C.byref(pot), C.byref(obs), int(c), rel_tol, abs_tol) for c in idx])


def jeans_ics(pot, pos, eps, h_R, h_z, b=1.0):
    """Jeans-equation initial conditions (Sec. 2.2.1) at positions pos [3][n]:
    returns (moments [5][n] = sigma_R, sigma_phi, sigma_z, mean v_phi, v_c; ics [6][n])."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    n = pos.shape[1]
    mom = np.zeros((5, n))
    ics = np.zeros((6, n))
    lib().orc_jeans(C.byref(pot), h_R, h_z, b, n, pos, eps, mom, ics)
    return mom, ics


def jacobi(pot, s):
    return lib().orc_jacobi(C.byref(pot), np.ascontiguousarray(s, dtype=np.float64))


def ferrers_lambda(a, b, c, x):
    return lib().orc_ferrers_lambda(a, b, c, np.ascontiguousarray(x, dtype=np.float64))


def set_ferrers_rule(n):
    """Timing mode of the Ferrers integrals: a fixed n-point Gauss-Legendre rule
    (n <= 128) instead of the adaptive one (n = 0, the default)."""
    if lib().orc_set_ferrers_rule(int(n)) != 0:
        raise ValueError(f"bad Ferrers rule {n}")


def nfw_derived(M200, c, H0=70.0):
    out = np.zeros(3)
    lib().orc_nfw_derived(M200, c, H0, out)
    return out  # R_s, M_DM, R200


def orbit(pot, ic, dt, nsteps):
    traj = np.zeros((nsteps + 1, 6))
    lib().orc_orbit(C.byref(pot), np.ascontiguousarray(ic, dtype=np.float64), dt, nsteps, traj)
    return traj


def ncon(obs):
    return lib().orc_ncon(C.byref(obs))


def integrate_and_bin(pot, obs, ics, dt, nsteps, nthreads=0, f32_state=False):
    """ics: [6][n] float64; dt: [n].  Returns (counts [n][ncon] int32,
    overflow [n][2] int64, drift [n], flags [n] uint8).  f32_state rounds the
    state to binary32 after every step (FP64 arithmetic otherwise)."""
    ics = np.ascontiguousarray(ics, dtype=np.float64)
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    n = ics.shape[1]
    nc = ncon(obs)
    counts = np.zeros((n, nc), dtype=np.int32)
    ov = np.zeros((n, 2), dtype=np.int64)
    drift = np.zeros(n)
    flags = np.zeros(n, dtype=np.uint8)
    fn = lib().orc_integrate_and_bin_f32state if f32_state else lib().orc_integrate_and_bin
    fn(C.byref(pot), C.byref(obs), n, ics, dt, nsteps, counts, ov, drift, flags, nthreads)
    return counts, ov, drift, flags


def orbit_bs23(pot, ic, h0, nsteps, rtol, atol):
    """Adaptive BS23 orbit: (traj [nsteps+1][6], dts [nsteps])."""
    traj = np.zeros((nsteps + 1, 6))
    dts = np.zeros(nsteps)
    lib().orc_orbit_bs23(C.byref(pot), np.ascontiguousarray(ic, dtype=np.float64), float(h0), int(nsteps),
                         float(rtol), float(atol), traj, dts)
    return traj, dts


def integrate_bs23_and_bin(pot, obs, ics, h0, nsteps, rtol, atol, nthreads=0):
    """Adaptive BS23 with time-weighted binning: (A [n][ncon] fractions,
    overflow [n][2] fractions, drift [n], flags [n])."""
    ics = np.ascontiguousarray(ics, dtype=np.float64)
    n = ics.shape[1]
    A = np.zeros((n, ncon(obs)))
    ov = np.zeros((n, 2))
    drift = np.zeros(n)
    flags = np.zeros(n, dtype=np.uint8)
    lib().orc_integrate_bs23_and_bin(C.byref(pot), C.byref(obs), n, ics, np.ascontiguousarray(h0, dtype=np.float64),
                                     int(nsteps), float(rtol), float(atol), A, ov, drift, flags, nthreads)
    return A, ov, drift, flags


def bin_points(obs, pts, precision="f64"):
    """pts: [6][n] phase-space points on the bar axes.  Returns (mass, kin) [n][4] int32."""
    n = pts.shape[1]
    mass = np.zeros((n, 4), dtype=np.int32)
    kin = np.zeros((n, 4), dtype=np.int32)
    if precision == "f64":
        lib().orc_bin_points_f64(C.byref(obs), n, np.ascontiguousarray(pts, dtype=np.float64), mass, kin)
    else:
        lib().orc_bin_points_f32(C.byref(obs), n, np.ascontiguousarray(pts, dtype=np.float32), mass, kin)
    return mass, kin


def time_fractions(counts, nsteps, symmetrize=True, obs=None):
    """Sec. 2.2.4: each sample carries weight dt / t_total = 1 / nsteps, split
    over the mirror copies.  With obs's surface block on, that block (the last
    n_ap columns) is the surface luminosity, the mass fraction divided by the
    mass-to-light ratio upsilon."""
    A = counts / float((4 if symmetrize else 1) * nsteps)
    if obs is not None and obs.surface:
        A[:, A.shape[1] - obs.n_ap:] /= obs.upsilon
    return A
