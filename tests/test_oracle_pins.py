"""Pins of the FP64 oracle against what the mathematics and the paper fix.

Each test checks the oracle against something other than itself: finite
differences of its own potential (forces), Poisson's equation against the
closed-form densities (Eq. 8, Eq. 11, textbook pairs), Gauss's theorem for the
spherical Ferrers limit, closed-form radial periods (Kepler, isochrone),
exact conservation laws of the integrator, orthogonality and special cases of
the Euler rotation (Eq. 1), a brute-force recount of the binning (Sec. 2.2.4,
Table 1), and brute-force / library solutions of the weight problem (Eq. 4).
"""
import math

import numpy as np
import pytest
import scipy.optimize as so

import oracle as O
from oracle import nnls as N

G = O.G


def fd_grad(pot, x, h):
    g = np.zeros(3)
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        g[i] = (O.phi(pot, x + e) - O.phi(pot, x - e)) / (2 * h)
    return g


def fd_laplacian(pot, x, h):
    lap = 0.0
    p0 = O.phi(pot, x)
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        lap += (O.phi(pot, x + e) - 2 * p0 + O.phi(pot, x - e)) / (h * h)
    return lap


COMPONENTS = [
    ("kepler", (1e10,)),
    ("isochrone", (1e10, 1.0)),
    ("plummer", (1e10, 0.5)),
    ("mn", (5e10, 3.0, 0.3)),
    ("nfw_q", (1e12, 10.0, 1.0, 70.0)),
    ("nfw_q", (1e12, 10.0, 0.9, 70.0)),
    ("ferrers2", (1e10, 4.0, 1.5, 1.0)),
    ("da_t3", (1e10, 1.5, 0.5, 3.0, 0.5)),
    ("da_v4", (5e9, 1.0, 0.8, 2.0, -0.3)),
]
POINTS = [np.array(p) for p in ([1.0, 2.0, 0.3], [0.2, -0.1, 0.05], [5.0, -1.0, 0.8], [3.9, 0.2, 0.1],
                                [12.0, 7.0, -4.0], [0.5, 1.4, -0.2])]


@pytest.mark.parametrize("comp", COMPONENTS, ids=lambda c: f"{c[0]}{c[1]}")
def test_force_is_minus_gradient(comp):
    pot = O.make_pot([comp])
    for x in POINTS:
        h = 1e-5 * max(1.0, np.linalg.norm(x))
        g = O.accel(pot, x)
        ref = -fd_grad(pot, x, h)
        assert np.allclose(g, ref, rtol=2e-7, atol=1e-9 * np.abs(ref).max()), (comp, x, g, ref)


@pytest.mark.parametrize("comp", [c for c in COMPONENTS if c[0] != "kepler" and not (c[0] == "nfw_q" and c[1][2] != 1.0)],
                         ids=lambda c: f"{c[0]}{c[1]}")
def test_poisson_equation(comp):
    """laplacian Phi = 4 pi G rho against the closed-form densities."""
    pot = O.make_pot([comp])
    scale = 4 * math.pi * G * O.density(pot, POINTS[1])  # inner-point density sets the absolute scale
    for x in POINTS:
        if comp[0] == "ferrers2":
            m2 = x[0] ** 2 / 16 + x[1] ** 2 / 2.25 + x[2] ** 2
            if abs(m2 - 1) < 0.05:
                continue  # rho is C^1 across the surface; skip the finite-difference kink
        h = 2e-3 * max(0.1, min(1.0, np.linalg.norm(x)))
        lap = fd_laplacian(pot, x, h)
        rho = O.density(pot, x)
        assert lap == pytest.approx(4 * math.pi * G * rho, rel=2e-4, abs=1e-6 * scale), (comp, x)


def test_flattened_nfw_density_positive():
    pot = O.make_pot([("nfw_q", (1e12, 10.0, 0.9, 70.0))])
    for x in POINTS:
        assert fd_laplacian(pot, x, 1e-3) > 0


@pytest.mark.parametrize("q", [0.6, 0.9, 1.4])
def test_nfw_flattening_direction(q):
    """Potential flattening m^2 = x^2 + y^2 + z^2/q^2: the flattened potential at
    height q r on the symmetry axis is the spherical one at r, the midplane is
    unchanged, and the vertical force there is the spherical one divided by q
    (chain rule through m = z/q).  Writing z^2 q^2 instead fails all three."""
    pq = O.make_pot([("nfw_q", (1e12, 10.0, q, 70.0))])
    p1 = O.make_pot([("nfw_q", (1e12, 10.0, 1.0, 70.0))])
    for r in (0.4, 3.0, 25.0, 180.0):
        assert O.phi(pq, np.array([0.0, 0.0, q * r])) == pytest.approx(O.phi(p1, np.array([0.0, 0.0, r])), rel=1e-13)
        gz_q = O.accel(pq, np.array([0.0, 0.0, q * r]))[2]
        gz_1 = O.accel(p1, np.array([0.0, 0.0, r]))[2]
        assert gz_q == pytest.approx(gz_1 / q, rel=1e-12)
        xm = np.array([0.6 * r, -0.8 * r, 0.0])
        assert O.phi(pq, xm) == pytest.approx(O.phi(p1, xm), rel=1e-14)
        np.testing.assert_allclose(O.accel(pq, xm), O.accel(p1, xm), rtol=1e-13, atol=0.0)


def test_ferrers_sphere_matches_gauss_theorem():
    a, M = 2.0, 3e9
    pot = O.make_pot([("ferrers2", (M, a, a, a))])
    rho_c = 105 * M / (32 * math.pi * a ** 3)
    for r in [0.3, 1.0, 1.7, 2.5, 6.0]:
        x = np.array([r / math.sqrt(3)] * 3)
        if r < a:
            Menc = 4 * math.pi * rho_c * (r ** 3 / 3 - 2 * r ** 5 / (5 * a * a) + r ** 7 / (7 * a ** 4))
        else:
            Menc = M
        g = O.accel(pot, x)
        assert np.linalg.norm(g) == pytest.approx(G * Menc / r ** 2, rel=1e-12)
    x = np.array([6.0, 0.0, 0.0])
    assert O.phi(pot, x) == pytest.approx(-G * M / 6.0, rel=1e-12)


def test_ferrers_far_field_and_continuity():
    M = 1e10
    pot = O.make_pot([("ferrers2", (M, 4.0, 1.5, 1.0))])
    x = np.array([300.0, 200.0, 100.0])
    assert O.phi(pot, x) == pytest.approx(-G * M / np.linalg.norm(x), rel=2e-4)
    # continuity across the surface m = 1 along the y axis
    for eps in [1e-7]:
        xi, xo = np.array([0.0, 1.5 - eps, 0.0]), np.array([0.0, 1.5 + eps, 0.0])
        dphi = O.phi(pot, xo) - O.phi(pot, xi)
        assert dphi == pytest.approx(-O.accel(pot, xi)[1] * 2 * eps, rel=1e-3)
        assert O.accel(pot, xi) == pytest.approx(O.accel(pot, xo), rel=1e-6)
    assert O.ferrers_lambda(4.0, 1.5, 1.0, np.array([1.0, 0.5, 0.2])) == 0.0
    lam = O.ferrers_lambda(4.0, 1.5, 1.0, np.array([4.0, 1.5, 0.0]))
    assert lam == pytest.approx(6.0, rel=1e-12)  # closed-form root of 16/(16+l) + 2.25/(2.25+l) = 1


def test_mn_limit_is_plummer_and_nfw_enclosed_mass():
    b = 0.7
    mn = O.make_pot([("mn", (1e10, 0.0, b))])
    pl = O.make_pot([("plummer", (1e10, b))])
    for x in POINTS:
        assert O.phi(mn, x) == pytest.approx(O.phi(pl, x), rel=1e-14)
    Rs, Mdm, R200 = O.nfw_derived(1e12, 10.0)
    assert Rs == pytest.approx(R200 / 10.0)
    # Eq. 9: M(<R) from the circular speed of the spherical potential
    nfw = O.make_pot([("nfw_q", (1e12, 10.0, 1.0, 70.0))])
    for R in [1.0, 10.0, 50.0]:
        g = O.accel(nfw, np.array([R, 0.0, 0.0]))
        Menc = -g[0] * R * R / G
        x = R / Rs
        assert Menc == pytest.approx(Mdm * (math.log(1 + x) - x / (1 + x)), rel=1e-12)
    assert Mdm * (math.log(11) - 10 / 11) == pytest.approx(1e12, rel=1e-12)
    # rho_crit at H0 = 70 and 200 rho_crit mean density inside R200
    rho_crit = 3 * 0.07 ** 2 / (8 * math.pi * G)
    assert 1e12 / (4 / 3 * math.pi * R200 ** 3) == pytest.approx(200 * rho_crit, rel=1e-12)


def radial_period(pot, ic, dt, nsteps):
    tr = O.orbit(pot, ic, dt, nsteps)
    r = np.linalg.norm(tr[:, :3], axis=1)
    # pericentre times by parabolic interpolation of the local minima of r
    idx = np.flatnonzero((r[1:-1] < r[:-2]) & (r[1:-1] <= r[2:])) + 1
    t = []
    for i in idx:
        a, b, c = r[i - 1], r[i], r[i + 1]
        den = a - 2 * b + c
        t.append((i + (0.5 * (a - c) / den if den != 0 else 0.0)) * dt)
    t = np.array(t)
    return np.mean(np.diff(t))


@pytest.mark.parametrize("kind", ["kepler", "isochrone"])
def test_radial_period_closed_form(kind):
    M, b = 1e10, 1.0
    pot = O.make_pot([(kind, (M, b) if kind == "isochrone" else (M,))])
    ic = np.array([3.0, 0.0, 0.0, 0.0, 80.0, 10.0])
    E = O.jacobi(pot, ic)
    Tr = 2 * math.pi * G * M / (-2 * E) ** 1.5
    errs = []
    for steps_per in [400, 800]:
        dt = Tr / steps_per
        errs.append(abs(radial_period(pot, ic, dt, 6 * steps_per) / Tr - 1))
    assert errs[1] < 2e-4
    assert errs[1] < errs[0]


def test_axisymmetric_invariants():
    pot = O.make_pot([("plummer", (1e10, 0.5)), ("mn", (5e10, 3.0, 0.3))], omega=0.0)
    ic = np.array([4.0, 1.0, 0.3, -30.0, 180.0, 25.0])
    tr = O.orbit(pot, ic, 2e-3, 2000)
    Lz = tr[:, 0] * tr[:, 4] - tr[:, 1] * tr[:, 3]
    assert np.max(np.abs(Lz / Lz[0] - 1)) < 1e-12
    # the same orbit in a frame rotating at 40 km/s/kpc: (R, z, |p|, p_z) unchanged
    rot = O.make_pot([("plummer", (1e10, 0.5)), ("mn", (5e10, 3.0, 0.3))], omega=40.0)
    tr2 = O.orbit(rot, ic, 2e-3, 2000)
    for f in (lambda t: np.hypot(t[:, 0], t[:, 1]), lambda t: t[:, 2],
              lambda t: np.linalg.norm(t[:, 3:], axis=1), lambda t: t[:, 5]):
        a, b = f(tr), f(tr2)
        assert np.max(np.abs(a - b)) < 1e-10 * np.max(np.abs(a))  # rounding growth over 2000 steps


def test_time_reversal_and_second_order():
    pot = O.make_pot([("plummer", (1e10, 0.5)), ("mn", (5e10, 3.0, 0.3))])
    ic = np.array([4.0, 1.0, 0.3, -30.0, 180.0, 25.0])
    tr = O.orbit(pot, ic, 1e-3, 3000)
    back = tr[-1].copy()
    back[3:] *= -1
    tb = O.orbit(pot, back, 1e-3, 3000)
    assert np.allclose(tb[-1, :3], ic[:3], atol=1e-10)
    assert np.allclose(-tb[-1, 3:], ic[3:], atol=1e-8)
    errs = []
    for dt in [4e-3, 2e-3]:
        t = O.orbit(pot, ic, dt, int(round(8.0 / dt)))
        E = np.array([O.jacobi(pot, s) for s in t])
        errs.append(np.max(np.abs(E / E[0] - 1)))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_jacobi_integral_conserved_in_bar_frame():
    """Sec. 2.2.2: E_J is the only integral of a rotating bar."""
    comps = [("mn", (4e10, 3.0, 0.3)), ("ferrers2", (1e10, 4.0, 1.5, 1.0)), ("nfw_q", (1e12, 10.0, 0.9, 70.0))]
    pot = O.make_pot(comps, omega=40.0)
    ic = np.array([3.0, 1.0, 0.2, -40.0, 150.0, 10.0])
    drifts = []
    for dt in [2e-4, 1e-4]:
        t = O.orbit(pot, ic, dt, int(round(0.05 / dt)))
        E = np.array([O.jacobi(pot, s) for s in t[::10]])
        drifts.append(np.max(np.abs(E / E[0] - 1)))
    assert drifts[1] < 1e-5
    assert 3.0 < drifts[0] / drifts[1] < 5.0


def test_euler_rotation():
    R = O.euler_matrix(0.3, 1.1, -0.7)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-15)
    assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-15)
    R0 = O.euler_matrix(0.4, 0.0, 0.9)  # face-on: line of sight is the z axis
    assert np.allclose(R0[2], [0, 0, 1], atol=1e-15)
    Re = O.euler_matrix(math.pi / 2, math.pi / 2, 0.0)  # end-on: line of sight along the bar (x)
    assert np.allclose(Re[2], [1, 0, 0], atol=1e-15)
    Rz = O.euler_matrix(0.5, 0.0, 0.0)
    assert np.allclose(Rz, [[math.cos(0.5), -math.sin(0.5), 0], [math.sin(0.5), math.cos(0.5), 0], [0, 0, 1]])


SMALL_OBS = dict(nx=10, ny=10, nz=10, lo=(-10.0, -10.0, -3.0), hi=(10.0, 10.0, 3.0), npx=10, npy=5,
                 plo=(-10.0, -5.0), phi=(10.0, 5.0), pix2ap=None, nv=15, vlo=-450.0, vhi=450.0,
                 symmetrize=1, drift_every=1)


def brute_cells(obs, R, s):
    """Independent restatement of the binning for the recount (floor in FP64)."""
    sg = [(1, 1, 1), (1, 1, -1), (-1, -1, 1), (-1, -1, -1)]
    out = []
    for sx, sy, sz in sg:
        x = np.array([sx * s[0], sy * s[1], sz * s[2]])
        p = np.array([sx * s[3], sy * s[4], sz * s[5]])
        idx = []
        for k, n in enumerate(("nx", "ny", "nz")):
            t = (x[k] - obs["lo"][k]) * (obs[n] / (obs["hi"][k] - obs["lo"][k]))
            idx.append(int(math.floor(t)) if 0 <= t < obs[n] else -1)
        m = -1 if min(idx) < 0 else (idx[0] * obs["ny"] + idx[1]) * obs["nz"] + idx[2]
        X = R[0] @ x
        Y = R[1] @ x
        V = R[2] @ p
        tx = (X - obs["plo"][0]) * (obs["npx"] / (obs["phi"][0] - obs["plo"][0]))
        ty = (Y - obs["plo"][1]) * (obs["npy"] / (obs["phi"][1] - obs["plo"][1]))
        tv = (V - obs["vlo"]) * (obs["nv"] / (obs["vhi"] - obs["vlo"]))
        ok = 0 <= tx < obs["npx"] and 0 <= ty < obs["npy"] and 0 <= tv < obs["nv"]
        k = (int(tx) * obs["npy"] + int(ty)) * obs["nv"] + int(tv) if ok else -1
        out.append((m, k))
    return out


def test_binning_brute_force_recount_and_normalisation():
    pot = O.make_pot([("plummer", (1e10, 0.5)), ("mn", (5e10, 3.0, 0.3))])
    R = O.euler_matrix(math.pi / 4, math.pi / 3, 0.0)
    obs = O.make_obs(SMALL_OBS, R)
    rng = np.random.default_rng(0)
    n, nsteps = 5, 300
    ics = np.stack([rng.uniform(-6, 6, n), rng.uniform(-6, 6, n), rng.uniform(-1, 1, n),
                    rng.normal(0, 100, n), rng.normal(0, 100, n), rng.normal(0, 40, n)])
    dt = np.full(n, 2e-3)
    counts, ov, drift, flags = O.integrate_and_bin(pot, obs, ics, dt, nsteps)
    nm = 1000
    for i in range(n):
        tr = O.orbit(pot, ics[:, i], dt[i], nsteps)
        ref = np.zeros(counts.shape[1], dtype=np.int64)
        om = ok = 0
        for s in tr[1:]:
            for m, k in brute_cells(SMALL_OBS, R, s):
                if m >= 0: ref[m] += 1
                else: om += 1
                if k >= 0: ref[nm + k] += 1
                else: ok += 1
        assert np.array_equal(ref, counts[i])
        assert (om, ok) == tuple(ov[i])
        assert counts[i, :nm].sum() + ov[i, 0] == 4 * nsteps
        assert counts[i, nm:].sum() + ov[i, 1] == 4 * nsteps
        E = np.array([O.jacobi(pot, s) for s in tr])
        assert drift[i] == pytest.approx(np.max(np.abs(E[1:] / E[0] - 1)), rel=1e-12, abs=1e-300)


def test_symmetrised_mass_histogram_is_mirror_invariant():
    """Table 1: with a grid symmetric about the origin the co-added mass
    histogram is invariant under iz -> nz-1-iz and (ix, iy) -> (nx-1-ix, ny-1-iy)."""
    pot = O.make_pot([("mn", (4e10, 3.0, 0.3)), ("ferrers2", (1e10, 4.0, 1.5, 1.0))], omega=40.0)
    obs = O.make_obs(SMALL_OBS, O.euler_matrix(0.3, 1.0, 0.0))
    ics = np.array([[3.0], [0.7], [0.25], [-20.0], [160.0], [15.0]])
    counts, *_ = O.integrate_and_bin(pot, obs, ics, np.array([1e-3]), 400)
    h = counts[0, :1000].reshape(10, 10, 10)
    assert np.array_equal(h, h[:, :, ::-1])
    assert np.array_equal(h, h[::-1, ::-1, :])


def test_bin_edges_are_half_open():
    obs = O.make_obs(SMALL_OBS, np.eye(3))
    # x exactly on the lower edge -> bin 0; exactly on the upper edge -> outside
    pts = np.array([[-10.0, 10.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, -3.0],
                    [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [-450.0, 0.0, 449.0]])
    mass, kin = O.bin_points(obs, pts)
    assert mass[0, 0] == (0 * 10 + 5) * 10 + 5
    assert mass[1, 0] == -1
    assert mass[2, 0] == (5 * 10 + 5) * 10 + 0
    assert kin[0, 0] == (0 * 5 + 2) * 15 + 0 and kin[1, 0] == -1 and kin[2, 0] == (5 * 5 + 2) * 15 + 14
    for prec in ("f64", "f32"):
        m, k = O.bin_points(obs, pts, prec)
        assert np.array_equal(m, mass)


def test_nnls_pins():
    rng = np.random.default_rng(1)
    # brute force == active set == scipy Lawson-Hanson on the augmented system
    for trial in range(5):
        U = rng.random((9, 8)) * (rng.random((9, 8)) < 0.6)
        y = rng.normal(size=9)
        mu = 0.03
        wb = N.nnls_bruteforce(U, y, mu)
        wa = N.nnls_active_set(U.T @ U + mu * np.eye(8), U.T @ y)
        ws, _ = so.nnls(np.vstack([U, math.sqrt(mu) * np.eye(8)]), np.concatenate([y, np.zeros(8)]))
        assert np.allclose(wb, wa, atol=1e-12) and np.allclose(wb, ws, atol=1e-10)
        assert N.kkt_residual(U, y, mu, wb) < 1e-12
    # U = I: w = max(y, 0) / (1 + mu)
    y = rng.normal(size=30)
    w = N.nnls_oracle(np.eye(30), y, 0.5)
    assert np.allclose(w, np.maximum(y, 0) / 1.5, atol=1e-14)
    # a non-negative ridge solution is the NNLS solution
    U = rng.random((40, 20)) + 0.5
    wt = rng.random(20) + 0.1
    y = U @ wt
    mu = 1e-3
    ridge = np.linalg.solve(U.T @ U + mu * np.eye(20), U.T @ y)
    assert np.all(ridge > 0)
    assert np.allclose(N.nnls_oracle(U, y, mu), ridge, atol=1e-10)
    # larger problem: active set vs scipy, KKT certificate
    U = rng.random((200, 300)) * (rng.random((200, 300)) < 0.1)
    y = U @ (rng.exponential(size=300) * (rng.random(300) < 0.1)) + 0.01 * rng.normal(size=200)
    mu = N.relative_mu(U, 1e-2)
    w = N.nnls_oracle(U, y, mu)
    ws, _ = so.nnls(np.vstack([U, math.sqrt(mu) * np.eye(300)]), np.concatenate([y, np.zeros(300)]), maxiter=5000)
    assert np.abs(w - ws).max() < 1e-9 * max(1, np.abs(w).max())
    assert N.kkt_residual(U, y, mu, w) < 1e-12 * np.abs(U.T @ y).max()


def test_chi2_is_zero_at_truth_and_matches_direct_sum():
    rng = np.random.default_rng(2)
    A = rng.random((50, 30))
    w = rng.exponential(size=50)
    d = A.T @ w
    sig = 0.01 * d
    assert N.chi2(A, w, d, sig, 10, 30) < 1e-20  # zero up to summation order
    d2 = d * (1 + 0.02 * rng.normal(size=30))
    direct = sum(((sum(w[i] * A[i, n] for i in range(50)) - d2[n]) / sig[n]) ** 2 for n in range(10, 30))
    assert N.chi2(A, w, d2, sig, 10, 30) == pytest.approx(direct, rel=1e-12)


def test_matrix_free_kkt_and_mu_match_the_scaled_problem():
    """The orbit-matrix forms used at full size (no U formed; dense or CSR A)
    agree with kkt_residual / relative_mu on U = w~ A^T / sigma (pinned above by
    brute force), vanish at the exact minimiser and see a one-weight
    perturbation."""
    import scipy.sparse as sp
    rng = np.random.default_rng(9)
    n, c = 120, 70
    A = rng.random((n, c)) * (rng.random((n, c)) < 0.2)
    d = A.T @ (rng.exponential(size=n) * (rng.random(n) < 0.2)) * (1 + 0.02 * rng.normal(size=c)) + 1e-3
    sig = 0.02 * d
    wt = 0.7
    U, y = N.scale_problem(A, d, sig, wt)
    mu = N.relative_mu(U, 1e-2)
    qmax = np.abs(U.T @ y).max()
    for Am in (A, sp.csr_matrix(A)):
        assert N.relative_mu_orbit_matrix(Am, sig, wt, 1e-2) == pytest.approx(mu, rel=1e-12)
    wp = N.nnls_oracle(U, y, mu)
    for Am in (A, sp.csr_matrix(A)):
        assert N.kkt_residual_orbit_matrix(Am, d, sig, wt, mu, wt * wp) < 1e-12
    w_bad = 1.5 * wp
    w_bad[int(np.argmin(wp))] = 0.5 * wp.max()
    direct = N.kkt_residual(U, y, mu, w_bad) / qmax
    assert direct > 1e3 * 1e-11  # well above the optimum's residual (min(w', g) is capped by the weights' scale)
    for Am in (A, sp.csr_matrix(A)):
        assert N.kkt_residual_orbit_matrix(Am, d, sig, wt, mu, wt * w_bad) == pytest.approx(direct, rel=1e-10)


def test_ferrers_fixed_rule_timing_mode_matches_adaptive():
    """The oracle's fixed 64-point Gauss-Legendre timing mode of the Ferrers
    integrals reproduces the adaptive rule to 1e-12 inside, on and outside the bar."""
    pot = O.make_pot([("ferrers2", (1e10, 4.0, 1.5, 1.0))])
    rng = np.random.default_rng(8)
    pts = np.concatenate([rng.uniform(-1, 1, (60, 3)) * [4, 1.5, 1], rng.uniform(-30, 30, (60, 3)),
                          [[4.0, 0.0, 0.0], [0.0, 1.5, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 0.0]]])
    ref = [(O.phi(pot, x), O.accel(pot, x)) for x in pts]
    O.set_ferrers_rule(64)
    try:
        for x, (p, g) in zip(pts, ref):
            assert O.phi(pot, x) == pytest.approx(p, rel=1e-12)
            np.testing.assert_allclose(O.accel(pot, x), g, rtol=0, atol=1e-12 * max(np.max(np.abs(g)), 1e-300))
    finally:
        O.set_ferrers_rule(0)
