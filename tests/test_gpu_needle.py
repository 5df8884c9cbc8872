"""GPU parity of the Dehnen-Aly needle bars (Eq. 12, App. A) against the
oracle, which integrates the needle adaptively (Gauss-Kronrod to 1e-14)
where the library uses a fixed Gauss-Legendre rule after a sinh change of
variable: the two forces agree to ~1e-13 in double precision, so double
trajectories agree closely (not to the bit), single ones to single-precision
accuracy, and the binned orbit matrices of a short double run are identical
except for rare events that sit on a bin edge.
"""
import numpy as np
import pytest

import oracle as O
from tests.gpu_common import lib

pytestmark = pytest.mark.gpu

COMPS = [("mn", (4e10, 3.0, 0.3)), ("da_t3", (8e9, 1.5, 0.6, 3.5, 0.4)), ("da_v4", (3e9, 1.0, 0.8, 2.0, -0.3))]
OMEGA = 40.0


def _ics(n, seed):
    rng = np.random.default_rng(seed)
    R = rng.uniform(0.5, 8.0, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    v = 200.0 + rng.normal(0, 20, n)
    ics = np.stack([R * np.cos(ph), R * np.sin(ph), rng.normal(0, 0.3, n),
                    -v * np.sin(ph) + rng.normal(0, 20, n), v * np.cos(ph) + rng.normal(0, 20, n),
                    rng.normal(0, 15, n)])
    dt = np.full(n, 2e-4)
    return ics, dt


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_needle_orbits_match_oracle(gpu, dtype):
    import torch
    P = lib()
    n, n_steps = 96, 300
    ics, dt = _ics(n, 3)
    pot = P.build_potential(COMPS, OMEGA, (0.0, 0.0, 0.0))
    td = torch.float64 if dtype == "f64" else torch.float32
    out = torch.empty((6, n), dtype=td, device=gpu)
    P.integrate_orbits(pot, torch.from_numpy(ics).to(gpu, td), torch.from_numpy(dt).to(gpu, td), n_steps, out)
    torch.cuda.synchronize()
    g = out.double().cpu().numpy()
    opot = O.make_pot(COMPS, OMEGA)
    err = []
    for i in range(n):
        ref = O.orbit(opot, ics[:, i], dt[i], n_steps)[-1]
        scale = np.array([np.linalg.norm(ref[:3])] * 3 + [np.linalg.norm(ref[3:])] * 3)
        err.append(np.max(np.abs(g[:, i] - ref) / scale))
    err = np.array(err)
    print(dtype, "max relative state error", err.max(), "median", np.median(err))
    assert np.all(np.isfinite(g))
    assert err.max() < (1e-11 if dtype == "f64" else 2e-4)


def test_needle_binned_matrix_matches_oracle(gpu):
    import torch
    P = lib()
    n, n_steps = 256, 200
    ics, dt = _ics(n, 4)
    obs = dict(nx=8, ny=8, nz=4, lo=(-8, -8, -2), hi=(8, 8, 2), npx=8, npy=6, plo=(-8, -6), phi=(8, 6),
               nv=12, vlo=-360, vhi=360, symmetrize=1, drift_every=10)
    euler = (0.6, 1.0, 0.2)
    pot = P.build_potential(COMPS, OMEGA, euler)
    o = P.obs_spec(obs)
    nc = P.ncon(o)
    A = torch.empty((n, nc), dtype=torch.float64, device=gpu)
    ov = torch.empty((n, 2), dtype=torch.float64, device=gpu)
    dr = torch.empty(n, dtype=torch.float64, device=gpu)
    fl = torch.empty(n, dtype=torch.uint8, device=gpu)
    ws = torch.empty(P.integrate_workspace_bytes(o, 1, n, n_steps, P.SW_F64), dtype=torch.uint8, device=gpu)
    P.integrate_and_bin(pot, [0, n], torch.from_numpy(ics).to(gpu), torch.from_numpy(dt).to(gpu), n_steps, o, A, ov,
                        dr, fl, ws)
    torch.cuda.synchronize()
    opot = O.make_pot(COMPS, OMEGA)
    oobs = O.make_obs(obs, O.euler_matrix(*euler))
    c_o, ov_o, dr_o, fl_o = O.integrate_and_bin(opot, oobs, ics, dt, n_steps)
    A_o = O.time_fractions(c_o, n_steps)
    A_g = A.cpu().numpy()
    same = np.all(A_g == A_o, axis=1)
    l1 = np.abs(A_g - A_o).sum(axis=1)
    print("identical rows", same.mean(), "max row L1", l1.max())
    assert same.mean() >= 0.95
    assert l1.max() <= 4 * 2 / (4 * n_steps)  # at most a few events moved to a neighbouring bin
    assert np.allclose(dr.cpu().numpy(), dr_o, rtol=1e-6, atol=1e-12)
