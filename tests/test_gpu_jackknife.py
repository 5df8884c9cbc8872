"""GPU parity of the aperture jackknife (Sec. 2.4: Delta chi^2 of Eq. 7) against
the oracle (`oracle/jackknife.py`): the small model's orbit matrix (bit-exact
from both sides), a noisy mock, the drift-flagged orbits masked, and one weight
solve per aperture without that aperture's data, the full problem's mu held
fixed.  Bar: each chi^2_a within 1e-3 relative (the chi^2 tolerance of the
build), Delta chi^2 within 1e-2 relative."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import jackknife as J
from oracle import nnls as N
from tests.gpu_common import gpu_integrate, lib, oracle_integrate

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("surface", [0, 1])
def test_jackknife_matches_oracle(gpu, surface):
    import torch
    P = lib()
    from paper_2607_00117_amd import jackknife as JK
    cfg = W.SMALL
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=1000)
    sel = np.arange(0, 2000, 5)
    ics, dt = ics[:, sel], dt[sel]
    n, n_steps = ics.shape[1], 300
    obs = dict(cfg["obs"], surface=surface, upsilon=1.0)
    A_g, _, _, fl_g = gpu_integrate(cfg, ics, dt, n_steps, "f64", obs=obs)
    c_o, _, _, fl_o = oracle_integrate(cfg, ics, dt, n_steps, obs=obs)
    oobs = O.make_obs(obs, O.euler_matrix(*cfg["euler"]))
    A_o = O.time_fractions(c_o, n_steps, obs=oobs)
    assert np.array_equal(A_g, A_o) and np.array_equal(fl_g, fl_o)
    n_mass, n_ap, nv = 1000, 50, 15
    kin0 = n_mass
    surf0 = kin0 + n_ap * nv if surface else None
    nc = A_o.shape[1]
    w_true = W.mock_draw(n, 2)
    d = A_o.T @ w_true * (1 + 0.02 * W.noise_draw(nc, 2))
    sig = N.sigma_from_data(d, [(0, n_mass), (n_mass, nc)], 0.02)
    wt = N.w_tilde_from_data(d, (0, n_mass), n)
    mask_o = (fl_o & 1).astype(np.uint8)
    rows = np.flatnonzero(mask_o == 0)
    mu_o = N.relative_mu(N.scale_problem(A_o[rows], d, sig, wt)[0], 1e-2)
    dchi_o, chis_o, _ = J.jackknife(A_o, d, sig, wt, mu_o, kin0, n_ap, nv, surf0=surf0, mask=mask_o)

    dev = torch.device("cuda:0")
    A_t = torch.from_numpy(A_g).to(dev)
    d_t, s_t = torch.from_numpy(d).to(dev), torch.from_numpy(sig).to(dev)
    mask_t = torch.from_numpy((fl_g & 1).astype(np.uint8)).to(dev)
    opts = P._lib.SolveOpts()
    opts.gram, opts.nu = P.SW_GRAM_BF16X3, 1e-2
    opts.mask = mask_t.data_ptr()
    w = torch.empty(n, dtype=torch.float64, device=dev)
    ws = torch.empty(P.solve_workspace_bytes(n, nc, opts), dtype=torch.uint8, device=dev)
    st, rep = P.solve_weights(A_t, d_t, s_t, wt, -1.0, opts, w, ws)
    assert rep.mu == pytest.approx(mu_o, rel=1e-4)  # the library takes mu from the trace of its fp32 Gram
    opts.mask = None
    dchi_g, chis_g, st_j, reps = JK.jackknife_dchi2(A_t, d_t, s_t, wt, rep.mu, kin0, n_ap, nv, surf0=surf0,
                                                    mask=mask_t, opts=opts)
    torch.cuda.synchronize()
    print(f"surface {surface}: dchi2 gpu {dchi_g:.6g} oracle {dchi_o:.6g}; chi2_a max rel err "
          f"{np.max(np.abs(chis_g / chis_o - 1)):.2e}; status {st_j}, kkt max {max(r.kkt for r in reps):.2e}")
    assert st_j == 0
    np.testing.assert_allclose(chis_g, chis_o, rtol=1e-3)
    assert dchi_g == pytest.approx(dchi_o, rel=1e-2)
    assert dchi_o > 0
