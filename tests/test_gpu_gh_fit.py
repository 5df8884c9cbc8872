"""GPU parity of the weight problem with Gauss-Hermite kinematics (Sec. 2.2.4,
Eq. 2-3, Eq. 5): the small model's orbit matrix with the surface block
(bit-exact from both sides), the fit matrix [density | Sigma | h_1..h_4] built
by gh_fit_matrix against the oracle's (closed-form bin integrals against
64-point Gauss-Legendre: 1e-10 relative), then the NNLS of Eq. 3 on it and
chi^2 of Eq. 5 over Sigma + GH against the oracle's exact solve (weights L1 <
1e-2, chi^2 < 1e-3 relative).

Mock (a stand-in for the paper's IFU maps): a seeded 10% orbit subset with
Exp(1) weights; Sigma* its surface block; the reference Gaussian of each
aperture its LOSVD's mean and dispersion; h* its h_m for the observed
luminosity gamma* = Sigma* plus Gaussian noise of Delta h* = 0.02; density and
Sigma at 1% (Eq. 3)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import gh as GH
from oracle import nnls as N
from tests.gpu_common import gpu_integrate, lib, oracle_integrate

pytestmark = pytest.mark.gpu


def _mock_maps(A_o, w_true, n_mass, kin0, surf0, n_ap, nv, vlo, vhi):
    d = A_o.T @ w_true
    sig_star = d[surf0:surf0 + n_ap]
    gamma = np.maximum(sig_star, 1e-3 * sig_star.max())
    hist = d[kin0:kin0 + n_ap * nv].reshape(n_ap, nv)
    vc = vlo + (np.arange(nv) + 0.5) * (vhi - vlo) / nv
    tot = np.maximum(hist.sum(1), 1e-300)
    v0 = (hist * vc).sum(1) / tot
    s = np.sqrt(np.maximum((hist * (vc - v0[:, None]) ** 2).sum(1) / tot, 20.0 ** 2))
    return d, gamma, v0, s


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gh_fit_end_to_end(gpu, dtype):
    import torch
    P = lib()
    cfg = W.SMALL
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=1000)
    sel = np.arange(0, 2000, 4)
    ics, dt = ics[:, sel], dt[sel]
    n, n_steps = ics.shape[1], 400
    obs = dict(cfg["obs"], surface=1, upsilon=1.0)
    n_mass, n_ap, nv, vlo, vhi = 1000, 50, 15, cfg["obs"]["vlo"], cfg["obs"]["vhi"]
    kin0, surf0 = n_mass, n_mass + n_ap * nv
    A_g, _, _, fl_g = gpu_integrate(cfg, ics, dt, n_steps, "f64", obs=obs)
    c_o, _, _, fl_o = oracle_integrate(cfg, ics, dt, n_steps, obs=obs)
    A_o = O.time_fractions(c_o, n_steps, obs=O.make_obs(obs, O.euler_matrix(*cfg["euler"])))
    assert np.array_equal(A_g, A_o)
    w_true = W.mock_draw(n, 2)
    d_full, gamma, v0, s = _mock_maps(A_o, w_true, n_mass, kin0, surf0, n_ap, nv, vlo, vhi)
    F_o = GH.fit_matrix(A_o, n_mass, kin0, surf0, n_ap, nv, vlo, vhi, v0, s, gamma)
    nf = F_o.shape[1]
    # data: density and Sigma of the mock, its h_m for the observed luminosity, plus noise on the h maps
    d = F_o.T @ w_true
    rng = np.random.default_rng(12)
    dh = 0.02
    d[n_mass + n_ap:] += dh * rng.standard_normal(nf - n_mass - n_ap)
    sig = np.empty(nf)
    sig[:n_mass + n_ap] = N.sigma_from_data(d[:n_mass + n_ap], [(0, n_mass), (n_mass, n_mass + n_ap)], 0.01)
    sig[n_mass + n_ap:] = dh
    wt = N.w_tilde_from_data(d, (0, n_mass), n)

    dev = torch.device("cuda:0")
    td = torch.float64 if dtype == "f64" else torch.float32
    A_t = torch.from_numpy(A_g).to(dev, td)
    F_t = torch.empty((n, nf), dtype=td, device=dev)
    ws = torch.empty(P.gh_fit_workspace_bytes(n_ap, nv), dtype=torch.uint8, device=dev)
    P.gh_fit_matrix(A_t, n_mass, kin0, surf0, n_ap, nv, vlo, vhi, v0, s, gamma, F_t, ws)
    torch.cuda.synchronize()
    F_g = F_t.cpu().numpy().astype(np.float64)
    if dtype == "f64":
        F_ref = F_o
    else:  # the library reads the single-precision matrix and rounds its output to single precision
        A32 = A_o.astype(np.float32).astype(np.float64)
        F_ref = GH.fit_matrix(A32, n_mass, kin0, surf0, n_ap, nv, vlo, vhi, v0, s, gamma)
        F_ref = F_ref.astype(np.float32).astype(np.float64)
    np.testing.assert_allclose(F_g, F_ref, rtol=1e-10 if dtype == "f64" else 2.4e-7, atol=1e-13)

    # the weight problem on the GPU's fit matrix and on the oracle's
    w_o = N.nnls_oracle(*N.scale_problem(F_ref, d, sig, wt), N.relative_mu(N.scale_problem(F_ref, d, sig, wt)[0],
                                                                            1e-2)) * wt
    opts = P._lib.SolveOpts()
    opts.gram, opts.nu = P.SW_GRAM_BF16X3, 1e-2
    w_t = torch.empty(n, dtype=torch.float64, device=dev)
    sws = torch.empty(P.solve_workspace_bytes(n, nf, opts), dtype=torch.uint8, device=dev)
    d_t, s_t = torch.from_numpy(d).to(dev), torch.from_numpy(sig).to(dev)
    st, rep = P.solve_weights(F_t, d_t, s_t, wt, -1.0, opts, w_t, sws)
    cws = torch.empty(P.chi2_workspace_bytes(nf), dtype=torch.uint8, device=dev)
    x_g = P.chi2(F_t, w_t, d_t, s_t, n_mass, nf, cws)
    torch.cuda.synchronize()
    w_g = w_t.cpu().numpy()
    x_o = N.chi2(F_ref, w_o, d, sig, n_mass, nf)
    l1 = np.abs(w_g - w_o).sum() / np.abs(w_o).sum()
    print(f"{dtype}: status {st}, iterations {rep.refine_iters}, kkt {rep.kkt:.2e}, weights L1 {l1:.2e}, "
          f"chi2 {x_g:.8g} vs {x_o:.8g} (Sigma + GH over {nf - n_mass} constraints)")
    assert st == 0 or (st == -4 and rep.kkt < 1e-6)
    assert l1 < 1e-2
    assert abs(x_g / x_o - 1) < 1e-3
