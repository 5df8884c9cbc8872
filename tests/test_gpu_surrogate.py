"""The learned chi^2 surrogate on the GPU, end to end: trained by the library's
MLP kernels on chi^2 values of builds of the method itself, it screens the
proposals of a delayed-acceptance sampler (Christen & Fox 2005) whose second
stage is the full Schwarzschild build.  What it gains over the same sampler
without it: fewer full builds for the same proposals, the screen rejecting the
proposals it predicts to be poor, while the second stage keeps the posterior
exact."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import lib

pytestmark = pytest.mark.gpu


def small_builder(P, torch, max_batch):
    from paper_2607_00117_amd import surrogate as S
    n_orb, n_steps = 256, 200
    table = W.load_table(W.BARRED["table"])
    ics, dt = W.disc_ics(table, n_orb, seed=3, n_steps=n_steps, periods=10.0)  # 20 steps per circular period
    obs_d = dict(W.SMALL["obs"])
    blocks = W.blocks(obs_d)
    dev = torch.device("cuda:0")
    # mock: binned sum of a seeded 10% subset at the nominal parameters
    comps, omega, euler = W.theta_to_model(W.theta_nominal())
    pot = P.build_potential(comps, omega, euler)
    obs = P.obs_spec(obs_d)
    nc = P.ncon(obs)
    A = torch.empty((n_orb, nc), dtype=torch.float32, device=dev)
    ov = torch.empty((n_orb, 2), dtype=torch.float64, device=dev)
    dr = torch.empty(n_orb, dtype=torch.float64, device=dev)
    fl = torch.empty(n_orb, dtype=torch.uint8, device=dev)
    ws = torch.empty(P.integrate_workspace_bytes(obs, 1, n_orb, n_steps, P.SW_F32), dtype=torch.uint8, device=dev)
    P.integrate_and_bin(pot, [0, n_orb], torch.from_numpy(ics.astype(np.float32)).to(dev),
                        torch.from_numpy(dt.astype(np.float32)).to(dev), n_steps, obs, A, ov, dr, fl, ws)
    d_t = torch.empty(nc, dtype=torch.float64, device=dev)
    P.model_observables(A, torch.from_numpy(W.mock_draw(n_orb, 4)).to(dev), d_t)
    d = d_t.cpu().numpy() * (1 + 0.02 * W.noise_draw(nc, 4))
    top = [float(np.max(d[b0:b1])) for b0, b1 in blocks]
    sig = np.concatenate([0.02 * np.maximum(d[b0:b1], 1e-3 * t) for (b0, b1), t in zip(blocks, top)])
    wt = float(np.sum(d[blocks[0][0]:blocks[0][1]])) / n_orb
    opts = P._lib.SolveOpts()
    opts.use_graph = 1
    return S.ModelBuilder(W.theta_to_model, ics, dt, n_steps, obs_d, d, sig, wt, max_batch, kin_block=blocks[1],
                          solve_opts=opts), obs_d


def test_surrogate_screen_saves_full_builds(gpu):
    import torch
    from paper_2607_00117_amd import surrogate as S
    P = lib()
    builder, obs_d = small_builder(P, torch, 64)
    nominal = W.theta_nominal()
    lo, hi = 0.7 * nominal, 1.3 * nominal
    n_ap = obs_d["npx"] * obs_d["npy"]
    dchi2, jk = builder.jackknife_dchi2(nominal, n_ap, obs_d["nv"])
    assert np.all(np.isfinite(jk)) and dchi2 > 0
    n_fit, n_test = 1024, 128
    thetas = lo + (hi - lo) * W.latin_hypercube(n_fit + n_test, 12, seed=7)
    chi = builder.chi2(thetas)
    assert np.all(np.isfinite(chi)) and np.all(chi > 0)
    assert np.unique(np.round(chi, 6)).size > 0.9 * len(chi)  # every build is its own model
    sur = S.Surrogate(lo, hi)
    sur.fit(thetas[:n_fit], chi[:n_fit], epochs=300, batch=128)
    err = np.abs(sur.predict(thetas[n_fit:]) - chi[n_fit:]) / dchi2
    base = np.abs(np.median(chi[:n_fit]) - chi[n_fit:]) / dchi2  # the method without the network: a constant guess
    print(f"dchi2 {dchi2:.4g}; held-out |chi2_s - chi2| / dchi2: median {np.median(err):.3g} "
          f"(constant guess {np.median(base):.3g})")
    assert np.median(err) < 0.5 * np.median(base)
    theta0 = W.walker_thetas(16, seed=8, spread=0.05)
    da = S.da_mcmc(builder, sur, theta0, lo, hi, 8, dchi2, use_surrogate=True)
    mh = S.da_mcmc(builder, sur, theta0, lo, hi, 8, dchi2, use_surrogate=False)
    print(f"full builds: delayed acceptance {da['n_full_builds']} (screened {da['n_stage1']} of "
          f"{da['proposals']}), plain {mh['n_full_builds']}; accepted {da['n_accepted']} vs {mh['n_accepted']}")
    assert np.all(np.isfinite(da["chains"])) and np.all(np.isfinite(mh["chains"]))
    assert da["n_full_builds"] < mh["n_full_builds"]
