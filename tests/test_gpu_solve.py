"""GPU parity of solve_weights / chi2 / model_observables against the exact
FP64 NNLS oracle (Eq. 4) and the FP64 chi^2 of Eq. 5.

Bar (from the build's target): weights L1 relative error < 1e-2 and chi^2
relative error < 1e-3 against the oracle, on the same matrix and data.
"""
import numpy as np
import pytest

import workloads as W
from oracle import nnls as N
from tests.gpu_common import counts_from_fractions, gpu_integrate, lib

pytestmark = pytest.mark.gpu

W_L1_TOL = 1e-2
CHI2_TOL = 1e-3


def mock_problem(A, blocks, mock_seed, noise, tol):
    A64 = A.astype(np.float64)
    n, c = A.shape
    w_true = W.mock_draw(n, mock_seed)
    d = A64.T @ w_true
    if noise > 0:
        d = d * (1 + noise * W.noise_draw(c, mock_seed))
    sig = N.sigma_from_data(d, blocks, tol)
    wt = N.w_tilde_from_data(d, blocks[0], n)
    return d, sig, wt


def oracle_solve(A, d, sig, wt, nu):
    U, y = N.scale_problem(A.astype(np.float64), d, sig, wt)
    mu = N.relative_mu(U, nu)
    return N.nnls_oracle(U, y, mu) * wt, mu


def gpu_solve(A, d, sig, wt, nu, gram, **kw):
    import torch
    P = lib()
    dev = torch.device("cuda:0")
    At = torch.from_numpy(np.ascontiguousarray(A)).to(dev)
    dt = torch.from_numpy(d).to(dev)
    st = torch.from_numpy(sig).to(dev)
    opts = P._lib.SolveOpts()
    opts.gram = gram
    opts.nu = nu
    opts.max_iter = kw.get("max_iter", 0)
    opts.refine_iter = kw.get("refine_iter", 0)
    opts.tol = kw.get("tol", 0.0)
    opts.tol_kkt = kw.get("tol_kkt", 0.0)
    opts.flags = kw.get("flags", 0)
    opts.quantum = kw.get("quantum", 0.0)
    w = torch.empty(A.shape[0], dtype=torch.float64, device=dev)
    ws = torch.empty(P.solve_workspace_bytes(A.shape[0], A.shape[1], opts), dtype=torch.uint8, device=dev)
    if "fill" in kw:  # byte pattern written over the whole workspace first
        ws.fill_(kw["fill"])
    status, rep = P.solve_weights(At, dt, st, wt, -1.0, opts, w, ws)
    cws = torch.empty(P.chi2_workspace_bytes(A.shape[1]), dtype=torch.uint8, device=dev)
    return w.cpu().numpy(), status, rep, (At, w, dt, st, cws)


def chi2_gpu(handles, cb, ce):
    P = lib()
    At, w, dt, st, cws = handles
    return P.chi2(At, w, dt, st, cb, ce, cws)


@pytest.mark.parametrize("gram", [0, 1, 2], ids=["bf16", "bf16x3", "f32"])
def test_solve_sparse_lognormal(gpu, gram):
    n, c = 1500, 600
    blocks = [(0, 200), (200, c)]
    A = W.sparse_lognormal_matrix(n, blocks, density=0.1, seed=6)
    d, sig, wt = mock_problem(A, blocks, 4, 0.02, 0.02)
    w_o, mu = oracle_solve(A, d, sig, wt, 1e-2)
    w_g, status, rep, h = gpu_solve(A, d, sig, wt, 1e-2, gram)
    print(rep.as_dict())
    assert status == 0 or (status == -4 and rep.kkt < 1e-6)
    assert rep.mu == pytest.approx(mu, rel=1e-4)
    l1 = np.abs(w_g - w_o).sum() / np.abs(w_o).sum()
    x_o = N.chi2(A.astype(np.float64), w_o, d, sig, 200, c)
    x_g = chi2_gpu(h, 200, c)
    print("L1", l1, "chi2", x_g, x_o)
    assert l1 < W_L1_TOL
    assert abs(x_g / x_o - 1) < CHI2_TOL


def test_workspace_contents_do_not_matter(gpu):
    """The solve must not read workspace memory it has not written: a workspace
    filled with NaN bytes (0xFF) gives the same weights as a zeroed one, with
    and without the Anderson acceleration."""
    P = lib()
    n, c = 1500, 600
    blocks = [(0, 200), (200, c)]
    A = W.sparse_lognormal_matrix(n, blocks, density=0.1, seed=6)
    d, sig, wt = mock_problem(A, blocks, 4, 0.02, 0.02)
    for flags in (0, P.SW_SOLVE_NO_ACCEL):
        w0, st0, rep0, _ = gpu_solve(A, d, sig, wt, 1e-2, 1, flags=flags, fill=0)
        w1, st1, rep1, _ = gpu_solve(A, d, sig, wt, 1e-2, 1, flags=flags, fill=255)
        print(flags, rep0.as_dict(), rep1.as_dict())
        assert st0 == 0 and st1 == 0 and np.all(np.isfinite(w1))
        assert np.abs(w1 - w0).sum() <= 1e-9 * np.abs(w0).sum()


@pytest.fixture(params=[0, 1], ids=["factor_fp32", "factor_bf16x3"])
def factor_gemm(request):
    """The factorisation's large products on fp32 MFMA or on bf16x3 MFMA."""
    P = lib()
    old = P.get_tuning("factor_gemm")
    P.set_tuning("factor_gemm", request.param)
    yield request.param
    P.set_tuning("factor_gemm", old)


def test_solve_ragged_larger(gpu, factor_gemm):
    n, c = 3001, 1003
    blocks = [(0, 300), (300, c)]
    A = W.sparse_lognormal_matrix(n, blocks, density=0.1, seed=7)
    d, sig, wt = mock_problem(A, blocks, 5, 0.02, 0.02)
    w_o, mu = oracle_solve(A, d, sig, wt, 1e-2)
    w_g, status, rep, h = gpu_solve(A, d, sig, wt, 1e-2, 1)
    assert status == 0 or (status == -4 and rep.kkt < 1e-6)
    l1 = np.abs(w_g - w_o).sum() / np.abs(w_o).sum()
    x_o = N.chi2(A.astype(np.float64), w_o, d, sig, 300, c)
    assert l1 < W_L1_TOL
    assert abs(chi2_gpu(h, 300, c) / x_o - 1) < CHI2_TOL


def test_small_workload_end_to_end(gpu, factor_gemm):
    """Plummer + MN workload, FP64 on both sides: the GPU builds the orbit matrix,
    solves and evaluates chi^2; the oracle does all three on its own matrix."""
    import oracle as O
    from tests.gpu_common import oracle_integrate
    cfg = W.SMALL
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=cfg["n_steps"])
    A, ov, dr, fl = gpu_integrate(cfg, ics, dt, cfg["n_steps"], "f64")
    c_o, *_ = oracle_integrate(cfg, ics, dt, cfg["n_steps"])
    A_o = O.time_fractions(c_o, cfg["n_steps"])
    blocks = W.blocks(cfg["obs"])
    d, sig, wt = mock_problem(A_o, blocks, cfg["mock"]["seed"], cfg["mock"]["noise"], cfg["mock"]["tol"])
    w_o, mu = oracle_solve(A_o, d, sig, wt, 1e-2)
    w_g, status, rep, h = gpu_solve(A, d, sig, wt, 1e-2, 1)
    assert status == 0 or (status == -4 and rep.kkt < 1e-6)
    l1 = np.abs(w_g - w_o).sum() / np.abs(w_o).sum()
    x_o = N.chi2(A_o, w_o, d, sig, blocks[1][0], blocks[1][1])
    x_g = chi2_gpu(h, blocks[1][0], blocks[1][1])
    print("L1", l1, "chi2", x_g, x_o, rep.as_dict())
    assert l1 < W_L1_TOL
    assert abs(x_g / x_o - 1) < CHI2_TOL


def test_anderson_and_plain_admm_agree(gpu):
    """The Anderson-accelerated FP64 stage (the default) and plain ADMM (the FP32
    stage, then the FP64 stage without acceleration) reach the same weights,
    both within the oracle tolerance, and the accelerated solve needs fewer
    iterations."""
    import oracle as O
    from tests.gpu_common import oracle_integrate
    P = lib()
    cfg = W.SMALL
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=cfg["n_steps"])
    A, ov, dr, fl = gpu_integrate(cfg, ics, dt, cfg["n_steps"], "f64")
    c_o, *_ = oracle_integrate(cfg, ics, dt, cfg["n_steps"])
    A_o = O.time_fractions(c_o, cfg["n_steps"])
    blocks = W.blocks(cfg["obs"])
    d, sig, wt = mock_problem(A_o, blocks, cfg["mock"]["seed"], cfg["mock"]["noise"], cfg["mock"]["tol"])
    w_o, mu = oracle_solve(A_o, d, sig, wt, 1e-2)
    w_a, st_a, rep_a, _ = gpu_solve(A, d, sig, wt, 1e-2, 1)
    w_p, st_p, rep_p, _ = gpu_solve(A, d, sig, wt, 1e-2, 1, flags=P.SW_SOLVE_NO_ACCEL)
    print("accelerated", rep_a.as_dict())
    print("plain", rep_p.as_dict())
    for w_g, st, rep in ((w_a, st_a, rep_a), (w_p, st_p, rep_p)):
        assert st == 0 and rep.converged == 1
        assert np.abs(w_g - w_o).sum() / np.abs(w_o).sum() < W_L1_TOL
    assert np.abs(w_a - w_p).sum() / np.abs(w_p).sum() < W_L1_TOL
    assert rep_a.iters == 0 and rep_p.iters > 0
    assert rep_a.refine_iters < rep_p.iters + rep_p.refine_iters


def test_chi2_and_model_observables(gpu):
    import torch
    P = lib()
    rng = np.random.default_rng(3)
    A = rng.random((777, 345)).astype(np.float32)
    w = rng.exponential(size=777)
    d = A.astype(np.float64).T @ w * (1 + 0.01 * rng.normal(size=345))
    sig = 0.01 * d
    At = torch.from_numpy(A).cuda()
    wt = torch.from_numpy(w).cuda()
    out = torch.empty(345, dtype=torch.float64, device="cuda")
    P.model_observables(At, wt, out)
    torch.cuda.synchronize()
    ref = A.astype(np.float64).T @ w
    assert np.allclose(out.cpu().numpy(), ref, rtol=1e-12)
    cws = torch.empty(P.chi2_workspace_bytes(345), dtype=torch.uint8, device="cuda")
    x = P.chi2(At, wt, torch.from_numpy(d).cuda(), torch.from_numpy(sig).cuda(), 45, 345, cws)
    assert x == pytest.approx(N.chi2(A.astype(np.float64), w, d, sig, 45, 345), rel=1e-12)


def test_solve_batched_matches_oracle_per_problem(gpu):
    """Three independent problems of different orbit counts solved in one batched call."""
    import torch
    P = lib()
    c = 500
    blocks = [(0, 150), (150, c)]
    sizes = [700, 1201, 333]
    mats, ds, sigs, wts, w_os = [], [], [], [], []
    for k, n in enumerate(sizes):
        A = W.sparse_lognormal_matrix(n, blocks, density=0.1, seed=20 + k)
        d, sig, wt = mock_problem(A, blocks, 30 + k, 0.02, 0.02)
        w_o, _ = oracle_solve(A, d, sig, wt, 1e-2)
        mats.append(A); ds.append(d); sigs.append(sig); wts.append(wt); w_os.append(w_o)
    A = np.concatenate(mats)
    off = np.concatenate([[0], np.cumsum(sizes)])
    dev = torch.device("cuda:0")
    opts = P._lib.SolveOpts()
    opts.gram = 1
    opts.nu = 1e-2
    At = torch.from_numpy(A).to(dev)
    dt = torch.from_numpy(np.stack(ds)).to(dev)
    st = torch.from_numpy(np.stack(sigs)).to(dev)
    w = torch.empty(A.shape[0], dtype=torch.float64, device=dev)
    ws = torch.empty(P.solve_batched_workspace_bytes(off, c, opts), dtype=torch.uint8, device=dev)
    status, reps = P.solve_weights_batched(At, off, dt, st, wts, -1.0, opts, w, ws)
    wg = w.cpu().numpy()
    print([(r.iters, r.refine_iters, r.kkt, r.converged) for r in reps])
    assert status == 0 or (status == -4 and max(r.kkt for r in reps) < 1e-6)
    for k in range(3):
        wk = wg[off[k]:off[k + 1]]
        l1 = np.abs(wk - w_os[k]).sum() / np.abs(w_os[k]).sum()
        x_o = N.chi2(mats[k].astype(np.float64), w_os[k], ds[k], sigs[k], 150, c)
        x_g = N.chi2(mats[k].astype(np.float64), wk, ds[k], sigs[k], 150, c)
        print(k, "L1", l1, "chi2", x_g, x_o, reps[k].iters, reps[k].refine_iters, reps[k].kkt)
        assert l1 < W_L1_TOL
        assert abs(x_g / x_o - 1) < CHI2_TOL


def test_solve_dense_matrix_path(gpu):
    """A fully dense matrix takes the uncompressed passes over A."""
    rng = np.random.default_rng(12)
    n, c = 900, 300
    blocks = [(0, 100), (100, c)]
    A = (rng.random((n, c)) + 0.01).astype(np.float32)
    d, sig, wt = mock_problem(A, blocks, 8, 0.02, 0.02)
    w_o, mu = oracle_solve(A, d, sig, wt, 1e-2)
    w_g, status, rep, h = gpu_solve(A, d, sig, wt, 1e-2, 1)
    print(rep.as_dict())
    assert rep.nnz == 0.0  # dense passes
    assert status == 0 or (status == -4 and rep.kkt < 1e-6)
    l1 = np.abs(w_g - w_o).sum() / np.abs(w_o).sum()
    x_o = N.chi2(A.astype(np.float64), w_o, d, sig, 100, c)
    assert l1 < W_L1_TOL
    assert abs(chi2_gpu(h, 100, c) / x_o - 1) < CHI2_TOL


def test_compressed_blocks_match_dense_passes(gpu):
    """A problem large enough that the compressed copies split into several
    LDS blocks (20,000 constraints = 2 column blocks; 40,000 orbits = 3 row
    blocks): the solve with compressed passes must agree with the solve that
    streams the dense matrix in every pass."""
    import torch
    P = lib()
    dev = torch.device("cuda:0")
    n, c = 40000, 20000
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    A = torch.rand((n, c), generator=g, device=dev) < 0.03
    A = torch.where(A, torch.exp(torch.randn((n, c), generator=g, device=dev)), torch.zeros((), device=dev))
    A = (A / A.sum(1, keepdim=True).clamp(min=1e-30)).to(torch.float32).contiguous()
    wtrue = torch.zeros(n, dtype=torch.float64, device=dev)
    pick = torch.randperm(n, generator=g, device=dev)[: n // 10]
    wtrue[pick] = torch.empty(n // 10, dtype=torch.float64, device=dev).exponential_(1.0, generator=g)
    d = A.double().T @ wtrue
    sig = 0.02 * torch.clamp(d, min=1e-3 * float(d.max()))
    wt = float(d.sum()) / n
    res = []
    # compressed passes with the automatic row-dot shape, then with 64 and 16
    # lanes per row forced; last the dense passes
    for flags, lanes in ((0, 0), (0, 64), (0, 16), (P.SW_SOLVE_DENSE, 0)):
        P.set_tuning("sparse_lanes_per_row", lanes)
        opts = P._lib.SolveOpts()
        opts.gram, opts.nu, opts.flags = P.SW_GRAM_BF16X3, 1e-2, flags
        w = torch.empty(n, dtype=torch.float64, device=dev)
        ws = torch.empty(P.solve_workspace_bytes(n, c, opts), dtype=torch.uint8, device=dev)
        status, rep = P.solve_weights(A, d, sig, wt, -1.0, opts, w, ws)
        cws = torch.empty(P.chi2_workspace_bytes(c), dtype=torch.uint8, device=dev)
        x2 = P.chi2(A, w, d, sig, 0, c, cws)
        print(flags, lanes, status, rep.as_dict(), x2)
        res.append((w.cpu().numpy(), status, rep, x2))
        del ws
    P.set_tuning("sparse_lanes_per_row", 0)
    w_d, st_d, rep_d, x_d = res[-1]
    assert rep_d.nnz == 0 and st_d == 0
    for w_s, st_s, rep_s, x_s in res[:-1]:
        assert rep_s.nnz > 0 and st_s == 0
        assert np.abs(w_s - w_d).sum() / np.abs(w_d).sum() < 1e-3
        assert abs(x_s / x_d - 1) < 1e-6


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_gh_moments_match_oracle(gpu, dtype):
    """Gauss-Hermite moments (Eq. 2) of the kinematic block of the small model's
    orbit matrix against the oracle's quadrature, per orbit and aperture."""
    import torch
    from oracle import gh as OG
    P = lib()
    cfg = W.SMALL
    n_steps = 300
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=n_steps)
    ics, dt = ics[:, ::4], dt[::4]
    A, _, _, _ = gpu_integrate(cfg, ics, dt, n_steps, "f64")
    if dtype == "f32":
        A = A.astype(np.float32)
    o = cfg["obs"]
    n_ap, nv, kin0 = o["npx"] * o["npy"], o["nv"], o["nx"] * o["ny"] * o["nz"]
    rng = np.random.default_rng(5)
    v0 = rng.uniform(-60, 60, n_ap)
    s = rng.uniform(40, 160, n_ap)
    dev = torch.device("cuda:0")
    At = torch.from_numpy(np.ascontiguousarray(A)).to(dev)
    out = torch.empty((A.shape[0], n_ap, 5), dtype=torch.float64, device=dev)
    ws = torch.empty(P.gh_workspace_bytes(n_ap, nv), dtype=torch.uint8, device=dev)
    P.gh_moments(At, kin0, n_ap, nv, o["vlo"], o["vhi"], v0, s, out, ws)
    g = out.cpu().numpy()
    ref = OG.orbit_moments(A[:, kin0:kin0 + n_ap * nv].astype(np.float64), n_ap, nv, o["vlo"], o["vhi"], v0, s)
    scale = np.abs(ref).max()
    err = np.abs(g - ref).max() / scale
    print("gh max rel err", err)
    assert err < 1e-12


def test_gram_panel_skipping_matches_dense_gram(gpu):
    """The Gram takes the orbits in footprint order and skips the 32-orbit stages
    whose panels are zero (a skipped stage adds exactly zero; only the fp32
    summation order of the Gram changes); the solve lands on the weights of
    the Gram that streams every stage in the rows' order, within the KKT
    tolerance, and within the oracle's bar."""
    P = lib()
    cfg = W.SMALL
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=cfg["n_steps"])
    A, *_ = gpu_integrate(cfg, ics, dt, 400, "f64")
    blocks = W.blocks(cfg["obs"])
    d, sig, wt = mock_problem(A, blocks, cfg["mock"]["seed"], 0.02, 0.02)
    w_o, _ = oracle_solve(A, d, sig, wt, 1e-2)
    out = {}
    old = P.get_tuning("gram_skip")
    try:
        for skip in (0, 1):
            P.set_tuning("gram_skip", skip)
            w, status, rep, _ = gpu_solve(A, d, sig, wt, 1e-2, 1)
            out[skip] = (w, status, rep.refine_iters)
    finally:
        P.set_tuning("gram_skip", old)
    print({k: (v[1], v[2]) for k, v in out.items()})
    assert out[0][1] == 0 and out[1][1] == 0
    assert np.abs(out[1][0] - out[0][0]).sum() <= 1e-5 * np.abs(out[0][0]).sum()
    assert np.abs(out[1][0] - w_o).sum() / np.abs(w_o).sum() < W_L1_TOL


@pytest.mark.parametrize("flags", [0, 2], ids=["anderson", "plain_admm"])
def test_two_pass_iterations_match_four(gpu, flags):
    """The FP64 stage with U^T U x carried along (two passes over A per
    iteration, the default) and with the residual recomputed from A every
    iteration (four passes) reach the same weights, both within the oracle's
    bar, with and without the Anderson acceleration."""
    import oracle as O
    from tests.gpu_common import oracle_integrate
    P = lib()
    cfg = W.SMALL
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=cfg["n_steps"])
    A, *_ = gpu_integrate(cfg, ics, dt, cfg["n_steps"], "f64")
    c_o, *_ = oracle_integrate(cfg, ics, dt, cfg["n_steps"])
    A_o = O.time_fractions(c_o, cfg["n_steps"])
    blocks = W.blocks(cfg["obs"])
    d, sig, wt = mock_problem(A_o, blocks, cfg["mock"]["seed"], 0.02, cfg["mock"]["tol"])
    w_o, _ = oracle_solve(A_o, d, sig, wt, 1e-2)
    out = {}
    old = P.get_tuning("refine_passes")
    try:
        for passes in (2, 4):
            P.set_tuning("refine_passes", passes)
            w, status, rep, _ = gpu_solve(A, d, sig, wt, 1e-2, 1, flags=flags)
            out[passes] = (w, status, rep.iters, rep.refine_iters, rep.kkt)
    finally:
        P.set_tuning("refine_passes", old)
    print({k: v[1:] for k, v in out.items()})
    for passes, (w, status, _, _, kkt) in out.items():
        assert status == 0, passes
        assert np.abs(w - w_o).sum() / np.abs(w_o).sum() < W_L1_TOL, passes
    assert np.abs(out[2][0] - out[4][0]).sum() <= 1e-4 * np.abs(out[4][0]).sum()


def test_two_pass_fallback_to_four(gpu):
    """The two-pass FP64 stage falls back to four passes when a problem's KKT
    residual rebounds; forced at the fourth check (rebound factor 0), the batched
    solve still converges, reports four passes, and reaches the weights of the
    plain four-pass solve within 1e-4 (L1) and the oracle's within the parity
    bar."""
    import torch
    P = lib()
    c = 500
    blocks = [(0, 150), (150, c)]
    sizes = [700, 1201]
    mats, ds, sigs, wts = [], [], [], []
    for k, n in enumerate(sizes):
        A = W.sparse_lognormal_matrix(n, blocks, density=0.1, seed=40 + k)
        d, sig, wt = mock_problem(A, blocks, 50 + k, 0.02, 0.02)
        mats.append(A); ds.append(d); sigs.append(sig); wts.append(wt)
    A = np.concatenate(mats)
    off = np.concatenate([[0], np.cumsum(sizes)])
    dev = torch.device("cuda:0")
    At = torch.from_numpy(A).to(dev)
    dt = torch.from_numpy(np.stack(ds)).to(dev)
    st = torch.from_numpy(np.stack(sigs)).to(dev)
    opts = P._lib.SolveOpts()
    opts.gram, opts.nu = 1, 1e-2
    ws = torch.empty(P.solve_batched_workspace_bytes(off, c, opts), dtype=torch.uint8, device=dev)
    out = {}
    old_p, old_r = P.get_tuning("refine_passes"), P.get_tuning("refine_rebound")
    try:
        for name, passes, rebound in (("fallback", 2, 0), ("four", 4, 10)):
            P.set_tuning("refine_passes", passes)
            P.set_tuning("refine_rebound", rebound)
            w = torch.empty(A.shape[0], dtype=torch.float64, device=dev)
            status, reps = P.solve_weights_batched(At, off, dt, st, wts, -1.0, opts, w, ws)
            out[name] = (w.cpu().numpy(), status, [r.passes for r in reps], [r.refine_iters for r in reps])
    finally:
        P.set_tuning("refine_passes", old_p)
        P.set_tuning("refine_rebound", old_r)
    print({k: v[1:] for k, v in out.items()})
    assert out["fallback"][1] == 0 and out["four"][1] == 0
    assert out["fallback"][2] == [4, 4]
    wf, w4 = out["fallback"][0], out["four"][0]
    assert np.abs(wf - w4).sum() <= 1e-4 * np.abs(w4).sum()
    for k in range(2):
        w_o, _ = oracle_solve(mats[k], ds[k], sigs[k], wts[k], 1e-2)
        wk = wf[off[k]:off[k + 1]]
        assert np.abs(wk - w_o).sum() / np.abs(w_o).sum() < W_L1_TOL


@pytest.mark.parametrize("gram_counts", [1, 0], ids=["gram_of_counts", "gram_of_values"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_count_quantum_compressed_copies(gpu, dtype, gram_counts):
    """A leapfrog orbit matrix is a histogram of counts of q = 1 / (ncopy
    n_steps).  With that quantum the compressed copies hold the counts and every
    pass computes with the exact multiples k q: the weights then meet the KKT
    tolerance on the exact matrix (checked by the oracle's residual, Eq. 4), as
    the value copies' weights do on A itself, and chi^2 agrees; the FP64 matrix
    also matches the oracle's weights and chi^2.  The Gram takes the counts as
    its operand (its low-plane products only where a count exceeds 256, then
    scaled) or the scaled values.  A quantum of which the entries are not
    multiples fails with SW_EINVAL."""
    import oracle as O
    from tests.gpu_common import oracle_integrate
    P = lib()
    old = P.get_tuning("gram_counts")
    P.set_tuning("gram_counts", gram_counts)
    try:
        _count_quantum_case(P, O, oracle_integrate, dtype)
    finally:
        P.set_tuning("gram_counts", old)


def _count_quantum_case(P, O, oracle_integrate, dtype):
    cfg = W.SMALL
    n_steps = cfg["n_steps"]
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=n_steps)
    A, *_ = gpu_integrate(cfg, ics, dt, n_steps, dtype)
    c_o, *_ = oracle_integrate(cfg, ics, dt, n_steps)
    A_o = O.time_fractions(c_o, n_steps)
    blocks = W.blocks(cfg["obs"])
    d, sig, wt = mock_problem(A_o, blocks, cfg["mock"]["seed"], 0.02, cfg["mock"]["tol"])
    q = P.count_quantum(P.obs_spec(cfg["obs"]), n_steps)
    assert q > 0
    A64 = A.astype(np.float64)
    A_k = np.rint(A64 / q) * q  # the exact multiples A rounds
    out = {}
    for quantum, A_ref in ((0.0, A64), (q, A_k)):
        w, status, rep, h = gpu_solve(A, d, sig, wt, 1e-2, 1, quantum=quantum)
        assert status == 0, quantum
        assert rep.nnz > 0  # the compressed copies were used
        kkt = N.kkt_residual_orbit_matrix(A_ref, d, sig, wt, rep.mu, w)
        x = N.chi2(A_ref, w, d, sig, blocks[1][0], blocks[1][1])
        out[quantum] = (w, x, kkt, rep.kkt, rep.refine_iters)
        print(quantum, "chi2", x, "kkt", kkt, rep.kkt, "iterations", rep.refine_iters)
        assert kkt <= 1.5e-7
    # solutions that meet the KKT tolerance of 1e-7 differ in chi^2 at the 1e-6 level
    assert abs(out[q][1] / out[0.0][1] - 1) < 1e-5
    if dtype == "f64":
        w_o, _ = oracle_solve(A_o, d, sig, wt, 1e-2)
        assert np.abs(out[q][0] - w_o).sum() / np.abs(w_o).sum() < W_L1_TOL
        x_o = N.chi2(A_o, w_o, d, sig, blocks[1][0], blocks[1][1])
        assert abs(out[q][1] / x_o - 1) < CHI2_TOL
    with pytest.raises(P.SchwError) as e:
        gpu_solve(A, d, sig, wt, 1e-2, 1, quantum=1.5 * q)
    assert e.value.status == -1 and "quantum" in str(e.value)


def test_triangle_pass_row_blocking(gpu):
    """The passes over the inverse factor's triangles with 16 rows per wave (one
    load of the vector for all of them, chunks across the diagonal masked) and
    with 2: both solves converge to the same weights (1e-4, L1), within the
    oracle's bar."""
    import oracle as O
    from tests.gpu_common import oracle_integrate
    P = lib()
    cfg = W.SMALL
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=cfg["n_steps"])
    A, *_ = gpu_integrate(cfg, ics, dt, cfg["n_steps"], "f64")
    c_o, *_ = oracle_integrate(cfg, ics, dt, cfg["n_steps"])
    A_o = O.time_fractions(c_o, cfg["n_steps"])
    blocks = W.blocks(cfg["obs"])
    d, sig, wt = mock_problem(A_o, blocks, cfg["mock"]["seed"], 0.02, cfg["mock"]["tol"])
    w_o, _ = oracle_solve(A_o, d, sig, wt, 1e-2)
    out = {}
    old = P.get_tuning("trmv_rows")
    try:
        for rows in (2, 16):
            P.set_tuning("trmv_rows", rows)
            w, status, rep, _ = gpu_solve(A, d, sig, wt, 1e-2, 1)
            out[rows] = (w, status, rep.refine_iters, rep.kkt)
    finally:
        P.set_tuning("trmv_rows", old)
    print({k: v[1:] for k, v in out.items()})
    for rows, (w, status, _, _) in out.items():
        assert status == 0, rows
        assert np.abs(w - w_o).sum() / np.abs(w_o).sum() < W_L1_TOL, rows
    assert np.abs(out[16][0] - out[2][0]).sum() <= 1e-4 * np.abs(out[2][0]).sum()
