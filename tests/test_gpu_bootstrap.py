"""GPU parity of the bootstrap path (Sec. 2.3-2.4, Eq. 6): the realisations of
the data (bootstrap_data: bit-exact), the weight problems of all realisations
solved on one shared orbit matrix (solve_weights_multi: per realisation against
the exact FP64 NNLS oracle, weights L1 relative error < 1e-2 and chi^2 relative
error < 1e-3), and the bootstrap-marginalised chi^2 of a small model build.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bootstrap as BS
from oracle import nnls as N
from tests.gpu_common import lib
from tests.test_gpu_solve import CHI2_TOL, W_L1_TOL, mock_problem, oracle_solve

pytestmark = pytest.mark.gpu


def multi_solve(A, D, sig, wt, nu=1e-2, gram=1, **kw):
    """solve_weights_multi on host arrays; returns (w [B][n], status, reports)."""
    import torch
    P = lib()
    dev = torch.device("cuda:0")
    opts = P._lib.SolveOpts()
    opts.gram, opts.nu = gram, nu
    opts.flags = kw.get("flags", 0)
    opts.quantum = kw.get("quantum", 0.0)
    w0 = None
    if kw.get("w0") is not None:  # warm start from one weight vector for every realisation
        w0 = torch.from_numpy(np.ascontiguousarray(kw["w0"])).to(dev)
        opts.w0, opts.w0_shared = w0.data_ptr(), 1
    At = A if isinstance(A, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(A)).to(dev)
    Dt = D if isinstance(D, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(D)).to(dev)
    st = sig if isinstance(sig, torch.Tensor) else torch.from_numpy(sig).to(dev)
    B, n = Dt.shape[0], At.shape[0]
    w = torch.empty((B, n), dtype=torch.float64, device=dev)
    ws = torch.empty(P.solve_multi_workspace_bytes(n, At.shape[1], B, opts), dtype=torch.uint8, device=dev)
    if "fill" in kw:
        ws.fill_(kw["fill"])
    status, reps = P.solve_weights_multi(At, Dt, st, wt, -1.0, opts, w, ws)
    return w.cpu().numpy(), status, reps


def _converged(status, reps):
    return status == 0 or (status == -4 and max(r.kkt for r in reps) < 1e-6)


def test_bootstrap_data_bit_exact(gpu):
    import torch
    P = lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(2)
    C, cb, B = 1750, 1000, 37
    d = rng.random(C) * 3 + 0.01
    sig = 0.02 * d
    eps = W.bootstrap_eps(B, C, seed=3)
    out = torch.empty((B, C), dtype=torch.float64, device=dev)
    P.bootstrap_data(torch.from_numpy(d).to(dev), torch.from_numpy(sig).to(dev), torch.from_numpy(eps).to(dev), cb, C,
                     out)
    assert np.array_equal(out.cpu().numpy(), BS.bootstrap_data(d, sig, eps, cb, C))


@pytest.fixture(params=[1, 2], ids=["dense_mfma_passes", "compressed_passes"])
def multi_dense(request):
    """The passes of the shared-matrix solve as dense FP64 MFMA products over all
    data vectors, or as compressed passes per group of vectors."""
    P = lib()
    old = P.get_tuning("multi_dense")
    P.set_tuning("multi_dense", request.param)
    yield request.param
    P.set_tuning("multi_dense", old)


@pytest.mark.parametrize("density", [0.1, 0.5])
def test_multi_rhs_matches_oracle_per_realisation(gpu, multi_dense, density):
    """Six realisations on one sparse log-normal matrix with a ragged orbit count,
    at 10% and 50% density, with either kind of pass."""
    n, c, cb = 1501, 600, 200
    blocks = [(0, cb), (cb, c)]
    A = W.sparse_lognormal_matrix(n, blocks, density=density, seed=6)
    d, sig, wt = mock_problem(A, blocks, 4, 0.02, 0.02)
    D = BS.bootstrap_data(d, sig, W.bootstrap_eps(6, c, seed=1), cb, c)
    w_g, status, reps = multi_solve(A, D, sig, wt)
    print([(r.refine_iters, r.kkt) for r in reps])
    assert _converged(status, reps)
    A64 = A.astype(np.float64)
    for b in range(D.shape[0]):
        w_o, mu = oracle_solve(A, D[b], sig, wt, 1e-2)
        assert reps[b].mu == pytest.approx(mu, rel=1e-4)
        l1 = np.abs(w_g[b] - w_o).sum() / np.abs(w_o).sum()
        x_o = N.chi2(A64, w_o, d, sig, cb, c)
        x_g = N.chi2(A64, w_g[b], d, sig, cb, c)
        print(b, "L1", l1, "chi2", x_g, x_o)
        assert l1 < W_L1_TOL
        assert abs(x_g / x_o - 1) < CHI2_TOL


def test_one_data_vector_is_solve_weights(gpu):
    """With one data vector the shared-matrix solve runs the kernels of
    solve_weights on the same operands: the weights are identical."""
    from tests.test_gpu_solve import gpu_solve
    n, c = 900, 400
    blocks = [(0, 100), (100, c)]
    A = W.sparse_lognormal_matrix(n, blocks, density=0.08, seed=9)
    d, sig, wt = mock_problem(A, blocks, 5, 0.02, 0.02)
    w_s, st_s, rep_s, _ = gpu_solve(A, d, sig, wt, 1e-2, 1)
    w_m, st_m, reps = multi_solve(A, d[None, :], sig, wt)
    assert st_s == st_m and rep_s.refine_iters == reps[0].refine_iters
    assert np.array_equal(w_s, w_m[0])


def test_multi_rhs_agrees_with_separate_solves_dense_and_masked(gpu):
    """Dense matrix (uncompressed passes) and masked orbits: each realisation
    agrees with its own solve_weights call."""
    import torch
    P = lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(12)
    n, c, cb = 700, 260, 90
    A = (rng.random((n, c)) + 0.01).astype(np.float32)
    blocks = [(0, cb), (cb, c)]
    d, sig, wt = mock_problem(A, blocks, 8, 0.02, 0.02)
    D = BS.bootstrap_data(d, sig, W.bootstrap_eps(3, c, seed=4), cb, c)
    mask = np.zeros(n, dtype=np.uint8)
    mask[rng.choice(n, 40, replace=False)] = 1
    mt = torch.from_numpy(mask).to(dev)
    opts = P._lib.SolveOpts()
    opts.gram, opts.nu, opts.mask = 1, 1e-2, mt.data_ptr()
    At = torch.from_numpy(A).to(dev)
    w = torch.empty((3, n), dtype=torch.float64, device=dev)
    ws = torch.empty(P.solve_multi_workspace_bytes(n, c, 3, opts), dtype=torch.uint8, device=dev)
    status, reps = P.solve_weights_multi(At, torch.from_numpy(D).to(dev), torch.from_numpy(sig).to(dev), wt, -1.0,
                                         opts, w, ws)
    assert reps[0].nnz == 0.0 and _converged(status, reps)
    w_m = w.cpu().numpy()
    assert np.all(w_m[:, mask == 1] == 0.0)
    keep = mask == 0
    for b in range(3):
        w_o, _ = oracle_solve(A[keep], D[b], sig, wt, 1e-2)
        l1 = np.abs(w_m[b][keep] - w_o).sum() / np.abs(w_o).sum()
        print(b, "L1", l1)
        assert l1 < W_L1_TOL


def test_multi_rhs_compressed_blocks(gpu):
    """20,000 constraints x 40,000 orbits (two column blocks, three row blocks
    of the compressed copies) with three data vectors: each realisation's
    weights agree with a separate solve_weights call, and its KKT residual
    meets the tolerance."""
    import torch
    P = lib()
    dev = torch.device("cuda:0")
    n, c, B = 40000, 20000, 3
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
    eps = torch.from_numpy(W.bootstrap_eps(B, c, seed=5)).to(dev)
    D = torch.empty((B, c), dtype=torch.float64, device=dev)
    P.bootstrap_data(d, sig, eps, 5000, c, D)
    w_m, status, reps = multi_solve(A, D, sig, wt)
    print([(r.refine_iters, r.kkt, r.nnz) for r in reps])
    assert reps[0].nnz > 0 and _converged(status, reps)
    opts = P._lib.SolveOpts()
    opts.gram, opts.nu = 1, 1e-2
    ws = torch.empty(P.solve_workspace_bytes(n, c, opts), dtype=torch.uint8, device=dev)
    for b in range(B):
        w = torch.empty(n, dtype=torch.float64, device=dev)
        st, rep = P.solve_weights(A, D[b].contiguous(), sig, wt, -1.0, opts, w, ws)
        ws_ = w.cpu().numpy()
        l1 = np.abs(w_m[b] - ws_).sum() / np.abs(ws_).sum()
        print(b, "L1 vs separate solve", l1, rep.refine_iters, reps[b].refine_iters)
        assert st == 0 and l1 < 1e-3


def test_bootstrap_chi2_model_small_build(gpu, multi_dense):
    """Small model build (FP64 integration, 2,000 orbits): 16 bootstrap
    realisations of the kinematic maps solved on the GPU (the multi-vector
    inverse products split over the columns of the factor), with either kind of
    pass over the matrix; the chi^2 of the first four realisations' weights
    against the observed data, and their marginalised chi2_model, against the
    oracle's solves of the same realisations (an oracle solve of this size takes
    several seconds); all 16 converge and their chi2_model lies in its bounds."""
    import torch
    import oracle as O
    P = lib()
    dev = torch.device("cuda:0")
    cfg = W.SMALL
    n_steps = 1000
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=n_steps)
    opot = O.make_pot(cfg["components"], cfg["omega"])
    oobs = O.make_obs(cfg["obs"], O.euler_matrix(*cfg["euler"]))
    c_o, _, _, _ = O.integrate_and_bin(opot, oobs, ics, dt, n_steps)
    A = O.time_fractions(c_o, n_steps)
    n, c = A.shape
    blocks = W.blocks(cfg["obs"])
    kin0 = blocks[1][0]
    d = A.T @ W.mock_draw(n, cfg["mock"]["seed"])
    sig = N.sigma_from_data(d, blocks, 0.01)
    wt = N.w_tilde_from_data(d, blocks[0], n)
    B = 16
    eps = W.bootstrap_eps(B, c, seed=6)
    D_o = BS.bootstrap_data(d, sig, eps, kin0, c)
    At = torch.from_numpy(A).to(dev)
    dt_, st_ = torch.from_numpy(d).to(dev), torch.from_numpy(sig).to(dev)
    D = torch.empty((B, c), dtype=torch.float64, device=dev)
    P.bootstrap_data(dt_, st_, torch.from_numpy(eps).to(dev), kin0, c, D)
    assert np.array_equal(D.cpu().numpy(), D_o)
    w_g, status, reps = multi_solve(At, D, st_, wt)
    assert _converged(status, reps)
    cws = torch.empty(P.chi2_workspace_bytes(c), dtype=torch.uint8, device=dev)
    x_g = [P.chi2(At, torch.from_numpy(w_g[b]).to(dev), dt_, st_, kin0, c, cws) for b in range(B)]
    x_o = []
    for b in range(4):
        w_o, _ = oracle_solve(A, D_o[b], sig, wt, 1e-2)
        x_o.append(N.chi2(A, w_o, d, sig, kin0, c))
        assert abs(x_g[b] / x_o[-1] - 1) < CHI2_TOL
    m_g, m_o = P.chi2_model(x_g[:4]), BS.chi2_model(x_o)
    print("chi2_b", np.round(x_g, 3), "chi2_model of 4", m_g, m_o)
    assert abs(m_g / m_o - 1) < CHI2_TOL
    m_all = P.chi2_model(x_g)
    assert min(x_g) <= m_all <= min(x_g) + 2 * np.log(B)


def test_warm_started_bootstraps(gpu, multi_dense):
    """Twelve realisations warm-started from the observed data's weights (x = z
    = w0 / w~ with the dual that makes that point stationary for each
    realisation's data) reach the same weights as cold starts (within 1e-4 in
    L1: both meet the KKT tolerance of the unique minimiser) in fewer
    iterations, and two of them match the oracle's exact NNLS to the parity
    bar.  With either kind of pass over the matrix."""
    from tests.test_gpu_solve import gpu_solve
    n, c, cb = 1501, 600, 200
    blocks = [(0, cb), (cb, c)]
    A = W.sparse_lognormal_matrix(n, blocks, density=0.1, seed=6)
    d, sig, wt = mock_problem(A, blocks, 4, 0.02, 0.02)
    w_base, st_b, rep_b, _ = gpu_solve(A, d, sig, wt, 1e-2, 1)
    assert st_b == 0
    D = BS.bootstrap_data(d, sig, W.bootstrap_eps(12, c, seed=2), cb, c)
    w_c, st_c, reps_c = multi_solve(A, D, sig, wt)
    w_w, st_w, reps_w = multi_solve(A, D, sig, wt, w0=w_base)
    it_c = max(r.refine_iters for r in reps_c)
    it_w = max(r.refine_iters for r in reps_w)
    print("iterations cold", it_c, "warm", it_w, "kkt warm max", max(r.kkt for r in reps_w))
    assert _converged(st_c, reps_c) and _converged(st_w, reps_w)
    assert it_w < it_c
    for b in range(D.shape[0]):
        assert np.abs(w_w[b] - w_c[b]).sum() <= 1e-4 * np.abs(w_c[b]).sum(), b
    for b in range(2):
        w_o, _ = oracle_solve(A, D[b], sig, wt, 1e-2)
        assert np.abs(w_w[b] - w_o).sum() / np.abs(w_o).sum() < W_L1_TOL


def test_warm_start_at_the_solution_converges_at_once(gpu):
    """Batched problems of different sizes started from their own solutions
    (w0 in the layout of w; their cold solves take 180-790 iterations) are
    converged by the second check (the iterations from a point within the KKT
    tolerance may first drift across it, by rounding) and return the same
    weights; w0_shared with unequal problem sizes is refused."""
    import torch
    P = lib()
    c = 500
    blocks = [(0, 150), (150, c)]
    sizes = [700, 1201, 333]
    mats, ds, sigs, wts = [], [], [], []
    for k, n in enumerate(sizes):
        A = W.sparse_lognormal_matrix(n, blocks, density=0.1, seed=20 + k)
        d, sig, wt = mock_problem(A, blocks, 30 + k, 0.02, 0.02)
        mats.append(A); ds.append(d); sigs.append(sig); wts.append(wt)
    A = np.concatenate(mats)
    off = np.concatenate([[0], np.cumsum(sizes)])
    dev = torch.device("cuda:0")
    At = torch.from_numpy(A).to(dev)
    dt = torch.from_numpy(np.stack(ds)).to(dev)
    st = torch.from_numpy(np.stack(sigs)).to(dev)
    opts = P._lib.SolveOpts()
    opts.gram, opts.nu = 1, 1e-2
    w = torch.empty(A.shape[0], dtype=torch.float64, device=dev)
    ws = torch.empty(P.solve_batched_workspace_bytes(off, c, opts), dtype=torch.uint8, device=dev)
    status, reps = P.solve_weights_batched(At, off, dt, st, wts, -1.0, opts, w, ws)
    assert status == 0
    w0 = w.clone()
    opts.w0 = w0.data_ptr()
    w2 = torch.empty_like(w)
    status2, reps2 = P.solve_weights_batched(At, off, dt, st, wts, -1.0, opts, w2, ws)
    print([(r.refine_iters, r.kkt) for r in reps2])
    assert status2 == 0 and all(r.refine_iters <= 20 for r in reps2)
    assert torch.sum(torch.abs(w2 - w)).item() <= 1e-5 * torch.sum(torch.abs(w)).item()
    opts.w0_shared = 1
    with pytest.raises(P.SchwError):
        P.solve_weights_batched(At, off, dt, st, wts, -1.0, opts, w2, ws)


def test_multi_rhs_count_quantum(gpu):
    """Bootstrap realisations on a count matrix (the oracle's time fractions of
    the small model, 1,000 steps) with the compressed passes per group of data
    vectors: with the quantum 1 / (ncopy n_steps) the copies hold the counts,
    and every realisation's weights meet the KKT tolerance by the oracle's
    residual (Eq. 4), chi^2 agrees with the value copies' weights, and the first
    realisation's weights match the oracle's within the parity bar."""
    import torch
    import oracle as O
    P = lib()
    dev = torch.device("cuda:0")
    cfg = W.SMALL
    n_steps = 1000
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=n_steps)
    opot = O.make_pot(cfg["components"], cfg["omega"])
    oobs = O.make_obs(cfg["obs"], O.euler_matrix(*cfg["euler"]))
    c_o, _, _, _ = O.integrate_and_bin(opot, oobs, ics, dt, n_steps)
    A = O.time_fractions(c_o, n_steps)
    n, c = A.shape
    blocks = W.blocks(cfg["obs"])
    kin0 = blocks[1][0]
    d = A.T @ W.mock_draw(n, cfg["mock"]["seed"])
    sig = N.sigma_from_data(d, blocks, 0.01)
    wt = N.w_tilde_from_data(d, blocks[0], n)
    B = 12
    D_o = BS.bootstrap_data(d, sig, W.bootstrap_eps(B, c, seed=8), kin0, c)
    q = P.count_quantum(P.obs_spec(cfg["obs"]), n_steps)
    old = P.get_tuning("multi_dense")
    try:
        P.set_tuning("multi_dense", 2)
        w_v, st_v, reps_v = multi_solve(A, D_o, sig, wt)
        w_q, st_q, reps_q = multi_solve(A, D_o, sig, wt, quantum=q)
    finally:
        P.set_tuning("multi_dense", old)
    print("iters", [r.refine_iters for r in reps_v], [r.refine_iters for r in reps_q])
    assert _converged(st_v, reps_v) and _converged(st_q, reps_q)
    for b in range(B):
        kkt = N.kkt_residual_orbit_matrix(A, D_o[b], sig, wt, reps_q[b].mu, w_q[b])
        x_q, x_v = (N.chi2(A, w_[b], D_o[b], sig, kin0, c) for w_ in (w_q, w_v))
        assert kkt <= 1.5e-7 and abs(x_q / x_v - 1) < 1e-5, (b, kkt, x_q, x_v)
    w_o, _ = oracle_solve(A, D_o[0], sig, wt, 1e-2)
    assert np.abs(w_q[0] - w_o).sum() / np.abs(w_o).sum() < W_L1_TOL
