"""The weight solve at the full size of its precision study: 200,000 orbits x
(mass grid + 900 apertures x 30 velocity bins) constraints, a synthetic
sparse log-normal orbit matrix in FP32 (each entry nonzero with probability
0.05, LogNormal(0, 1), each orbit's row normalised to 1 within each block),
mock data from a seeded 10% subset with Exp(1) weights plus 2% noise.

The exact minimiser is out of the oracle's reach at this size, so parity is
checked by properties that hold at any size: the oracle re-evaluates, in FP64
on the CPU from a CSR copy of the same matrix, the regularisation, the KKT
natural residual of the GPU's weights (Eq. 4 is strictly convex, so a small
residual certifies the unique minimiser) and their chi^2 (Eq. 5); and the
solves with different Gram precisions (bf16x3, fp32, plain bf16) land on the
same weights.
"""
import numpy as np
import pytest

import workloads as W
from oracle import nnls as N
from tests.gpu_common import lib

pytestmark = pytest.mark.gpu

N_ORB = 200000


def _build(mass_cells, seed=6):
    """The matrix on the GPU (torch, seeded), its CSR copy on the host, the
    mock data, sigma and w_tilde computed on the host in FP64."""
    import scipy.sparse as sp
    import torch
    dev = torch.device("cuda:0")
    n, c = N_ORB, mass_cells + 900 * 30
    blocks = [(0, mass_cells), (mass_cells, c)]
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    A = torch.zeros((n, c), dtype=torch.float32, device=dev)
    parts = []
    chunk = 10000
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        for b0, b1 in blocks:
            m = torch.rand((r1 - r0, b1 - b0), generator=g, device=dev) < 0.05
            v = torch.where(m, torch.exp(torch.randn((r1 - r0, b1 - b0), generator=g, device=dev)),
                            torch.zeros((), device=dev))
            s = v.sum(1, keepdim=True)
            s[s == 0] = 1.0
            A[r0:r1, b0:b1] = (v / s).to(torch.float32)
        csr = A[r0:r1].to_sparse_csr()
        parts.append(sp.csr_matrix((csr.values().cpu().numpy().astype(np.float64),
                                    csr.col_indices().cpu().numpy().astype(np.int32),
                                    csr.crow_indices().cpu().numpy().astype(np.int64)), shape=(r1 - r0, c)))
        del csr
    A_csr = sp.vstack(parts, format="csr")
    del parts
    d = np.asarray(A_csr.T @ W.mock_draw(n, seed)).ravel()
    d = d * (1 + 0.02 * W.noise_draw(c, seed))
    sig = N.sigma_from_data(d, blocks, 0.02)
    wt = N.w_tilde_from_data(d, blocks[0], n)
    return A, A_csr, d, sig, wt, blocks


def _solve(A, d, sig, wt, gram):
    import torch
    P = lib()
    dev = A.device
    opts = P._lib.SolveOpts()
    opts.gram, opts.nu = gram, 1e-2
    w = torch.empty(A.shape[0], dtype=torch.float64, device=dev)
    ws = torch.empty(P.solve_workspace_bytes(A.shape[0], A.shape[1], opts), dtype=torch.uint8, device=dev)
    d_t, s_t = torch.from_numpy(d).to(dev), torch.from_numpy(sig).to(dev)
    status, rep = P.solve_weights(A, d_t, s_t, wt, -1.0, opts, w, ws)
    del ws
    cws = torch.empty(P.chi2_workspace_bytes(A.shape[1]), dtype=torch.uint8, device=dev)
    return w.cpu().numpy(), status, rep, (w, d_t, s_t, cws)


@pytest.mark.parametrize("mass_cells", [30 * 30 * 20, 30 * 20 * 10], ids=["45000", "33000"])
def test_full_size_solve_certified_by_the_oracle(gpu, mass_cells):
    P = lib()
    A, A_csr, d, sig, wt, blocks = _build(mass_cells)
    kin0, c = blocks[1]
    mu_o = N.relative_mu_orbit_matrix(A_csr, sig, wt, 1e-2)
    print(f"{A.shape[0]} x {A.shape[1]}, nnz {A_csr.nnz}")
    grams = [P.SW_GRAM_BF16X3] if mass_cells == 18000 else [P.SW_GRAM_BF16X3, P.SW_GRAM_F32, P.SW_GRAM_BF16]
    sols = {}
    for gram in grams:
        w, status, rep, (w_t, d_t, s_t, cws) = _solve(A, d, sig, wt, gram)
        kkt_o = N.kkt_residual_orbit_matrix(A_csr, d, sig, wt, rep.mu, w)
        x_g = P.chi2(A, w_t, d_t, s_t, kin0, c, cws)
        x_o = N.chi2(A_csr, w, d, sig, kin0, c)
        print(f"gram {gram}: status {status}, iterations {rep.refine_iters}, kkt {rep.kkt:.2e} (oracle {kkt_o:.2e}), "
              f"chi2 {x_g:.8g} (oracle {x_o:.8g}), gram {rep.t_gram_ms:.0f} ms, factor {rep.t_factor_ms:.0f} ms, "
              f"iterations {rep.t_refine_ms:.0f} ms")
        assert rep.mu == pytest.approx(mu_o, rel=1e-4)
        assert abs(x_g / x_o - 1) < 1e-10
        if gram != P.SW_GRAM_BF16:
            assert status == 0 and kkt_o < 1e-6
        if status == 0:
            sols[gram] = (w, x_o)
    # every mode meets the same KKT tolerance; the weights of this ill-conditioned
    # problem still move within it (the Gram's precision changes the iterates'
    # path and so where within the tolerance each solve stops: measured 2e-4 in
    # L1 between fp32 and bf16x3), so every mode is held to the parity bar
    ref_w, ref_x = sols[P.SW_GRAM_BF16X3]
    for gram, (w, x) in sols.items():
        l1 = np.abs(w - ref_w).sum() / np.abs(ref_w).sum()
        print(f"gram {gram} vs bf16x3: weights L1 {l1:.2e}, chi2 {x / ref_x - 1:.2e}")
        assert l1 < 1e-2 and abs(x / ref_x - 1) < 1e-3


def test_barred_build_solve_certified_by_the_oracle(gpu):
    """The benchmark's own headline problem: the barred model's 100,000 orbits x
    10,000 FP32 steps binned into 48,000 constraints on the GPU, its mock (10%
    subset with Exp(1) weights + 2% noise, computed on the host from a CSR copy of
    that matrix), the drift-flagged orbits masked, the bf16x3 solve; the oracle
    re-evaluates in FP64 the regularisation, the KKT natural residual of the
    GPU's weights and their chi^2 (kinematic block, Eq. 5).  Solved with fp32
    values in the compressed copies and, as the benchmark runs it, with the
    counts (the KKT residual then on the exact multiples of the quantum)."""
    import scipy.sparse as sp
    import torch
    P = lib()
    cfg = W.BARRED
    dev = torch.device("cuda:0")
    n, n_steps = cfg["n_orb"], cfg["n_steps"]
    ics, dt = W.disc_ics(W.load_table(cfg["table"]), n, seed=cfg["ic_seed"], n_steps=n_steps)
    pot = P.build_potential(cfg["components"], cfg["omega"], cfg["euler"])
    obs = P.obs_spec(cfg["obs"])
    nc = P.ncon(obs)
    A = torch.empty((n, nc), dtype=torch.float32, device=dev)
    ov = torch.empty((n, 2), dtype=torch.float64, device=dev)
    dr = torch.empty(n, dtype=torch.float64, device=dev)
    fl = torch.empty(n, dtype=torch.uint8, device=dev)
    iws = torch.empty(P.integrate_workspace_bytes(obs, 1, n, n_steps, P.SW_F32), dtype=torch.uint8, device=dev)
    P.integrate_and_bin(pot, [0, n], torch.from_numpy(ics).to(dev, torch.float32),
                        torch.from_numpy(dt).to(dev, torch.float32), n_steps, obs, A, ov, dr, fl, iws)
    torch.cuda.synchronize()
    del iws
    parts = []
    for r0 in range(0, n, 10000):
        csr = A[r0:r0 + 10000].to_sparse_csr()
        parts.append(sp.csr_matrix((csr.values().cpu().numpy().astype(np.float64),
                                    csr.col_indices().cpu().numpy().astype(np.int32),
                                    csr.crow_indices().cpu().numpy().astype(np.int64)),
                                   shape=(min(10000, n - r0), nc)))
        del csr
    A_csr = sp.vstack(parts, format="csr")
    del parts
    blocks = W.blocks(cfg["obs"])
    d = np.asarray(A_csr.T @ W.mock_draw(n, cfg["mock"]["seed"])).ravel()
    d = d * (1 + cfg["mock"]["noise"] * W.noise_draw(nc, cfg["mock"]["seed"]))
    sig = N.sigma_from_data(d, blocks, cfg["mock"]["tol"])
    wt = N.w_tilde_from_data(d, blocks[0], n)
    mask = fl.cpu().numpy()
    keep = np.flatnonzero(mask == 0)
    mu_o = N.relative_mu_orbit_matrix(A_csr[keep], sig, wt, 1e-2)
    # the count copies: the solve computes with the exact multiples k q that A rounds
    q = P.count_quantum(obs, n_steps)
    A_k = A_csr.copy()
    A_k.data = np.rint(A_k.data / q) * q
    for quantum, A_ref in ((0.0, A_csr), (q, A_k)):
        opts = P._lib.SolveOpts()
        opts.gram, opts.nu, opts.use_graph = P.SW_GRAM_BF16X3, 1e-2, 1
        opts.mask = fl.data_ptr()
        opts.quantum = quantum
        w_t = torch.empty(n, dtype=torch.float64, device=dev)
        ws = torch.empty(P.solve_workspace_bytes(n, nc, opts), dtype=torch.uint8, device=dev)
        d_t, s_t = torch.from_numpy(d).to(dev), torch.from_numpy(sig).to(dev)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            status, rep = P.solve_weights(A, d_t, s_t, wt, -1.0, opts, w_t, ws)
            cws = torch.empty(P.chi2_workspace_bytes(nc), dtype=torch.uint8, device=dev)
            x_g = P.chi2(A, w_t, d_t, s_t, blocks[1][0], blocks[1][1], cws)
        torch.cuda.synchronize()
        del ws
        w = w_t.cpu().numpy()
        assert np.all(w[mask != 0] == 0) and np.all(w >= 0)
        kkt_o = N.kkt_residual_orbit_matrix(A_ref[keep], d, sig, wt, rep.mu, w[keep])
        x_o = N.chi2(A_csr, w, d, sig, blocks[1][0], blocks[1][1])
        print(f"barred build, quantum {quantum:g}: nnz {A_csr.nnz}, masked {int((mask != 0).sum())}, status {status}, "
              f"iterations {rep.iters}+{rep.refine_iters}, kkt {rep.kkt:.2e} (oracle {kkt_o:.2e}), mu {rep.mu:.6g} "
              f"(oracle {mu_o:.6g}), chi2 {x_g:.10g} (oracle {x_o:.10g})")
        assert status == 0
        assert rep.mu == pytest.approx(mu_o, rel=1e-4)
        assert kkt_o < 1e-6
        assert abs(x_g / x_o - 1) < 1e-10
