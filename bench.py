"""Benchmark: one Schwarzschild model build per step on one MI355X.

A step is one pass of the whole hot path for one trial potential of the
barred model (MN disc + rotating Ferrers n=2 bar + flattened NFW halo,
100,000 orbits x 10,000 FP32 steps, 30x30x20 mass grid + 1,000 apertures x 30
velocity bins = 48,000 constraints): integrate_and_bin -> solve_weights ->
chi2, with every input already resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload barred|small]
                  [--bootstrap B]   (also B bootstrap solves per build, Eq. 6)
  python bench.py --workload paper  (the paper's own pipeline: Jeans initial conditions
                  x 4 dithers, BS23 at rtol 1e-4 for 5,000 steps, cylindrical grid,
                  ~600 apertures, Gauss-Hermite fit, 100 bootstrap solves, chi^2_model)
  python bench.py --workload walkers | surrogate   (batched walkers; DA-MCMC)

The default line's `roofline` is the dominant stage's, its `achieved` the
method's algorithmic work over the stage time; `cpu_baseline` is the FP64
oracle's whole build of a seeded orbit subsample, and `errors_vs_oracle` the
GPU's errors against the oracle on that subsample and on the headline solve.
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

METRIC = "orbit-steps/s and model builds/s vs FP64 oracle; surrogate-MCMC models/s @Δχ²<1"
PEAK_HBM = 8.0e12           # bytes/s
PEAK_BF16 = 2.5e15          # dense MFMA flop/s
PEAK_F32_MFMA = 157.3e12
PEAK_F32_VALU = 157.3e12     # vector FP32 with packed FP32 (this build compiles without it: 78.6)
PEAK_F64_VALU = 78.6e12
# FP32 (FP64 for the small model) flops per orbit-step of each workload's
# integrate-and-bin, counted from the kernel's formulas (FMA = 2)
FLOP_PER_ORBIT_STEP = {"mn_ferrers_nfwq_100k_orbits_10k_steps_f32": 686.0,
                       "plummer_mn_2k_orbits_1k_steps_f64": 168.0}
# HBM bytes measured by rocprofv3 FETCH_SIZE + WRITE_SIZE (calibrated on a 4 GiB
# copy) for the kernels as they stand: per build for the factorisation, per
# iteration for the ADMM stages; stages not listed were not measured
BARRED = "mn_ferrers_nfwq_100k_orbits_10k_steps_f32"
TRAFFIC = {(BARRED, "factorise"): 748 * (1.256e9 + 0.1149e9) + 748 * (0.01296e9 + 0.01229e9),
           (BARRED, "gram"): 831.3e9 + 4.633e9}
# per FP64 iteration (two passes over the count copies, and a pair more every 10 iterations for U^T U x
# and for the KKT check; the two triangles; the Anderson kernels)
TRAFFIC_PER_ITER = {(BARRED, "refine_fp64"): 1.2 * (1.895e9 + 1.854e9) + 2 * 4.634e9 + 0.06e9}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def mock_sigma(d, blocks, tol, floor=1e-3):
    """Mock uncertainties: relative tolerance with a floor at `floor` x block maximum."""
    s = np.empty_like(d)
    for b0, b1 in blocks:
        top = float(np.max(d[b0:b1])) if b1 > b0 else 0.0
        s[b0:b1] = tol * np.maximum(d[b0:b1], floor * top)
    s[s <= 0] = tol * floor
    return s


def host_threads():
    """Threads the oracle runs on: the CPUs this process may use, capped by
    OMP_NUM_THREADS when it is set; and the physical cores lscpu reports."""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    threads = min(avail, omp) if omp > 0 else avail
    phys = None
    try:
        import subprocess
        out = subprocess.run(["lscpu", "-p=Core,Socket"], capture_output=True, text=True, timeout=10).stdout
        phys = len({ln for ln in out.splitlines() if ln and not ln.startswith("#")})
    except Exception:
        pass
    return threads, phys


def _csr_copy(A):
    """Host FP64 CSR copy of a device orbit matrix (row chunks converted on the GPU)."""
    import scipy.sparse as sp
    n, c = A.shape
    parts = []
    for r0 in range(0, n, 10000):
        csr = A[r0:r0 + 10000].to_sparse_csr()
        parts.append(sp.csr_matrix((csr.values().cpu().numpy().astype(np.float64),
                                    csr.col_indices().cpu().numpy().astype(np.int32),
                                    csr.crow_indices().cpu().numpy().astype(np.int64)), shape=(min(10000, n - r0), c)))
        del csr
    return sp.vstack(parts, format="csr")


def cpu_baseline_leg(cfg, run):
    """The oracle leg: times the FP64 oracle's whole model build (integrate+bin
    with its fixed 64-point Gauss-Legendre Ferrers timing mode, exact NNLS,
    chi^2) on the seeded 1,000-orbit subsample of the workload, and states the
    GPU's errors against the oracle on that subsample and on the headline solve:
      * integration: per-orbit row L1 between the GPU's FP32 rows and the
        oracle's FP64 rows (the floor: the oracle whose state is rounded to
        binary32 every step), |drift difference|;
      * weight solve on one matrix (the oracle's FP64 subsample matrix in FP32,
        its own mock, the oracle's drift mask): weights L1, chi^2;
      * headline solve: the oracle's FP64 KKT residual and chi^2 of the GPU's
        weights from a CSR copy of the GPU's matrix.
    `run` holds the GPU objects of the timed build."""
    import oracle as O
    from oracle import nnls as N
    P, torch, dev = run["P"], run["torch"], run["dev"]
    threads, phys = host_threads()
    n_steps = cfg["n_steps"]
    blocks = W.blocks(cfg["obs"])
    kin0, kin1 = blocks[1]
    sub = W.subsample_draw(cfg["n_orb"], cfg["subsample"]["n"], cfg["subsample"]["seed"])
    ns = len(sub)
    f64 = cfg["dtype"] == "f64"
    npd = np.float64 if f64 else np.float32
    ic = np.ascontiguousarray(run["ics"][:, sub].astype(npd))
    dt = np.ascontiguousarray(run["dt"][sub].astype(npd))
    ic64, dt64 = ic.astype(np.float64), dt.astype(np.float64)
    pot = O.make_pot(cfg["components"], cfg["omega"])
    ob = O.make_obs(cfg["obs"], O.euler_matrix(*cfg["euler"]))
    O.set_ferrers_rule(64)
    try:
        t0 = time.perf_counter()
        c_o, _, dr_o, fl_o = O.integrate_and_bin(pot, ob, ic64, dt64, n_steps, nthreads=threads)
        A_o = O.time_fractions(c_o, n_steps)
        w_mock = W.mock_draw(ns, cfg["mock"]["seed"])
        nc = A_o.shape[1]
        d_s = A_o.T @ w_mock
        if cfg["mock"]["noise"] > 0:
            d_s = d_s * (1 + cfg["mock"]["noise"] * W.noise_draw(nc, cfg["mock"]["seed"]))
        sig_s = N.sigma_from_data(d_s, blocks, cfg["mock"]["tol"])
        wt_s = N.w_tilde_from_data(d_s, blocks[0], ns)
        mask_o = ((fl_o & 1) != 0) | ((fl_o & 2) != 0)
        keep = np.flatnonzero(~mask_o)
        U, y = N.scale_problem(A_o[keep], d_s, sig_s, wt_s)
        mu_s = N.relative_mu(U, 1e-2)
        wp = N.nnls_oracle(U, y, mu_s)
        w_o = np.zeros(ns)
        w_o[keep] = wp * wt_s
        x_o = N.chi2(A_o, w_o, d_s, sig_s, kin0, kin1)
        el = time.perf_counter() - t0
        f32_floor = None
        if not f64:
            c_p, *_ = O.integrate_and_bin(pot, ob, ic64, dt64, n_steps, nthreads=threads, f32_state=True)
            f32_floor = O.time_fractions(c_p, n_steps)
    finally:
        O.set_ferrers_rule(0)
    errors = {}
    # GPU integration of the same subsample, same launch configuration
    td = torch.float64 if f64 else torch.float32
    code = P.SW_F64 if f64 else P.SW_F32
    obs = run["obs"]
    A_g = torch.empty((ns, nc), dtype=td, device=dev)
    ov = torch.empty((ns, 2), dtype=torch.float64, device=dev)
    dr = torch.empty(ns, dtype=torch.float64, device=dev)
    fl = torch.empty(ns, dtype=torch.uint8, device=dev)
    ws = torch.empty(P.integrate_workspace_bytes(obs, 1, ns, n_steps, code), dtype=torch.uint8, device=dev)
    P.integrate_and_bin(run["pot"], [0, ns], torch.from_numpy(ic).to(dev), torch.from_numpy(dt).to(dev), n_steps, obs,
                        A_g, ov, dr, fl, ws)
    torch.cuda.synchronize()
    Ag = A_g.cpu().numpy().astype(np.float64)
    l1 = np.abs(Ag - A_o).sum(1) / 2
    ddr = np.abs(dr.cpu().numpy() - dr_o)
    errors["integrate_subsample"] = {
        "orbits": ns, "row_l1_median": float(np.median(l1)), "row_l1_p90": float(np.percentile(l1, 90)),
        "drift_absdiff_median": float(np.median(ddr)), "drift_absdiff_p99": float(np.percentile(ddr, 99)),
        "flagged_frac_gpu": float(np.mean(fl.cpu().numpy() & 1)), "flagged_frac_oracle": float(np.mean(fl_o & 1))}
    if f32_floor is not None:
        l1p = np.abs(f32_floor - A_o).sum(1) / 2
        errors["integrate_subsample"].update(row_l1_floor_median=float(np.median(l1p)),
                                             row_l1_floor_p90=float(np.percentile(l1p, 90)))
    else:
        errors["integrate_subsample"]["bit_exact"] = bool(np.array_equal(Ag, A_o))
    # the weight solve on one matrix: the oracle's subsample matrix and mock
    A_s = torch.from_numpy(A_o.astype(npd)).to(dev)
    mk = torch.from_numpy(mask_o.astype(np.uint8)).to(dev)
    opts = type(run["opts"]).from_buffer_copy(run["opts"])
    opts.mask = mk.data_ptr()
    w_s = torch.empty(ns, dtype=torch.float64, device=dev)
    sws = torch.empty(P.solve_workspace_bytes(ns, nc, opts), dtype=torch.uint8, device=dev)
    d_t, s_t = torch.from_numpy(d_s).to(dev), torch.from_numpy(sig_s).to(dev)
    cws = torch.empty(P.chi2_workspace_bytes(nc), dtype=torch.uint8, device=dev)
    with torch.cuda.stream(run["stream"]):
        st, rep = P.solve_weights(A_s, d_t, s_t, wt_s, -1.0, opts, w_s, sws)
        x_g = P.chi2(A_s, w_s, d_t, s_t, kin0, kin1, cws)
    torch.cuda.synchronize()
    wg = w_s.cpu().numpy()
    # the GPU solved the FP32-rounded matrix: the oracle's chi^2 of the GPU's weights is taken on that same matrix
    A_s64 = A_o.astype(npd).astype(np.float64)
    errors["solve_subsample"] = {
        "orbits": ns, "status": st, "weights_l1_rel": float(np.abs(wg - w_o).sum() / np.abs(w_o).sum()),
        "chi2_rel": float(abs(x_g / x_o - 1)), "chi2_rel_same_matrix": float(abs(x_g / N.chi2(A_s64, wg, d_s, sig_s,
                                                                                               kin0, kin1) - 1)),
        "kkt_gpu": rep.kkt}
    del A_s, sws, ws, A_g
    # the headline solve: the oracle's certificate from a CSR copy of the GPU's own matrix
    A_csr = _csr_copy(run["A"])
    w = run["w"].cpu().numpy()
    d, sig, wt = run["d"], run["sig"], run["w_tilde"]
    keep_h = np.flatnonzero(run["fl"].cpu().numpy() == 0)
    kkt_o = N.kkt_residual_orbit_matrix(A_csr[keep_h], d, sig, wt, run["mu"], w[keep_h])
    x_h = N.chi2(A_csr, w, d, sig, kin0, kin1)
    errors["headline_solve"] = {"kkt_oracle": kkt_o, "kkt_gpu": run["kkt"], "chi2_rel": float(abs(run["chi2"] / x_h - 1)),
                                "mu_rel": float(abs(run["mu"] / N.relative_mu_orbit_matrix(A_csr[keep_h], sig, wt, 1e-2)
                                                    - 1))}
    del A_csr
    base = {"value": ns * n_steps / el, "unit": "orbit-steps/s", "cores": threads, "physical_cores": phys,
            "kind": "oracle",
            "sample": f"whole model build by the FP64 oracle (integrate+bin with its 64-point Gauss-Legendre "
                      f"Ferrers timing mode, exact NNLS by active set, chi^2) of the seeded {ns}-orbit subsample x "
                      f"{n_steps} steps with the workload's {nc} constraints and a mock of that subsample "
                      f"({el:.1f} s on {threads} threads); its solve is smaller than the full library's"}
    return base, errors


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="barred", choices=["barred", "small", "walkers", "surrogate", "paper"])
    ap.add_argument("--bs23-steps", type=int, default=0, help="paper: accepted BS23 steps (0: the paper's 5,000)")
    ap.add_argument("--refit-epochs", type=int, default=150,
                    help="surrogate workload: epochs of each local refit during the burn-in")
    ap.add_argument("--no-quantum", action="store_true",
                    help="store the compressed copies of a count matrix as fp32 values, not as counts")
    ap.add_argument("--warm-bootstraps", action="store_true",
                    help="paper: fit the observed maps first and start the bootstrap solves from those weights")
    ap.add_argument("--bs23-precision", default="f32", choices=["f32", "f64"],
                    help="paper: arithmetic of the BS23 integration (the drift check is FP64 either way)")
    ap.add_argument("--n-train", type=int, default=20000, help="surrogate: training builds")
    ap.add_argument("--mcmc-steps", type=int, default=200, help="surrogate: DA-MCMC steps per walker")
    ap.add_argument("--gram", default="bf16x3", choices=["bf16", "bf16x3", "f32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-iter", type=int, default=0, help="cap of the FP32 ADMM stage (0: library default)")
    ap.add_argument("--refine-iter", type=int, default=0, help="cap of the FP64 stage (0: library default)")
    ap.add_argument("--no-graph", action="store_true", help="launch the solve iterations one by one")
    ap.add_argument("--no-accel", action="store_true", help="plain ADMM (no Anderson acceleration)")
    ap.add_argument("--rho", type=float, default=None,
                    help="ADMM penalty as a multiple of trace(U U^T)/N (default: the library's, 1)")
    ap.add_argument("--bootstrap", type=int, default=0,
                    help="also solve this many bootstrap realisations of the data per build (shared matrix) "
                         "and report chi2_model")
    ap.add_argument("--refine-passes", type=int, choices=[2, 4], default=None,
                    help="passes over A per FP64 iteration (2: U^T U x carried, 4: residual from A)")
    ap.add_argument("--factor-gemm", type=int, choices=[0, 1], default=None,
                    help="factorisation products on fp32 MFMA (0) or bf16x3 MFMA (1); default: the library's")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="end with a 4 GiB device-to-device copy (scale for the HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is described in DESIGN.md but not run.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2607_00117_amd as P

    if args.factor_gemm is not None:
        P.set_tuning("factor_gemm", args.factor_gemm)
    if args.refine_passes is not None:
        P.set_tuning("refine_passes", args.refine_passes)
    if args.workload == "walkers":
        return bench_walkers(args)
    if args.workload == "paper":
        return bench_paper(args)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    cfg = W.BARRED if args.workload == "barred" else W.SMALL
    dev = torch.device("cuda:0")
    f64 = cfg["dtype"] == "f64"
    td = torch.float64 if f64 else torch.float32
    code = P.SW_F64 if f64 else P.SW_F32
    n, n_steps = cfg["n_orb"], cfg["n_steps"]
    table = W.load_table(cfg["table"])
    if cfg is W.BARRED:
        ics, dt = W.disc_ics(table, n, seed=cfg["ic_seed"], n_steps=n_steps)
    else:
        ics, dt = W.grid_ics(table, seed=cfg["ic_seed"], n_steps=n_steps)
    pot = P.build_potential(cfg["components"], cfg["omega"], cfg["euler"])
    obs = P.obs_spec(cfg["obs"])
    nc = P.ncon(obs)
    blocks = W.blocks(cfg["obs"])
    ic_t = torch.from_numpy(np.ascontiguousarray(ics)).to(dev, td)
    dt_t = torch.from_numpy(np.ascontiguousarray(dt)).to(dev, td)
    A = torch.empty((n, nc), dtype=td, device=dev)
    ov = torch.empty((n, 2), dtype=torch.float64, device=dev)
    dr = torch.empty(n, dtype=torch.float64, device=dev)
    fl = torch.empty(n, dtype=torch.uint8, device=dev)
    iws = torch.empty(P.integrate_workspace_bytes(obs, 1, n, n_steps, code), dtype=torch.uint8, device=dev)
    log(f"workload {cfg['name']}: {n} orbits x {n_steps} steps, {nc} constraints")

    # mock data (untimed): the binned sum of a seeded 10% orbit subset with Exp(1) weights, plus noise
    P.integrate_and_bin(pot, [0, n], ic_t, dt_t, n_steps, obs, A, ov, dr, fl, iws)
    w_mock = torch.from_numpy(W.mock_draw(n, cfg["mock"]["seed"])).to(dev)
    d_t = torch.empty(nc, dtype=torch.float64, device=dev)
    P.model_observables(A, w_mock, d_t)
    torch.cuda.synchronize()
    d = d_t.cpu().numpy()
    if cfg["mock"]["noise"] > 0:
        d = d * (1 + cfg["mock"]["noise"] * W.noise_draw(nc, cfg["mock"]["seed"]))
    sig = mock_sigma(d, blocks, cfg["mock"]["tol"])
    w_tilde = float(np.sum(d[blocks[0][0]:blocks[0][1]])) / n
    d_t = torch.from_numpy(d).to(dev)
    s_t = torch.from_numpy(sig).to(dev)
    mask = fl  # orbits above the Jacobi-drift cut are excluded (Sec. 2.2.2)
    opts = P._lib.SolveOpts()
    opts.gram = {"bf16": P.SW_GRAM_BF16, "bf16x3": P.SW_GRAM_BF16X3, "f32": P.SW_GRAM_F32}[args.gram]
    opts.nu = 1e-2
    opts.mask = mask.data_ptr()
    if not args.no_quantum:
        opts.quantum = P.count_quantum(obs, n_steps)  # the compressed copies hold counts
    if args.rho is not None:
        opts.rho = -args.rho
    w = torch.empty(n, dtype=torch.float64, device=dev)
    sws = torch.empty(P.solve_workspace_bytes(n, nc, opts), dtype=torch.uint8, device=dev)
    cws = torch.empty(P.chi2_workspace_bytes(nc), dtype=torch.uint8, device=dev)
    log(f"workspaces: integrate {iws.numel() / 1e9:.1f} GB, solve {sws.numel() / 1e9:.1f} GB")

    reps, chis, t_int = [], [], []
    boot = []  # per step: (status, reports, chi2_b, chi2_model, ms)
    n_boot = args.bootstrap
    kin0 = blocks[1][0]
    if n_boot > 0:
        # bootstrap realisations of the observed maps (Sec. 2.3): seeded normal deviates, resident in HBM
        eps_t = torch.from_numpy(W.bootstrap_eps(n_boot, nc, seed=9)).to(dev)
        D_t = torch.empty((n_boot, nc), dtype=torch.float64, device=dev)
        w_b = torch.empty((n_boot, n), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()  # default priority; the solve captures its iterations into HIP graphs on it
    opts.use_graph = 0 if args.no_graph else 1
    opts.max_iter = args.max_iter
    opts.refine_iter = args.refine_iter
    if args.no_accel:
        opts.flags |= P.SW_SOLVE_NO_ACCEL
    if n_boot > 0:
        bws = torch.empty(P.solve_multi_workspace_bytes(n, nc, n_boot, opts), dtype=torch.uint8, device=dev)
        log(f"bootstrap: {n_boot} realisations, workspace {bws.numel() / 1e9:.1f} GB")

    def step():
        with torch.cuda.stream(stream):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            P.integrate_and_bin(pot, [0, n], ic_t, dt_t, n_steps, obs, A, ov, dr, fl, iws)
            e1.record()
            st, rep = P.solve_weights(A, d_t, s_t, w_tilde, -1.0, opts, w, sws)
            x = P.chi2(A, w, d_t, s_t, blocks[1][0], blocks[1][1], cws)
            if n_boot > 0:
                tb = time.perf_counter()
                P.bootstrap_data(d_t, s_t, eps_t, kin0, nc, D_t)
                stb, repb = P.solve_weights_multi(A, D_t, s_t, w_tilde, -1.0, opts, w_b, bws)
                xb = [P.chi2(A, w_b[b], d_t, s_t, kin0, nc, cws) for b in range(n_boot)]
                boot.append((stb, repb, xb, P.chi2_model(xb), 1e3 * (time.perf_counter() - tb)))
        torch.cuda.synchronize()
        t_int.append(e0.elapsed_time(e1))
        reps.append(rep.as_dict() | {"status": st})
        chis.append(x)

    for i in range(args.warmup):
        step()
        log(f"warmup {i}: integrate {t_int[-1]:.1f} ms, solve {reps[-1]}")
    reps.clear(); chis.clear(); t_int.clear(); boot.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log(f"step {i}: integrate {t_int[-1]:.1f} ms, chi2 {chis[-1]:.6g}, solve {reps[-1]}")
        if n_boot > 0:
            stb, repb, xb, xm, msb = boot[-1]
            rit = [r.refine_iters for r in repb]
            log(f"  bootstrap: {msb:.0f} ms, status {stb}, iterations max {max(rit)} median {int(np.median(rit))}, "
                f"kkt max {max(r.kkt for r in repb):.2e}, chi2_b {min(xb):.6g}..{max(xb):.6g}, chi2_model {xm:.6g}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = 1e3 * el / args.steps
    orbit_steps = n * n_steps
    value = orbit_steps * args.steps / el

    # rooflines per stage: the algorithmic work of the method per build (the unit of
    # `achieved`), over the stage's HIP-event time on the solve stream; the work the
    # kernels issue (extra MFMA passes of the bf16x3 split, the explicit inverse,
    # residual-correction passes, Anderson mixing) is reported beside it as `issued`
    t_prep = float(np.mean([r["t_prep_ms"] for r in reps]))
    t_gram = float(np.mean([r["t_gram_ms"] for r in reps]))
    t_factor = float(np.mean([r["t_factor_ms"] for r in reps]))
    t_admm = float(np.mean([r["t_admm_ms"] for r in reps]))
    t_ref = float(np.mean([r["t_refine_ms"] for r in reps]))
    t_i = float(np.mean(t_int))
    it1 = float(np.mean([r["iters"] for r in reps]))
    it2 = float(np.mean([r["refine_iters"] for r in reps]))
    nnz = float(reps[-1]["nnz"])
    C, N = float(nc), float(n)
    stages = {"integrate_and_bin": t_i, "solve_prep": t_prep, "gram": t_gram, "factorise": t_factor,
              "admm_fp32": t_admm, "refine_fp64": t_ref}
    # |U|: one pass over the orbit matrix as stored for the iterations (per nonzero a 16-bit
    # index and a 16-bit count, or an fp32 value; or the dense matrix); |L|: one triangle of
    # the fp32 inverse factor
    counts = opts.quantum > 0
    u_bytes = (4.0 if counts else 6.0) * nnz if nnz > 0 else N * C * (8.0 if f64 else 4.0)
    l_bytes = 4.0 * C * (C + 1) / 2.0
    per_iter = 2 * u_bytes + 2 * l_bytes
    # Anderson mixing per FP64 iteration: 91 vectors of N doubles read or written
    aa_bytes = 0.0 if args.no_accel else 91.0 * N * 8.0
    # passes over A per FP64 iteration: 2 with U^T U x carried (plus 2 per batch of
    # iterations between checks to recompute it), 4 with the residual from A
    check = 10.0
    refine_passes = (2.0 + 2.0 / check if P.get_tuning("refine_passes") == 2 else 4.0) + 2.0 / check  # + the KKT pair
    rooflines = {
        "integrate_and_bin": {"kernel": "k_integrate + k_hist", "bound": "alu", "unit": "TFLOP/s",
                              "peak": (PEAK_F64_VALU if f64 else PEAK_F32_VALU) / 1e12,
                              "work": FLOP_PER_ORBIT_STEP[cfg["name"]] * N * n_steps, "ms": t_i,
                              "work_rule": "flop per orbit-step counted from the formulas x orbit-steps"},
        "gram": {"kernel": (f"k_gram_bf16 ({args.gram}{' of the counts' if counts else ''})" if args.gram != "f32"
                            else "k_gemm_nt_f32 (Gram)"),
                 "bound": "mfma", "unit": "TFLOP/s",
                 "peak": (PEAK_BF16 if args.gram != "f32" else PEAK_F32_MFMA) / 1e12,
                 "work": C * (C + 1) * N, "ms": t_gram, "work_rule": "SYRK C(C+1)N"},
        "factorise": {"kernel": "k_potrf_diag + k_gemm_nt_x3 (split-bf16 Cholesky, inverse factor)", "bound": "mfma",
                      "unit": "TFLOP/s", "peak": PEAK_F32_MFMA / 1e12, "work": C ** 3 / 3.0,
                      "issued": 2.0 * C ** 3 / 3.0, "ms": t_factor, "work_rule": "Cholesky C^3/3"},
        "admm_fp32": {"kernel": "k_csc_colsum + k_rowdot_csr + k_trmv16", "bound": "hbm", "unit": "GB/s",
                      "peak": PEAK_HBM / 1e9, "work": it1 * per_iter, "issued": it1 * per_iter, "ms": t_admm,
                      "work_rule": "2|U| + 2|L| per iteration"},
        "refine_fp64": {"kernel": "k_csc_colsum + k_rowdot_csr + k_trmv16 (+ k_aa_*)", "bound": "hbm", "unit": "GB/s",
                        "peak": PEAK_HBM / 1e9, "work": it2 * per_iter,
                        "issued": it2 * (refine_passes * u_bytes + 2 * l_bytes + aa_bytes), "ms": t_ref,
                        "work_rule": "2|U| + 2|L| per iteration"},
    }
    if it1 == 0:
        del rooflines["admm_fp32"], stages["admm_fp32"]  # the FP32 stage did not run (accelerated FP64 stage only)
    if n_boot > 0:
        # the bootstrap solves' FP64 stage: per iteration each data vector needs 2|U| + 2|L| of
        # algorithmic traffic; issued: each group of rg vectors streams the compressed copies four
        # times, the two triangles are read once for all vectors, and each vector's Anderson mixing
        # moves 91 N doubles
        repb = boot[-1][1]
        rg = P.get_tuning("rhs_per_group") or 4
        rg = 1 << max(0, math.ceil(math.log2(min(rg, n_boot))))
        its_sum = float(sum(r.refine_iters for r in repb))
        its_max = float(max(r.refine_iters for r in repb))
        t_boot_ref = float(repb[0].t_refine_ms)
        stages["bootstrap_refine_fp64"] = t_boot_ref
        stages["bootstrap_rest"] = float(np.mean([b[4] for b in boot])) - t_boot_ref
        # the shared matrix's passes: compressed per group of rg vectors, or (reported nnz 0)
        # dense FP64 MFMA products that read A once per pass for all vectors; the multi-vector
        # inverse products read the fp32 factor
        l32 = 4.0 * C * (C + 1) / 2.0
        if repb[0].nnz > 0:
            kern, a_issued = "k_csc_colsum_rhs + k_rowdot_csr_rhs + k_trmm_rhs (+ k_aa_*)", its_sum / rg * 4 * u_bytes
        else:
            kern = "k_dgemm_rhs + k_trmm_rhs (+ k_aa_*)"
            a_issued = its_max * refine_passes * N * C * (8.0 if f64 else 4.0)
        rooflines["bootstrap_refine_fp64"] = {
            "kernel": kern, "bound": "hbm", "unit": "GB/s",
            "peak": PEAK_HBM / 1e9, "ms": t_boot_ref, "work": its_max * (2 * u_bytes + 2 * l32),
            "issued": a_issued + its_max * 2 * l32 + its_sum * aa_bytes,
            "work_rule": "2|U| + 2|L| per iteration of the batch (A and the factor read once for all "
                         "data vectors)"}
    for k, r in rooflines.items():
        scale = 1e12 if r["unit"] == "TFLOP/s" else 1e9
        r["achieved"] = round(r["work"] / (r["ms"] * 1e-3) / scale, 3) if r["ms"] > 0 else None
        r["frac"] = round(r["achieved"] / r["peak"], 4) if r["achieved"] is not None else None
        if "issued" in r and r["ms"] > 0:
            r["issued_rate"] = round(r["issued"] / (r["ms"] * 1e-3) / scale, 3)
            r["issued"] = float(r["issued"])
        r["traffic"] = TRAFFIC.get((cfg["name"], k))
        if (cfg["name"], k) in TRAFFIC_PER_ITER:
            r["traffic"] = TRAFFIC_PER_ITER[(cfg["name"], k)] * (it1 if k == "admm_fp32" else it2)
        r["work"] = float(r["work"])
    dominant = max(stages, key=stages.get)
    roof = dict(rooflines[dominant], stage=dominant)

    out = {
        "metric": METRIC, "value": value, "unit": "orbit-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if not f64 else "f64", "data": "synthetic",
        "config": {"workload": cfg["name"] + (f"+{n_boot}_bootstraps" if n_boot else ""), "n_orbits": n,
                   "n_steps": n_steps, "n_constraints": nc,
                   "gram": args.gram, "mock": cfg["mock"]},
        "model_builds_per_s": 1e3 / ms,
        "stage_ms": {k: round(v, 3) for k, v in stages.items()},
        "dominant_stage": dominant,
        "solve": {k: reps[-1][k] for k in ("iters", "refine_iters", "converged", "kkt", "mu", "rho", "status")},
        "precision": {"integrate": "fp32 (Jacobi drift in fp64)", "gram": args.gram + " MFMA, fp32 accumulate",
                      "factorise": "fp32", "iterations": f"{int(it1)} fp32 ADMM + {int(it2)} fp64 "
                      "(the accelerated solve runs its ADMM iterations in fp64 from the start)",
                      "chi2": "fp64"},
        "chi2": chis[-1],
        "integrate_orbit_steps_per_s": orbit_steps / (t_i * 1e-3),
        "bootstrap": None if n_boot == 0 else {
            "n": n_boot, "ms": float(np.mean([b[4] for b in boot])), "status": boot[-1][0],
            "solves_per_s": n_boot / (1e-3 * float(np.mean([b[4] for b in boot]))),
            "refine_iters_max": int(max(r.refine_iters for r in boot[-1][1])),
            "refine_iters_median": float(np.median([r.refine_iters for r in boot[-1][1]])),
            "kkt_max": float(max(r.kkt for r in boot[-1][1])),
            "chi2_b_range": [float(min(boot[-1][2])), float(max(boot[-1][2]))], "chi2_model": boot[-1][3]},
        "roofline": roof,
        "rooflines": rooflines,
    }
    if not args.no_cpu_baseline and "subsample" in cfg:
        run = dict(P=P, torch=torch, dev=dev, ics=ics, dt=dt, obs=obs, pot=pot, opts=opts, stream=stream, A=A, w=w,
                   fl=fl, d=d, sig=sig, w_tilde=w_tilde, mu=reps[-1]["mu"], kkt=reps[-1]["kkt"], chi2=chis[-1])
        out["cpu_baseline"], out["errors_vs_oracle"] = cpu_baseline_leg(cfg, run)
    if args.calibration_copy:
        src = torch.ones(1 << 30, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(json.dumps(out))


def shared_mock(P, torch, comps, omega, euler, ics, dt, n_steps, obs_d, mock, dev):
    """Mock data from one build at fixed parameters: binned sum of a seeded 10%
    orbit subset with Exp(1) weights, optional Gaussian noise."""
    n = ics.shape[1]
    pot = P.build_potential(comps, omega, euler)
    obs = P.obs_spec(obs_d)
    nc = P.ncon(obs)
    A = torch.empty((n, nc), dtype=torch.float32, device=dev)
    ov = torch.empty((n, 2), dtype=torch.float64, device=dev)
    dr = torch.empty(n, dtype=torch.float64, device=dev)
    fl = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = torch.empty(P.integrate_workspace_bytes(obs, 1, n, n_steps, P.SW_F32), dtype=torch.uint8, device=dev)
    P.integrate_and_bin(pot, [0, n], torch.from_numpy(ics.astype(np.float32)).to(dev),
                        torch.from_numpy(dt.astype(np.float32)).to(dev), n_steps, obs, A, ov, dr, fl, ws)
    w = torch.from_numpy(W.mock_draw(n, mock["seed"])).to(dev)
    d = torch.empty(nc, dtype=torch.float64, device=dev)
    P.model_observables(A, w, d)
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    if mock["noise"] > 0:
        d = d * (1 + mock["noise"] * W.noise_draw(nc, mock["seed"]))
    del A, ws
    return d


def bench_walkers(args):
    """64 MCMC walkers' trial potentials (barred family, +-30% around the nominal
    12 parameters), orbit counts uniform in 20k..150k, small-model observables,
    1,000 FP32 steps over 50 circular periods; one batched integrate_and_bin
    launch, one batched weight solve, chi^2 per walker.  A step = the 64 builds."""
    import torch
    import paper_2607_00117_amd as P
    from paper_2607_00117_amd import autotune
    dev = torch.device("cuda:0")
    n_w, n_steps = 64, 1000
    thetas = W.walker_thetas(n_w, seed=5)
    counts = W.walker_orbit_counts(n_w, seed=5)
    table = W.load_table(W.BARRED["table"])
    ics, dt = W.disc_ics(table, int(counts.max()), seed=3, n_steps=n_steps)
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n_tot = int(offs[-1])
    idx = np.concatenate([np.arange(c) for c in counts])
    obs_d = dict(W.SMALL["obs"])
    obs = P.obs_spec(obs_d)
    nc = P.ncon(obs)
    blocks = W.blocks(obs_d)
    comps, omega, euler = W.theta_to_model(W.theta_nominal())
    n_mock = int(np.mean(counts))
    d = shared_mock(P, torch, comps, omega, euler, ics[:, :n_mock], dt[:n_mock], n_steps, obs_d, W.BARRED["mock"], dev)
    sig = mock_sigma(d, blocks, W.BARRED["mock"]["tol"])
    mass = float(np.sum(d[blocks[0][0]:blocks[0][1]]))
    w_tilde = [mass / float(c) for c in counts]
    pots = [P.build_potential(*W.theta_to_model(th)) for th in thetas]
    ic_t = torch.from_numpy(ics[:, idx].astype(np.float32)).to(dev)
    dt_t = torch.from_numpy(dt[idx].astype(np.float32)).to(dev)
    A = torch.empty((n_tot, nc), dtype=torch.float32, device=dev)
    ov = torch.empty((n_tot, 2), dtype=torch.float64, device=dev)
    dr = torch.empty(n_tot, dtype=torch.float64, device=dev)
    fl = torch.empty(n_tot, dtype=torch.uint8, device=dev)
    iws = torch.empty(min(P.integrate_workspace_bytes(obs, n_w, n_tot, n_steps, P.SW_F32), 24 << 30),
                      dtype=torch.uint8, device=dev)
    log(f"walkers: {n_w} potentials, {n_tot} orbits x {n_steps} steps, {nc} constraints")
    # autotune the integration launch on a sample of the batch
    s_off = offs[:9] if offs[8] < 400000 else offs[:2]
    s_n = int(s_off[-1])
    s_ws = torch.empty(P.integrate_workspace_bytes(obs, len(s_off) - 1, s_n, 200, P.SW_F32), dtype=torch.uint8,
                       device=dev)

    def sample():
        P.integrate_and_bin(pots[:len(s_off) - 1], s_off, ic_t[:, :s_n], dt_t[:s_n], 200, obs, A[:s_n], ov[:s_n],
                            dr[:s_n], fl[:s_n], s_ws)
        torch.cuda.synchronize()
    best, table_t = autotune.tune(sample, autotune.shape_key(obs, len(s_off) - 1, s_n, 200, "f32"), log=log)
    del s_ws
    log(f"autotune best {best}")
    d_t = torch.from_numpy(np.tile(d, (n_w, 1))).to(dev)
    s_t = torch.from_numpy(np.tile(sig, (n_w, 1))).to(dev)
    d1, s1 = torch.from_numpy(d).to(dev), torch.from_numpy(sig).to(dev)
    opts = P._lib.SolveOpts()
    opts.gram, opts.nu, opts.use_graph = P.SW_GRAM_BF16X3, 1e-2, 1
    opts.mask = fl.data_ptr()
    if not args.no_quantum:
        opts.quantum = P.count_quantum(obs, n_steps)
    opts.refine_iter = 5000  # the hardest walkers need up to ~2,500 accelerated iterations
    if args.rho is not None:
        opts.rho = -args.rho
    if args.no_accel:
        opts.flags |= P.SW_SOLVE_NO_ACCEL
    w = torch.empty(n_tot, dtype=torch.float64, device=dev)
    sws = torch.empty(P.solve_batched_workspace_bytes(offs, nc, opts), dtype=torch.uint8, device=dev)
    cws = torch.empty(P.chi2_workspace_bytes(nc), dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream()
    chis, t_int, t_solve, n_conv = [], [], [], []

    def step():
        with torch.cuda.stream(stream):
            t0 = time.perf_counter()
            P.integrate_and_bin(pots, offs, ic_t, dt_t, n_steps, obs, A, ov, dr, fl, iws)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, reps = P.solve_weights_batched(A, offs, d_t, s_t, w_tilde, -1.0, opts, w, sws)
            x = [P.chi2(A[offs[k]:offs[k + 1]], w[offs[k]:offs[k + 1]], d1, s1, blocks[1][0], blocks[1][1], cws)
                 for k in range(n_w)]
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        t_int.append(1e3 * (t1 - t0)); t_solve.append(1e3 * (t2 - t1)); chis.append(x)
        n_conv.append(sum(int(r.converged) for r in reps))
        return reps

    for _ in range(args.warmup):
        step()
    t_int.clear(); t_solve.clear(); chis.clear(); n_conv.clear()
    t0 = time.perf_counter()
    for i in range(args.steps):
        reps = step()
        its = np.array([r.iters for r in reps]); rits = np.array([r.refine_iters for r in reps])
        kkts = np.array([r.kkt for r in reps])
        log(f"step {i}: integrate {t_int[-1]:.1f} ms, solve+chi2 {t_solve[-1]:.1f} ms, "
            f"iters max {its.max()}+{rits.max()} median {int(np.median(its))}+{int(np.median(rits))}, "
            f"converged {sum(r.converged for r in reps)}/{len(reps)}, kkt max {kkts.max():.2e}, nnz {reps[0].nnz:.3g}, "
            f"fp64 passes per iteration {reps[0].passes}")
        slow = np.argsort(-(its + 2 * rits))[:4]
        log("slowest walkers: " + "; ".join(f"#{k} n={offs[k + 1] - offs[k]} it={its[k]}+{rits[k]} kkt={kkts[k]:.1e} "
                                            f"chi2={chis[-1][k]:.4g}" for k in slow))
    el = time.perf_counter() - t0
    out = {"metric": METRIC, "value": n_w * args.steps / el, "unit": "model builds/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "walkers_64_barred_family_20k-150k_orbits_1k_steps", "n_orbits_total": n_tot,
                      "n_constraints": nc, "autotune": best},
           "orbit_steps_per_s": n_tot * n_steps * args.steps / el,
           "integrate_ms": float(np.mean(t_int)), "solve_chi2_ms": float(np.mean(t_solve)),
           "chi2_range": [float(np.min(chis[-1])), float(np.max(chis[-1]))],
           "converged": f"{min(n_conv)}/{n_w}", "fp64_passes_per_iteration": int(reps[0].passes),
           "converged_builds_per_s": min(n_conv) * args.steps / el}
    print(json.dumps(out))


# FP64 flop per force evaluation of the barred potential (32-point Gauss-Legendre
# Ferrers bar: 3 warm Newton steps x 21, setup 14, 32 nodes x 28, scaling 12;
# MN 22; NFW_q 27) and per attempted BS23 step (three force evaluations with
# FSAL, the stage combinations and the error norm, 6 x 27 + 30)
FLOP_PER_FORCE_F64 = 63 + 14 + 32 * 28 + 12 + 22 + 27
FLOP_PER_BS23_STEP = 3 * FLOP_PER_FORCE_F64 + 6 * 27 + 30
# the single-precision force: the 16-node rule (Ferrers 537 as counted for the
# leapfrog integrator, MN 22, NFW_q 27)
FLOP_PER_FORCE_F32 = 537 + 22 + 27
FLOP_PER_BS23_STEP_F32 = 3 * FLOP_PER_FORCE_F32 + 6 * 27 + 30


def paper_maps(raw, cfg, n_ap, kin0, surf0):
    """The observed luminosity gamma* (Sigma*, floored at 1e-3 of its maximum) and the
    reference Gaussian (v0, s) of each aperture: the mean and dispersion of the
    binned LOSVD (at least 20 km/s), from the binned maps `raw` of a mock."""
    o = cfg["obs"]
    nv, vlo, vhi = o["nv"], o["vlo"], o["vhi"]
    sig_obs = raw[surf0:surf0 + n_ap]
    gamma = np.maximum(sig_obs, 1e-3 * sig_obs.max())
    hist = raw[kin0:kin0 + n_ap * nv].reshape(n_ap, nv)
    vc = vlo + (np.arange(nv) + 0.5) * (vhi - vlo) / nv
    tot = np.maximum(hist.sum(1), 1e-300)
    v0 = (hist * vc).sum(1) / tot
    s = np.sqrt(np.maximum((hist * (vc - v0[:, None]) ** 2).sum(1) / tot, 20.0 ** 2))
    return gamma, v0, s


def paper_data(model, cfg, n_mass, n_ap, m_star=None):
    """The observed data vector and its uncertainties from the fit-matrix
    observables `model` of a mock: the density block (m*_n when given), Sigma*
    with 1% noise and h* with noise of Delta h*, seeded; sigma 1% of the density
    and Sigma (floored at 1e-3 of their maxima), Delta h* on the h-blocks."""
    d = np.array(model, dtype=np.float64)
    rng = np.random.default_rng(cfg["mock"]["seed"] + 4000)
    if m_star is not None:
        d[:n_mass] = m_star
    d[n_mass:n_mass + n_ap] *= 1 + cfg["mock"]["noise"] * rng.standard_normal(n_ap)
    d[n_mass + n_ap:] += cfg["dh"] * rng.standard_normal(d.size - n_mass - n_ap)
    sig = np.empty(d.size)
    for b0, b1 in ((0, n_mass), (n_mass, n_mass + n_ap)):
        top = float(np.max(np.abs(d[b0:b1])))
        sig[b0:b1] = cfg["mock"]["tol"] * np.maximum(np.abs(d[b0:b1]), 1e-3 * top)
    sig[n_mass + n_ap:] = cfg["dh"]
    return d, sig


def paper_mock(P, torch, dev, cfg, pot, obs, pix2ap, n_ap, A_b, m_star, n_mass, kin0, surf0):
    """The observed maps (a stand-in for the paper's IFU data): a seeded 10% subset of
    the bundles with Exp(1) weights scaled to the stellar mass of the density grid;
    Sigma* its surface block (+1% noise), the reference Gaussian of each aperture its
    LOSVD's mean and dispersion (at least 20 km/s), h* its h_m for the observed
    luminosity gamma* = Sigma* (+ noise of Delta h*); the density data are m*_n."""
    o = cfg["obs"]
    nb = A_b.shape[0]
    w = torch.from_numpy(W.mock_draw(nb, cfg["mock"]["seed"])).to(dev)
    full = torch.empty(A_b.shape[1], dtype=torch.float64, device=dev)
    P.model_observables(A_b, w, full)
    torch.cuda.synchronize()
    raw = full.cpu().numpy()
    ms = m_star.cpu().numpy()
    scale = float(ms.sum()) / float(raw[:n_mass].sum())
    raw = raw * scale
    nv, vlo, vhi = o["nv"], o["vlo"], o["vhi"]
    gamma, v0, s = paper_maps(raw, cfg, n_ap, kin0, surf0)
    n_gh = cfg["n_gh"]
    nf = n_mass + n_ap + n_gh * n_ap
    F = torch.empty((nb, nf), dtype=torch.float64, device=dev)
    gws = torch.empty(P.gh_fit_workspace_bytes(n_ap, nv, n_gh), dtype=torch.uint8, device=dev)
    P.gh_fit_matrix(A_b, n_mass, kin0, surf0, n_ap, nv, vlo, vhi, v0, s, gamma, F, gws, n_gh=n_gh)
    model = torch.empty(nf, dtype=torch.float64, device=dev)
    P.model_observables(F, w * scale, model)
    torch.cuda.synchronize()
    d, sig = paper_data(model.cpu().numpy(), cfg, n_mass, n_ap, m_star=ms)
    return d, sig, v0, s, gamma, float(ms.sum()) / nb


def paper_oracle_leg(cfg, run, n_bundles=16):
    """The oracle leg of the paper pipeline: the FP64 oracle's whole model
    (Jeans initial conditions, dithers, BS23 with time-weighted binning, bundle
    means, the Gauss-Hermite fit matrix, the exact NNLS of the observed maps and
    chi^2) for the first n_bundles of the seeded initial conditions, timed on the
    host; and the GPU's errors against the oracle on that sample: the Jeans
    moments, the BS23 rows (from the oracle's initial conditions), the fit
    matrix (from the oracle's bundle rows) and the weight solve on the oracle's
    fit matrix."""
    import oracle as O
    from oracle import gh as GH
    from oracle import ics as OI
    from oracle import nnls as N
    P, torch, dev = run["P"], run["torch"], run["dev"]
    threads, phys = host_threads()
    o = cfg["obs"]
    nd, S = cfg["n_dither"], run["S"]
    pos, eps, u = run["pos"][:, :n_bundles], run["eps"][:, :n_bundles], run["u"][:, :, :n_bundles]
    comps, omega, euler = W.BARRED["components"], W.BARRED["omega"], W.BARRED["euler"]
    pot = O.make_pot(comps, omega)
    ob = O.make_obs(dict(o, pix2ap=run["pmap"], n_ap=run["n_ap"]), O.euler_matrix(*euler))
    n_mass, kin0, surf0, n_ap, n_gh = run["n_mass"], run["kin0"], run["surf0"], run["n_ap"], cfg["n_gh"]
    O.set_ferrers_rule(64)
    try:
        t0 = time.perf_counter()
        mom_o, ic_o = O.jeans_ics(pot, pos, eps, cfg["h_R"], cfg["h_z"], cfg["jeans_b"])
        ics_o = OI.dither(ic_o, mom_o[4], u, cfg["dx"], cfg["fv"])
        h0 = np.full(ics_o.shape[1], cfg["h0"])
        A_o, _, dr_o, _ = O.integrate_bs23_and_bin(pot, ob, ics_o, h0, S, cfg["rtol"], cfg["atol"], nthreads=threads)
        Ab_o = OI.bundle_rows(A_o, nd)
        # the sample's own mock (the same recipe: a 10% subset with Exp(1) weights)
        w_s = W.mock_draw(n_bundles, cfg["mock"]["seed"])
        gamma, v0, sw = paper_maps(Ab_o.T @ w_s, cfg, n_ap, kin0, surf0)
        F_o = GH.fit_matrix(Ab_o, n_mass, kin0, surf0, n_ap, o["nv"], o["vlo"], o["vhi"], v0, sw, gamma, n_gh)
        d, sig = paper_data(F_o.T @ w_s, cfg, n_mass, n_ap)
        wt = float(d[:n_mass].sum()) / n_bundles
        U, y = N.scale_problem(F_o, d, sig, wt)
        mu = N.relative_mu(U, 1e-2)
        w_o = N.nnls_oracle(U, y, mu) * wt
        x_o = N.chi2(F_o, w_o, d, sig, n_mass, F_o.shape[1])
        el = time.perf_counter() - t0
    finally:
        O.set_ferrers_rule(0)
    errors = {}
    # Jeans moments on the same positions
    mom = torch.empty((5, n_bundles), dtype=torch.float64, device=dev)
    ic1 = torch.empty((6, n_bundles), dtype=torch.float64, device=dev)
    P.jeans_ics(run["pot"], torch.from_numpy(np.ascontiguousarray(pos)).to(dev),
                torch.from_numpy(np.ascontiguousarray(eps)).to(dev), cfg["h_R"], cfg["h_z"], cfg["jeans_b"], mom, ic1)
    torch.cuda.synchronize()
    # each moment's largest error relative to its largest magnitude (a moment can vanish at
    # a position, e.g. the mean rotation on the minor axis)
    mg = mom.cpu().numpy()
    scale = np.maximum(np.abs(mom_o).max(axis=1, keepdims=True), 1e-300)
    errors["jeans_moments_max_rel"] = float(np.max(np.abs(mg - mom_o) / scale))
    # BS23 from the oracle's initial conditions
    n = ics_o.shape[1]
    A = torch.empty((n, A_o.shape[1]), dtype=torch.float64, device=dev)
    ov = torch.empty((n, 2), dtype=torch.float64, device=dev)
    dr = torch.empty(n, dtype=torch.float64, device=dev)
    fl = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = torch.empty(P.integrate_bs23_workspace_bytes(n, S), dtype=torch.uint8, device=dev)
    P.integrate_bs23_and_bin(run["pot"], torch.from_numpy(ics_o).to(dev), torch.from_numpy(h0).to(dev), S,
                             cfg["rtol"], cfg["atol"], run["obs"], A, ov, dr, fl, ws, precision=run["prec"])
    torch.cuda.synchronize()
    Ag = A.cpu().numpy()
    l1 = np.abs(Ag - A_o).sum(1) / 2
    drg = dr.cpu().numpy()
    errors["bs23_rows"] = {"orbits": n, "precision": "f32" if run["prec"] == P.SW_F32 else "f64",
                           "row_l1_median": float(np.median(l1)), "row_l1_p90": float(np.percentile(l1, 90)),
                           "rows_above_1e-6": float(np.mean(l1 > 1e-6)),
                           "summed_maps_l1": float(np.abs(Ag.sum(0) - A_o.sum(0)).sum() / np.abs(A_o.sum(0)).sum()),
                           "drift_median": float(np.median(drg)), "drift_median_oracle": float(np.median(dr_o))}
    # the fit matrix from the oracle's bundle rows
    Ab = torch.from_numpy(Ab_o).to(dev)
    F = torch.empty(F_o.shape, dtype=torch.float64, device=dev)
    gws = torch.empty(P.gh_fit_workspace_bytes(n_ap, o["nv"], n_gh), dtype=torch.uint8, device=dev)
    P.gh_fit_matrix(Ab, n_mass, kin0, surf0, n_ap, o["nv"], o["vlo"], o["vhi"], v0, sw, gamma, F, gws, n_gh=n_gh)
    torch.cuda.synchronize()
    Fg = F.cpu().numpy()
    errors["fit_matrix_max_abs"] = float(np.max(np.abs(Fg - F_o)))
    # the weight solve on the oracle's fit matrix
    opts = P._lib.SolveOpts()
    opts.gram, opts.nu = P.SW_GRAM_BF16X3, 1e-2
    Ft = torch.from_numpy(F_o).to(dev)
    w = torch.empty(n_bundles, dtype=torch.float64, device=dev)
    sws = torch.empty(P.solve_workspace_bytes(n_bundles, F_o.shape[1], opts), dtype=torch.uint8, device=dev)
    d_t, s_t = torch.from_numpy(d).to(dev), torch.from_numpy(sig).to(dev)
    st, rep = P.solve_weights(Ft, d_t, s_t, wt, -1.0, opts, w, sws)
    cws = torch.empty(P.chi2_workspace_bytes(F_o.shape[1]), dtype=torch.uint8, device=dev)
    x_g = P.chi2(Ft, w, d_t, s_t, n_mass, F_o.shape[1], cws)
    wg = w.cpu().numpy()
    errors["solve_sample"] = {"bundles": n_bundles, "status": st, "kkt_gpu": rep.kkt,
                              "weights_l1_rel": float(np.abs(wg - w_o).sum() / max(np.abs(w_o).sum(), 1e-300)),
                              "chi2_rel": float(abs(x_g / x_o - 1))}
    base = {"value": n * S / el, "unit": "orbit-steps/s", "cores": threads, "physical_cores": phys, "kind": "oracle",
            "sample": f"the FP64 oracle's model (Jeans initial conditions, {nd} dithers, BS23 at rtol {cfg['rtol']} "
                      f"for {S} steps with time-weighted binning, bundle means, the Gauss-Hermite fit matrix, one "
                      f"exact NNLS of the observed maps, chi^2) for the first {n_bundles} of the {cfg['n_ic']} "
                      f"seeded initial conditions ({el:.1f} s on {threads} threads; no bootstrap solves)"}
    return base, errors


def bench_paper(args):
    """The paper's pipeline for one trial potential of the barred model, every
    step in the library's kernels: Jeans initial velocities at 7,500 seeded
    positions, 4 dithered realisations each (Sec. 2.2.1), BS23 orbits in FP64
    at rtol 1e-4 for 5,000 accepted steps with time-weighted binning into a
    600-cell cylindrical grid, ~600 irregular apertures x 30 velocity bins and
    the surface block (Sec. 2.2.2-2.2.4), bundle means, the target cell masses,
    the Gauss-Hermite fit matrix (Eq. 2-3), 100 bootstrap realisations of the
    maps solved on the shared matrix, chi^2_b and chi^2_model (Eq. 5-6).
    A step = one model."""
    import torch
    import paper_2607_00117_amd as P
    cfg = W.PAPER
    o = cfg["obs"]
    dev = torch.device("cuda:0")
    n_ic, nd, S = cfg["n_ic"], cfg["n_dither"], args.bs23_steps or cfg["n_steps"]
    n = n_ic * nd
    comps, omega, euler = W.BARRED["components"], W.BARRED["omega"], W.BARRED["euler"]
    pot = P.build_potential(comps, omega, euler)
    pmap, n_ap = W.voronoi_map(o["npx"], o["npy"], o["plo"], o["phi"], cfg["n_gen"], cfg["ap_seed"], cfg["ap_scale"])
    pix_t = torch.from_numpy(pmap).to(dev)
    obs = P.obs_spec(dict(o, n_ap=n_ap), pix_t)
    nc = P.ncon(obs)
    n_mass = o["nx"] * o["ny"] * o["nz"]
    kin0, surf0 = n_mass, n_mass + n_ap * o["nv"]
    n_gh = cfg["n_gh"]
    nf = n_mass + n_ap + n_gh * n_ap
    pos, eps = W.disc_positions(n_ic, seed=cfg["ic_seed"], h_R=cfg["h_R"], h_z=cfg["h_z"])
    pos_t, eps_t = torch.from_numpy(pos).to(dev), torch.from_numpy(eps).to(dev)
    u_t = torch.from_numpy(W.dither_deviates(nd, n_ic, seed=cfg["ic_seed"])).to(dev)
    mom = torch.empty((5, n_ic), dtype=torch.float64, device=dev)
    ic1 = torch.empty((6, n_ic), dtype=torch.float64, device=dev)
    ics = torch.empty((6, n), dtype=torch.float64, device=dev)
    h0 = torch.full((n,), cfg["h0"], dtype=torch.float64, device=dev)
    A = torch.empty((n, nc), dtype=torch.float64, device=dev)
    ov = torch.empty((n, 2), dtype=torch.float64, device=dev)
    dr = torch.empty(n, dtype=torch.float64, device=dev)
    fl = torch.empty(n, dtype=torch.uint8, device=dev)
    bws = torch.empty(P.integrate_bs23_workspace_bytes(n, S), dtype=torch.uint8, device=dev)
    A_b = torch.empty((n_ic, nc), dtype=torch.float64, device=dev)
    m_star = torch.empty(n_mass, dtype=torch.float64, device=dev)
    F = torch.empty((n_ic, nf), dtype=torch.float64, device=dev)
    gws = torch.empty(P.gh_fit_workspace_bytes(n_ap, o["nv"], n_gh), dtype=torch.uint8, device=dev)
    log(f"paper pipeline: {n_ic} x {nd} orbits, BS23 rtol {cfg['rtol']} x {S} steps, {nc} binned constraints, "
        f"{n_ap} apertures, fit matrix {n_ic} x {nf}, {cfg['n_boot']} bootstraps")
    stream = torch.cuda.Stream()
    B = cfg["n_boot"]
    opts = P._lib.SolveOpts()
    opts.gram, opts.nu, opts.use_graph = P.SW_GRAM_BF16X3, 1e-2, 1
    opts.rho = -(args.rho if args.rho is not None else cfg["rho"])
    prec = P.SW_F32 if args.bs23_precision == "f32" else P.SW_F64

    def build():
        """The orbit library's part of a model: returns the stage events."""
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        ev[0].record()
        P.jeans_ics(pot, pos_t, eps_t, cfg["h_R"], cfg["h_z"], cfg["jeans_b"], mom, ic1)
        P.dither_ics(ic1, mom[4].contiguous(), u_t, cfg["dx"], cfg["fv"], ics)
        ev[1].record()
        P.integrate_bs23_and_bin(pot, ics, h0, S, cfg["rtol"], cfg["atol"], obs, A, ov, dr, fl, bws,
                                 precision=prec)
        ev[2].record()
        P.bundle_rows(A, nd, A_b)
        P.cell_masses(pot, obs, cfg["stellar_mask"], cfg["n_sub"], m_star)
        ev[3].record()
        return ev

    # the observed maps, from one build at the same parameters (untimed)
    with torch.cuda.stream(stream):
        build()
    torch.cuda.synchronize()
    d, sig, v0, s, gamma, w_tilde = paper_mock(P, torch, dev, cfg, pot, obs, pix_t, n_ap, A_b, m_star, n_mass, kin0,
                                               surf0)
    d_t, s_t = torch.from_numpy(d).to(dev), torch.from_numpy(sig).to(dev)
    e_t = torch.from_numpy(W.bootstrap_eps(B, nf, seed=cfg["mock"]["seed"])).to(dev)
    D_t = torch.empty((B, nf), dtype=torch.float64, device=dev)
    Wb = torch.empty((B, n_ic), dtype=torch.float64, device=dev)
    sws = torch.empty(P.solve_multi_workspace_bytes(n_ic, nf, B, opts), dtype=torch.uint8, device=dev)
    cws = torch.empty(P.chi2_workspace_bytes(nf), dtype=torch.uint8, device=dev)
    # with --warm-bootstraps: the observed maps' own fit, whose weights start the bootstrap solves
    warm = args.warm_bootstraps
    w_obs = torch.empty(n_ic, dtype=torch.float64, device=dev)
    ows = torch.empty(P.solve_workspace_bytes(n_ic, nf, opts) if warm else 1, dtype=torch.uint8, device=dev)
    mopts = P._lib.SolveOpts()
    ctypes.memmove(ctypes.addressof(mopts), ctypes.addressof(opts), ctypes.sizeof(opts))
    if warm:
        mopts.w0, mopts.w0_shared = w_obs.data_ptr(), 1
    res = []

    def step():
        with torch.cuda.stream(stream):
            ev = build()
            P.gh_fit_matrix(A_b, n_mass, kin0, surf0, n_ap, o["nv"], o["vlo"], o["vhi"], v0, s, gamma, F, gws,
                            n_gh=n_gh)
            P.bootstrap_data(d_t, s_t, e_t, n_mass, nf, D_t)
            ev[4].record()
            it_obs = 0
            if warm:
                st_o, rep_o = P.solve_weights(F, d_t, s_t, w_tilde, -1.0, opts, w_obs, ows)
                it_obs = rep_o.refine_iters
            st, reps = P.solve_weights_multi(F, D_t, s_t, w_tilde, -1.0, mopts, Wb, sws)
            chis = [P.chi2(F, Wb[b], d_t, s_t, n_mass, nf, cws) for b in range(B)]
            xm = P.chi2_model(chis)
            ev[5].record()
        torch.cuda.synchronize()
        res.append({"ms": {"ics": ev[0].elapsed_time(ev[1]), "bs23": ev[1].elapsed_time(ev[2]),
                           "bundle_cellmass": ev[2].elapsed_time(ev[3]), "fit_matrix": ev[3].elapsed_time(ev[4]),
                           "bootstrap_solve_chi2": ev[4].elapsed_time(ev[5])},
                    "status": st, "iters_max": max(r.refine_iters for r in reps), "iters_observed_fit": it_obs,
                    "kkt_max": max(r.kkt for r in reps), "chi2_range": [min(chis), max(chis)], "chi2_model": xm,
                    "flagged_orbits": int((fl != 0).sum().item())})

    for _ in range(args.warmup):
        step()
    res.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log(f"step {i}: {res[-1]}")
    el = time.perf_counter() - t0
    ms = 1e3 * el / args.steps
    st_ms = {k: float(np.mean([r["ms"][k] for r in res])) for k in res[0]["ms"]}
    t_b = st_ms["bs23"]
    f32 = args.bs23_precision == "f32"
    per = FLOP_PER_BS23_STEP_F32 if f32 else FLOP_PER_BS23_STEP
    work = per * n * S
    roof = {"kernel": "k_bs23 + k_hist_w", "bound": "alu", "unit": "TFLOP/s",
            "peak": (PEAK_F32_VALU if f32 else PEAK_F64_VALU) / 1e12,
            "work": float(work), "ms": t_b, "achieved": round(work / (t_b * 1e-3) / 1e12, 3),
            "work_rule": f"{per} {'FP32' if f32 else 'FP64'} flop per accepted step (three force evaluations) "
                         f"x orbit-steps",
            "traffic": None, "stage": "bs23"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    out = {"metric": METRIC, "value": n * S * args.steps / el, "unit": "orbit-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": args.bs23_precision, "data": "synthetic",
           "config": {"workload": (cfg["name"] if S == cfg["n_steps"] else cfg["name"].replace("5k", f"{S}")).replace(
                          "_f64", "_" + args.bs23_precision),
                      "n_orbits": n, "n_bundles": n_ic, "n_steps": S, "rtol": cfg["rtol"], "n_apertures": n_ap,
                      "n_binned_constraints": nc, "n_fit_constraints": nf, "n_bootstraps": B,
                      "admm_penalty": f"{-opts.rho} x trace(U U^T)/N"},
           "model_builds_per_s": 1e3 / ms, "stage_ms": {k: round(v, 2) for k, v in st_ms.items()},
           "dominant_stage": max(st_ms, key=st_ms.get), "last": res[-1], "roofline": roof,
           "context": "the paper quotes about 1.3 s per model (build + 100 bootstrap solves + chi^2) on one A100"}
    if not args.no_cpu_baseline:
        run = dict(P=P, torch=torch, dev=dev, S=S, pos=pos, eps=eps, u=W.dither_deviates(nd, n_ic, seed=cfg["ic_seed"]),
                   pmap=pmap, n_ap=n_ap, n_mass=n_mass, kin0=kin0, surf0=surf0, pot=pot, obs=obs, prec=prec)
        out["cpu_baseline"], out["errors_vs_oracle"] = paper_oracle_leg(cfg, run)
    print(json.dumps(out))


def bench_surrogate(args):
    """Learned chi^2 surrogate: Latin-hypercube training builds (small-model
    size, 2,000 orbits x 1,000 FP32 steps, barred family, +-30% priors), MLP
    training with the library's kernels, held-out error in units of dchi2, and
    delayed-acceptance MCMC (32 walkers) against plain Metropolis."""
    import torch
    import paper_2607_00117_amd as P
    from paper_2607_00117_amd import surrogate as S
    dev = torch.device("cuda:0")
    n_orb, n_steps, batch = 2000, 1000, 256
    nominal = W.theta_nominal()
    lo, hi = 0.7 * nominal, 1.3 * nominal
    table = W.load_table(W.BARRED["table"])
    ics, dt = W.disc_ics(table, n_orb, seed=3, n_steps=n_steps)
    obs_d = dict(W.SMALL["obs"])
    blocks = W.blocks(obs_d)
    comps, omega, euler = W.theta_to_model(nominal)
    d = shared_mock(P, torch, comps, omega, euler, ics, dt, n_steps, obs_d, W.BARRED["mock"], dev)
    sig = mock_sigma(d, blocks, W.BARRED["mock"]["tol"])
    wt = float(np.sum(d[blocks[0][0]:blocks[0][1]])) / n_orb
    opts = P._lib.SolveOpts()
    opts.use_graph = 1
    builder = S.ModelBuilder(W.theta_to_model, ics, dt, n_steps, obs_d, d, sig, wt, batch, kin_block=blocks[1],
                             solve_opts=opts)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        # dchi2: spread of chi^2 at the nominal parameters over independently seeded libraries
        seeds = []
        for sd in range(8):
            ics_s, dt_s = W.disc_ics(table, n_orb, seed=100 + sd, n_steps=n_steps)
            b2 = S.ModelBuilder(W.theta_to_model, ics_s, dt_s, n_steps, obs_d, d, sig, wt, 1, kin_block=blocks[1],
                                solve_opts=opts)
            seeds.append(float(b2.chi2(nominal[None, :])[0]))
            del b2
        seed_spread = float(np.std(seeds, ddof=1))
        n_ap = obs_d["npx"] * obs_d["npy"]
        dchi2, jk = builder.jackknife_dchi2(nominal, n_ap, obs_d["nv"])
        log(f"dchi2 (aperture jackknife, {n_ap} solves) = {dchi2:.4g}; chi2 spread over 8 library seeds "
            f"{seed_spread:.4g} (values {np.round(seeds, 1).tolist()})")
        u = W.latin_hypercube(args.n_train, 12, seed=7)
        thetas = lo + (hi - lo) * u
        t0 = time.perf_counter()
        chi = builder.chi2(thetas)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        conv = builder.last_converged
        log(f"{args.n_train} training builds in {t_build:.1f} s ({args.n_train / t_build:.1f} builds/s), "
            f"{int((~conv).sum())} weight solves not converged (left out of the training set)")
        thetas, chi = thetas[conv], chi[conv]
        n_tr = int(0.9 * len(thetas))
        sur = S.Surrogate(lo, hi)
        t0 = time.perf_counter()
        sur.fit(thetas[:n_tr], chi[:n_tr], epochs=200, batch=512)
        t_fit = time.perf_counter() - t0
        pred = sur.predict(thetas[n_tr:])
        err = np.abs(pred - chi[n_tr:]) / dchi2
        log(f"surrogate fit {t_fit:.1f} s; held-out |chi2_s - chi2|/dchi2 median {np.median(err):.3g}, "
            f"frac<1 {np.mean(err < 1):.3f}")
        theta0 = W.walker_thetas(32, seed=8, spread=0.05)
        adapt = args.mcmc_steps // 2

        def refit(th_b, chi_b):
            # the chains' neighbourhood only: the full builds of the chains so far, with the target
            # standardised over them, so that the network resolves chi^2 differences of a few dchi2
            # there instead of the range of the whole prior box
            sur.fit(th_b, chi_b, epochs=args.refit_epochs, batch=256, seed=len(chi_b))

        res_da = S.da_mcmc(builder, sur, theta0, lo, hi, args.mcmc_steps, dchi2, use_surrogate=True, log=log,
                           refit=refit, refit_every=max(10, adapt // 10), adapt_steps=adapt)
        res_mh = S.da_mcmc(builder, sur, theta0, lo, hi, args.mcmc_steps, dchi2, use_surrogate=False, log=log,
                           adapt_steps=adapt)
        # the screen's error where the chains walk: full builds made after adaptation
        bt, bc = res_da["built"]
        n_late = res_da["n_full_builds_after_adapt"]
        loc_err = np.abs(sur.predict(bt[-n_late:]) - bc[-n_late:]) / dchi2 if n_late > 0 else np.zeros(1)
        # chain moments after adaptation, DA against plain Metropolis (same random numbers)
        cd, cm = res_da["chains"][adapt:].reshape(-1, 12), res_mh["chains"][adapt:].reshape(-1, 12)
        moment_diff = float(np.max(np.abs(cd.mean(0) - cm.mean(0)) / np.maximum(cm.std(0), 1e-300)))
        log(f"after adaptation: DA full builds {res_da['n_full_builds_after_adapt']} vs plain MH "
            f"{res_mh['n_full_builds_after_adapt']}; screen error near the chains median "
            f"{np.median(loc_err):.3g} dchi2; max |mean difference| / std {moment_diff:.3g}")
        # the plain single-model path: one trial potential per build, no batching, no surrogate
        single = S.ModelBuilder(W.theta_to_model, ics, dt, n_steps, obs_d, d, sig, wt, 1, kin_block=blocks[1],
                                solve_opts=opts)
        single.chi2(theta0[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_single = 16
        single.chi2(theta0[:n_single])
        torch.cuda.synchronize()
        single_per_s = n_single / (time.perf_counter() - t0)
        del single
        log(f"plain single-model path: {single_per_s:.2f} models/s; batched MH {res_mh['models_per_s']:.2f}; "
            f"DA {res_da['models_per_s']:.2f}")
    out = {"metric": METRIC, "value": res_da["models_per_s"], "unit": "surrogate-MCMC models/s", "n_gpus": 1,
           "steps": args.mcmc_steps, "warmup": 0, "ms_per_step": 1e3 * res_da["seconds"] / args.mcmc_steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "surrogate_da_mcmc_32_walkers_small_model_barred_family", "n_train": args.n_train,
                      "mcmc_steps": args.mcmc_steps},
           "dchi2": dchi2, "dchi2_rule": "aperture jackknife", "chi2_seed_spread": seed_spread,
           "train_builds_per_s": args.n_train / t_build, "train_builds_unconverged": int((~conv).sum()),
           "heldout_err_over_dchi2_median": float(np.median(err)), "heldout_frac_err_below_dchi2": float(np.mean(err < 1)),
           "plain_mh_models_per_s": res_mh["models_per_s"], "single_model_path_per_s": single_per_s,
           "speedup_vs_single_model_path": res_da["models_per_s"] / single_per_s,
           "da": {k: res_da[k] for k in ("n_full_builds", "n_stage1", "n_accepted", "seconds", "proposals",
                                          "n_full_builds_after_adapt", "n_stage1_after_adapt",
                                          "n_unconverged_builds")},
           "mh": {k: res_mh[k] for k in ("n_full_builds", "n_accepted", "seconds", "proposals",
                                          "n_full_builds_after_adapt", "n_unconverged_builds")},
           "adapt_steps": adapt,
           "full_builds_ratio_after_adapt": res_da["n_full_builds_after_adapt"] / max(1, res_mh[
               "n_full_builds_after_adapt"]),
           "local_err_over_dchi2_median": float(np.median(loc_err)),
           "chain_mean_diff_over_std_max": moment_diff}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
