"""GPU parity of the adaptive Bogacki-Shampine 3(2) path (Sec. 2.2.2) with
time-weighted binning (Sec. 2.2.4) against the oracle.  The tests at the
paper's tolerance (rtol 1e-4) state their own bars below.

Both sides take the same FP64 operations in the same order (no fused
multiply-adds); the step-size factor's cube root (pow) and the order in which
the weights are added into the histogram differ in the last bit.  The step
control amplifies such differences: the error estimate is a difference of the
two embedded solutions, of relative size ~rtol, so a last-bit change of the
state moves it, and the next step, by ~u / rtol = 1e-16 / 1e-8 = 1e-8
relative; the sample weights dt_k / t_total (each ~1e-3 for 1,000 steps) and
sample positions move accordingly.  Bar: every matrix entry and overflow
fraction within 1e-8, drift within 1e-9, flags equal on the small model
(regular orbits); on the rotating barred model (chaotic orbits) rows within
1e-6 in L1 over short runs, on the barred grid whose blocks need several
histogram windows.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_common import lib

pytestmark = pytest.mark.gpu


def gpu_bs23(cfg, obs, ics, h0, n_steps, rtol, atol, precision=2):
    import torch
    P = lib()
    dev = torch.device("cuda:0")
    pot = P.build_potential(cfg["components"], cfg["omega"], cfg["euler"])
    o = P.obs_spec(obs)
    n = ics.shape[1]
    A = torch.empty((n, P.ncon(o)), dtype=torch.float64, device=dev)
    ov = torch.empty((n, 2), dtype=torch.float64, device=dev)
    dr = torch.empty(n, dtype=torch.float64, device=dev)
    fl = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = torch.empty(P.integrate_bs23_workspace_bytes(n, n_steps), dtype=torch.uint8, device=dev)
    ic_t = torch.from_numpy(np.ascontiguousarray(ics)).to(dev)
    h_t = torch.from_numpy(np.ascontiguousarray(h0)).to(dev)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    P.integrate_bs23_and_bin(pot, ic_t, h_t, n_steps, rtol, atol, o, A, ov, dr, fl, ws, precision=precision)
    t1.record()
    torch.cuda.synchronize()
    print(f"{n} orbits x {n_steps} accepted steps: {t0.elapsed_time(t1):.1f} ms")
    return A.cpu().numpy(), ov.cpu().numpy(), dr.cpu().numpy(), fl.cpu().numpy()


def oracle_bs23(cfg, obs, ics, h0, n_steps, rtol, atol):
    pot = O.make_pot(cfg["components"], cfg["omega"])
    ob = O.make_obs(obs, O.euler_matrix(*cfg["euler"]))
    return O.integrate_bs23_and_bin(pot, ob, ics, h0, n_steps, rtol, atol)


def test_small_model_matches_oracle(gpu):
    cfg = W.SMALL
    obs = dict(cfg["obs"], surface=1, upsilon=2.0)
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=1000)
    A, ov, dr, fl = gpu_bs23(cfg, obs, ics, dt, 1000, 1e-8, 1e-10)
    A_o, ov_o, dr_o, fl_o = oracle_bs23(cfg, obs, ics, dt, 1000, 1e-8, 1e-10)
    print("max |dA|", np.abs(A - A_o).max(), "max |d overflow|", np.abs(ov - ov_o).max(), "max |d drift|",
          np.abs(dr - dr_o).max())
    assert np.array_equal(fl, fl_o) and np.all(fl == 0)
    assert np.abs(A - A_o).max() <= 1e-8 and np.abs(ov - ov_o).max() <= 1e-8
    assert np.abs(dr - dr_o).max() <= 1e-9
    assert np.allclose(A[:, :1000].sum(1) + ov[:, 0], 1.0, rtol=0, atol=1e-12)


def test_barred_model_windows(gpu):
    """Rotating Ferrers bar, 64 orbits x 300 steps on the barred model's grid
    (18,000 mass and 30,000 kinematic cells: 3 and 4 histogram windows)."""
    cfg = W.BARRED
    ics, dt = W.disc_ics(W.load_table(cfg["table"]), 64, seed=11, n_steps=2000)
    A, ov, dr, fl = gpu_bs23(cfg, cfg["obs"], ics, dt, 300, 1e-7, 1e-9)
    A_o, ov_o, dr_o, fl_o = oracle_bs23(cfg, cfg["obs"], ics, dt, 300, 1e-7, 1e-9)
    l1 = np.abs(A - A_o).sum(1)
    print("max row L1", l1.max())
    assert np.array_equal(fl, fl_o)
    assert l1.max() <= 1e-6 and np.abs(ov - ov_o).max() <= 1e-6
    assert A.shape[1] == 48000 and (A[:, 18000:] > 0).any()


def test_repeated_runs_are_identical(gpu):
    """The time-weighted histograms sum fixed-point integers, so two runs give
    the same matrix to the bit (rotating barred model, several windows)."""
    cfg = W.BARRED
    ics, dt = W.disc_ics(W.load_table(cfg["table"]), 200, seed=12, n_steps=2000)
    r1 = gpu_bs23(cfg, cfg["obs"], ics, dt, 400, 1e-4, 1e-6)
    r2 = gpu_bs23(cfg, cfg["obs"], ics, dt, 400, 1e-4, 1e-6)
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b)


def test_paper_tolerance_small_model(gpu):
    """The paper's settings (Sec. 2.2.2): rtol 1e-4 and 5,000 accepted steps per
    orbit, on the small model's 2,000 orbits (static potential).  Most orbits
    take the same steps on both sides (the step control amplifies last-bit
    state differences by only ~u / rtol = 1e-12) and agree to rounding; on a few
    an accept/reject decision sits at the threshold, flips on a last-bit
    difference, and the two sides then follow different, equally valid step
    sequences whose samples differ by the integration error of rtol 1e-4
    itself (measured: 7% of the rows above 1e-6, the median at 5e-13).  Bar:
    median row L1 <= 1e-8, at most 15% of rows above 1e-6, median drift
    difference <= 1e-9 and every drift difference within the drift scale of this
    tolerance (1e-2); flags equal; every row's blocks normalised."""
    cfg = W.SMALL
    obs = dict(cfg["obs"], surface=1, upsilon=1.0)
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=5000)
    A, ov, dr, fl = gpu_bs23(cfg, obs, ics, dt, 5000, 1e-4, 1e-6)
    A_o, ov_o, dr_o, fl_o = oracle_bs23(cfg, obs, ics, dt, 5000, 1e-4, 1e-6)
    l1 = np.abs(A - A_o).sum(1)
    ddr = np.abs(dr - dr_o)
    print(f"row L1 median {np.median(l1):.3g} p99 {np.percentile(l1, 99):.3g} max {l1.max():.3g}, rows above 1e-6: "
          f"{np.mean(l1 > 1e-6):.4f}; |d drift| median {np.median(ddr):.3g} max {ddr.max():.3g}; drift median "
          f"{np.median(dr_o):.3g}")
    assert np.array_equal(fl, fl_o)
    assert np.median(ddr) <= 1e-9 and ddr.max() <= 1e-2
    assert np.median(l1) <= 1e-8 and np.mean(l1 > 1e-6) <= 0.15
    assert np.allclose(A[:, :1000].sum(1) + ov[:, 0], 1.0, rtol=0, atol=1e-11)
    assert np.allclose(A[:, 1000:1750].sum(1) + ov[:, 1], 1.0, rtol=0, atol=1e-11)


def test_paper_tolerance_barred_model(gpu):
    """rtol 1e-4 on the rotating barred model (chaotic orbits: the paper's
    Sec. 2.4 notes that chi^2 moves with the integration tolerance), 128 orbits
    x 1,000 steps: flags equal, drift within 1e-6, most rows close and every
    row's blocks normalised."""
    cfg = W.BARRED
    ics, dt = W.disc_ics(W.load_table(cfg["table"]), 128, seed=13, n_steps=2000)
    A, ov, dr, fl = gpu_bs23(cfg, cfg["obs"], ics, dt, 1000, 1e-4, 1e-6)
    A_o, ov_o, dr_o, fl_o = oracle_bs23(cfg, cfg["obs"], ics, dt, 1000, 1e-4, 1e-6)
    l1 = np.abs(A - A_o).sum(1)
    print(f"row L1 median {np.median(l1):.3g} p90 {np.percentile(l1, 90):.3g} max {l1.max():.3g}; "
          f"max |d drift| {np.abs(dr - dr_o).max():.3g}")
    assert np.array_equal(fl, fl_o)
    assert np.median(np.abs(dr - dr_o)) <= 1e-6
    assert np.median(l1) <= 1e-3
    assert np.allclose(A[:, :18000].sum(1) + ov[:, 0], 1.0, rtol=0, atol=1e-11)


def test_single_precision_small_model(gpu):
    """The single-precision integration (state, stages and step control in FP32,
    the total time and the Jacobi drift in FP64) at the paper's settings, rtol
    1e-4 and 5,000 accepted steps, on the small model's 2,000 orbits, against the
    FP64 oracle.  FP32 rounding (6e-8 relative) sits far below the tolerance, but
    the step control turns it into different, equally valid step sequences (a
    state change of u moves the next step by ~u / rtol = 6e-4), so rows differ
    by the integration error of rtol 1e-4 itself, not by rounding.  Bar: flags
    equal, the median and the largest Jacobi drift within a factor 2 of the
    oracle's (the drift measures the tolerance's integration error, which FP32
    must not inflate), the median row L1 below 5e-2, the summed matrix (the
    model's maps for equal weights) within 1e-2 in L1, and every row's blocks
    normalised."""
    cfg = W.SMALL
    obs = dict(cfg["obs"], surface=1, upsilon=1.0)
    ics, dt = W.grid_ics(W.load_table(cfg["table"]), seed=cfg["ic_seed"], n_steps=5000)
    A, ov, dr, fl = gpu_bs23(cfg, obs, ics, dt, 5000, 1e-4, 1e-6, precision=1)
    A_o, ov_o, dr_o, fl_o = oracle_bs23(cfg, obs, ics, dt, 5000, 1e-4, 1e-6)
    l1 = np.abs(A - A_o).sum(1)
    tot = np.abs(A.sum(0) - A_o.sum(0)).sum() / np.abs(A_o.sum(0)).sum()
    print(f"row L1 median {np.median(l1):.3g} p90 {np.percentile(l1, 90):.3g} max {l1.max():.3g}; summed maps L1 "
          f"{tot:.3g}; drift median {np.median(dr):.3g} (oracle {np.median(dr_o):.3g}) max {dr.max():.3g} (oracle "
          f"{dr_o.max():.3g})")
    assert np.array_equal(fl, fl_o)
    assert 0.5 <= np.median(dr) / np.median(dr_o) <= 2.0 and dr.max() <= 2.0 * dr_o.max()
    assert np.median(l1) <= 5e-2 and tot <= 1e-2
    assert np.allclose(A[:, :1000].sum(1) + ov[:, 0], 1.0, rtol=0, atol=1e-11)
    assert np.allclose(A[:, 1000:1750].sum(1) + ov[:, 1], 1.0, rtol=0, atol=1e-11)
