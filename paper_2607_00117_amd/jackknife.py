"""Aperture jackknife of chi^2 (Sec. 2.4): the likelihood scale Delta chi^2 of Eq. 7.

The weights are solved once per aperture with that aperture's data left out,
and Delta chi^2 is the scatter of the resulting chi^2 values.  Here:
  * aperture a's data are its nv kinematic constraints and, when the orbit
    matrix carries the surface-density block, its surface-density column; the
    intrinsic density block is never left out;
  * a constraint is left out exactly by zeroing its column of the orbit matrix
    and its datum (its term of Eq. 4 is then identically zero);
  * the regularisation mu = 2 lambda / N of the full problem is held fixed
    (passed as the absolute lambda = mu N / 2), so leaving data out changes
    only the data term;
  * chi^2_a is Eq. 5 of solve a's weights over the observational constraints
    that solve a kept, Delta chi^2 = sqrt((N_ap - 1)/N_ap sum_a (chi^2_a - mean)^2).
All n_ap solves run as one solve_weights_batched call over n_ap copies of the
orbit matrix; every chi^2 is the library's chi2 over contiguous column ranges.
Host orchestration only: the arithmetic runs in the library's kernels.
"""
import math

import numpy as np

from . import _lib as P


def aperture_ranges(kin0, n_ap, nv, a, surf0=None):
    """Contiguous column ranges of the observational constraints kept when aperture a is left out."""
    r = [(kin0, kin0 + a * nv), (kin0 + (a + 1) * nv, kin0 + n_ap * nv)]
    if surf0 is not None:
        r += [(surf0, surf0 + a), (surf0 + a + 1, surf0 + n_ap)]
    return [(b, e) for b, e in r if e > b]


def jackknife_dchi2(A, d, sigma, w_tilde, mu, kin0, n_ap, nv, surf0=None, mask=None, opts=None, work=None):
    """A: device [N][C] (float32 or float64); d, sigma: device [C] double;
    mu: 2 lambda / N of the full problem (solve_weights' report.mu); mask:
    device uint8 [N] (nonzero = orbit excluded) or None; opts: SolveOpts.
    work: optional dict of reusable device buffers.
    Returns (Delta chi^2, chi^2_a [n_ap], status, reports)."""
    import torch
    n, nc = A.shape
    dev = A.device
    opts = opts or P.SolveOpts()
    work = {} if work is None else work
    Ar = work.get("A")
    if Ar is None or Ar.shape[0] < n * n_ap or Ar.shape[1] != nc or Ar.dtype != A.dtype:
        Ar = work["A"] = torch.empty((n * n_ap, nc), dtype=A.dtype, device=dev)
    Ar = Ar[:n * n_ap]
    dr = torch.empty((n_ap, nc), dtype=torch.float64, device=dev)
    for a in range(n_ap):
        blk = Ar[a * n:(a + 1) * n]
        blk.copy_(A)
        dr[a].copy_(d)
        blk[:, kin0 + a * nv:kin0 + (a + 1) * nv] = 0
        dr[a, kin0 + a * nv:kin0 + (a + 1) * nv] = 0
        if surf0 is not None:
            blk[:, surf0 + a] = 0
            dr[a, surf0 + a] = 0
    sr = sigma.reshape(1, nc).expand(n_ap, nc).contiguous()
    mk = None
    n_eff = n
    if mask is not None:
        mk = mask.repeat(n_ap).contiguous()
        n_eff = int((mask == 0).sum().item())
    n_eff = max(n_eff, 1)
    opts.mask = None if mk is None else mk.data_ptr()
    offs = [n * j for j in range(n_ap + 1)]
    ws = work.get("solve")
    need = P.solve_batched_workspace_bytes(offs, nc, opts)
    if ws is None or ws.numel() < need:
        ws = work["solve"] = torch.empty(need, dtype=torch.uint8, device=dev)
    w = torch.empty(n * n_ap, dtype=torch.float64, device=dev)
    lam = mu * n_eff / 2.0
    st, reps = P.solve_weights_batched(Ar, offs, dr, sr, [w_tilde] * n_ap, lam, opts, w, ws)
    opts.mask = None
    cws = work.get("chi2")
    if cws is None or cws.numel() < P.chi2_workspace_bytes(nc):
        cws = work["chi2"] = torch.empty(P.chi2_workspace_bytes(nc), dtype=torch.uint8, device=dev)
    chis = []
    for a in range(n_ap):
        wa = w[a * n:(a + 1) * n]
        chis.append(math.fsum(P.chi2(A, wa, d, sigma, b, e, cws) for b, e in aperture_ranges(kin0, n_ap, nv, a, surf0)))
    chis = np.array(chis)
    m = math.fsum(chis.tolist()) / n_ap
    dchi2 = math.sqrt((n_ap - 1) / n_ap * math.fsum(((chis - m) ** 2).tolist()))
    return dchi2, chis, st, reps
