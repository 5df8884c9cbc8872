"""Batched model builds, the learned chi^2 surrogate, and delayed-acceptance MCMC.

Host-side orchestration only: every model build runs integrate_and_bin over
many trial potentials in one launch, solve_weights_batched and chi2 through
the C ABI; the surrogate is trained and evaluated with the library's MLP
kernels.  The control flow of the sampler (proposals, accept/reject) lives
here on the host.

Likelihood (Sec. 2.4, Eq. 7): ln L = -chi^2 / dchi2.  dchi2 is the paper's
jackknife scale (Sec. 2.4): the weights are solved again once per aperture
with that aperture's kinematic constraints left out, and dchi2 is the
jackknife standard deviation of the resulting chi^2 values.  The spread of
chi^2 over independently seeded orbit libraries is reported beside it.

Sampler: random-walk Metropolis with delayed acceptance (Christen & Fox 2005):
a proposal must first pass the surrogate screen min(1, L~(theta')/L~(theta));
only then is the full model built and the move accepted with
min(1, L(theta') L~(theta) / (L(theta) L~(theta'))), which keeps the exact
posterior invariant while skipping full builds for proposals the screen rejects.
"""
import math
import time

import numpy as np

from . import _lib as P
from . import jackknife


class ModelBuilder:
    """Builds chi^2 for batches of trial potentials on a fixed orbit library.

    family: callable theta -> (components, omega, euler)
    ics, dt: numpy [6][n], [n] (single precision is used on the device)
    obs: observable spec dict; d, sigma: numpy [n_con] (shared mock data)
    counts: the weight solves take the leapfrog matrices as counts of
    1 / (ncopy n_steps) (solve opts.quantum; off with surface-density columns)
    """

    def __init__(self, family, ics, dt, n_steps, obs, d, sigma, w_tilde, max_batch, nu=1e-2, gram=P.SW_GRAM_BF16X3,
                 kin_block=None, drift_mask=True, solve_opts=None, counts=True):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda:0")
        self.family = family
        self.n = ics.shape[1]
        self.n_steps = n_steps
        self.obs = P.obs_spec(obs)
        self.nc = P.ncon(self.obs)
        self.max_batch = max_batch
        self.kin = kin_block
        self.w_tilde = w_tilde
        self.drift_mask = drift_mask
        n_tot = self.n * max_batch
        ic1 = torch.from_numpy(np.ascontiguousarray(ics, dtype=np.float32)).to(self.dev)
        self.ics = ic1.repeat(1, max_batch).contiguous()
        self.dt = torch.from_numpy(np.ascontiguousarray(dt, dtype=np.float32)).to(self.dev).repeat(max_batch)
        self.A = torch.empty((n_tot, self.nc), dtype=torch.float32, device=self.dev)
        self.ov = torch.empty((n_tot, 2), dtype=torch.float64, device=self.dev)
        self.dr = torch.empty(n_tot, dtype=torch.float64, device=self.dev)
        self.fl = torch.empty(n_tot, dtype=torch.uint8, device=self.dev)
        self.iws = torch.empty(P.integrate_workspace_bytes(self.obs, max_batch, n_tot, n_steps, P.SW_F32),
                               dtype=torch.uint8, device=self.dev)
        self.d = torch.from_numpy(np.tile(d, (max_batch, 1))).to(self.dev)
        self.sig = torch.from_numpy(np.tile(sigma, (max_batch, 1))).to(self.dev)
        self.d1 = torch.from_numpy(np.asarray(d, dtype=np.float64)).to(self.dev)
        self.s1 = torch.from_numpy(np.asarray(sigma, dtype=np.float64)).to(self.dev)
        self.opts = solve_opts or P.SolveOpts()
        self.opts.gram = gram
        self.opts.nu = nu
        if counts:
            self.opts.quantum = P.count_quantum(self.obs, n_steps)
        offs = [self.n * k for k in range(max_batch + 1)]
        self.sws = torch.empty(P.solve_batched_workspace_bytes(offs, self.nc, self.opts), dtype=torch.uint8,
                               device=self.dev)
        self.w = torch.empty(n_tot, dtype=torch.float64, device=self.dev)
        self.cws = torch.empty(P.chi2_workspace_bytes(self.nc), dtype=torch.uint8, device=self.dev)
        self.n_built = 0
        self.n_resolved = 0
        self.n_unconverged = 0
        self.last_converged = np.zeros(0, dtype=bool)
        self._sws1 = None
        self._jk_work = {}

    def chi2(self, thetas):
        """chi^2 of each parameter vector (rows of thetas); batches of max_batch.
        self.last_converged holds, per row, whether its weight solve met the
        KKT tolerance (a solve that reaches the batch's cap is repeated alone
        with a 4x higher cap first); self.n_unconverged counts the builds that
        never did."""
        out, conv = [], []
        for k0 in range(0, len(thetas), self.max_batch):
            r, c = self._chi2_batch(thetas[k0:k0 + self.max_batch])
            out.extend(r)
            conv.extend(c.tolist())
        self.last_converged = np.array(conv, dtype=bool)
        self.n_unconverged += int((~self.last_converged).sum())
        return np.array(out)

    def jackknife_dchi2(self, theta, n_ap, nv):
        """Sec. 2.4: one build at theta, then the aperture jackknife of its
        chi^2 (`jackknife.jackknife_dchi2`: n_ap weight solves of the same
        matrix, each without one aperture's data, the full problem's
        regularisation held fixed).  Returns (dchi2, chi^2 values)."""
        self._chi2_batch(np.asarray(theta, dtype=np.float64)[None, :])
        n = self.n
        mu = self.last_reports[0].mu
        o = self.obs
        surf0 = o.nx * o.ny * o.nz + o.n_ap * o.nv if o.surface else None
        mask = self.fl[:n] if self.drift_mask else None
        opts = type(self.opts).from_buffer_copy(self.opts)
        dchi2, chis, _, _ = jackknife.jackknife_dchi2(self.A[:n], self.d1, self.s1, self.w_tilde, mu, self.kin[0],
                                                      n_ap, nv, surf0=surf0, mask=mask, opts=opts,
                                                      work=self._jk_work)
        return dchi2, chis

    def _chi2_batch(self, thetas):
        k = len(thetas)
        pots = []
        for th in thetas:
            comps, omega, euler = self.family(th)
            pots.append(P.build_potential(comps, omega, euler))
        n_tot = self.n * k
        offs = [self.n * j for j in range(k + 1)]
        A = self.A[:n_tot]
        P.integrate_and_bin(pots, offs, self.ics[:, :n_tot], self.dt[:n_tot], self.n_steps, self.obs, A,
                            self.ov[:n_tot], self.dr[:n_tot], self.fl[:n_tot], self.iws)
        self.opts.mask = self.fl.data_ptr() if self.drift_mask else None
        st, reps = P.solve_weights_batched(A, offs, self.d[:k], self.sig[:k], [self.w_tilde] * k, -1.0, self.opts,
                                           self.w[:n_tot], self.sws)
        conv = np.array([bool(r.converged) for r in reps])
        for j in np.flatnonzero(~conv):
            # a problem that reached the batch's iteration cap is solved again on its own with a higher cap;
            # if it still does not converge it is reported as such
            conv[j], reps[j] = self._resolve(A[offs[j]:offs[j + 1]], offs[j])
        cb, ce = self.kin if self.kin else (0, self.nc)
        res = []
        for j in range(k):
            res.append(P.chi2(A[offs[j]:offs[j + 1]], self.w[offs[j]:offs[j + 1]], self.d1, self.s1, cb, ce,
                              self.cws))
        self.n_built += k
        self.last_reports = reps
        return res, conv

    def _resolve(self, A1, i0):
        n = self.n
        opts = type(self.opts).from_buffer_copy(self.opts)
        opts.refine_iter = 4 * (self.opts.refine_iter if self.opts.refine_iter > 0 else 2000)
        opts.mask = self.fl[i0:i0 + n].data_ptr() if self.drift_mask else None
        need = P.solve_workspace_bytes(n, self.nc, opts)
        if self._sws1 is None or self._sws1.numel() < need:
            self._sws1 = self.torch.empty(need, dtype=self.torch.uint8, device=self.dev)
        st, rep = P.solve_weights(A1, self.d1, self.s1, self.w_tilde, -1.0, opts, self.w[i0:i0 + n], self._sws1)
        self.n_resolved += 1
        return bool(rep.converged), rep


class Surrogate:
    """MLP emulator of chi^2(theta) on the unit box of a prior.

    Inputs are mapped to [-1, 1]^12 from the prior box (lo, hi); the target is
    the standardised log chi^2.  Training: mini-batch Adam with the library's
    fp32 forward/backward kernels; inference: fused bf16 kernel."""

    def __init__(self, lo, hi, seed=0):
        import torch
        self.torch = torch
        self.lo, self.hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
        self.n_param = P.mlp_param_count()
        rng = np.random.default_rng(seed)
        p = []
        # fan-in scaled uniform initialisation, layer by layer in the packed order
        for (o, i) in [(256, 12), (256, 0), (256, 256), (256, 0), (256, 256), (256, 0), (1, 256), (1, 0)]:
            if i:
                lim = math.sqrt(6.0 / i) * (0.5 if o == 1 else 1.0)
                p.append(rng.uniform(-lim, lim, size=o * i))
            else:
                p.append(np.zeros(o))
        self.params = torch.from_numpy(np.concatenate(p).astype(np.float32)).cuda()
        self.packed = torch.empty(self.n_param, dtype=torch.bfloat16, device="cuda")
        self.mu_t, self.sd_t = 0.0, 1.0

    def _x(self, thetas):
        x = 2.0 * (np.asarray(thetas, dtype=np.float64) - self.lo) / (self.hi - self.lo) - 1.0
        return self.torch.from_numpy(x.astype(np.float32)).cuda()

    def fit(self, thetas, chi2, epochs=200, batch=512, lr=1e-3, seed=1, keep_scaling=False):
        """Mini-batch Adam on (theta, log chi^2); keep_scaling: continue from the
        current weights with the current target standardisation (a refit)."""
        torch = self.torch
        t = np.log(np.asarray(chi2, dtype=np.float64))
        if not keep_scaling:
            self.mu_t, self.sd_t = float(t.mean()), float(t.std() + 1e-12)
        batch = min(batch, len(t))
        tt = torch.from_numpy(((t - self.mu_t) / self.sd_t).astype(np.float32)).cuda()
        x = self._x(thetas)
        n = x.shape[0]
        m = torch.zeros_like(self.params)
        v = torch.zeros_like(self.params)
        g = torch.empty_like(self.params)
        y = torch.empty(batch, device="cuda")
        dy = torch.empty(batch, device="cuda")
        ws = torch.empty(P.mlp_workspace_bytes(batch), dtype=torch.uint8, device="cuda")
        rng = np.random.default_rng(seed)
        step = 0
        history = []
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(n)).cuda()
            tot = 0.0
            for b0 in range(0, n - batch + 1, batch):
                idx = perm[b0:b0 + batch]
                xb, tb = x[idx].contiguous(), tt[idx].contiguous()
                P.mlp_forward(self.params, xb, y, ws)
                P.mlp_mse_grad(y, tb, dy)
                P.mlp_backward(self.params, xb, dy, g, ws)
                step += 1
                P.mlp_adam_step(self.params, g, m, v, step, lr=lr)
            history.append(step)
        P.mlp_pack_bf16(self.params, self.packed)
        torch.cuda.synchronize()
        return history

    def predict(self, thetas):
        torch = self.torch
        x = self._x(np.atleast_2d(thetas))
        y = torch.empty(x.shape[0], device="cuda")
        P.mlp_infer_bf16(self.packed, x, y)
        return np.exp(y.cpu().numpy().astype(np.float64) * self.sd_t + self.mu_t)


def da_mcmc(builder, surrogate, theta0, lo, hi, n_steps, dchi2, step_frac=0.05, seed=8, use_surrogate=True,
            log=None, normals=None, uniforms=None, refit=None, refit_every=50, adapt_steps=0):
    """Delayed-acceptance random-walk Metropolis over a uniform prior box,
    many walkers advanced together: each step proposes for every walker,
    screens with the surrogate, and builds the survivors' models in one batch.
    The random numbers are drawn from `seed` (per step: normals [n_w, d], then
    uniforms [n_w, 2]) unless given as normals [n_steps][n_w][d] and uniforms
    [n_steps][n_w][2].
    refit(thetas, chi2s): optional, called every refit_every steps during the
    first adapt_steps steps with every full build made so far (the chains'
    neighbourhood); it retrains the surrogate, whose values at the current
    states are then recomputed.  The screen is fixed after adapt_steps (the
    chain after that point leaves the posterior invariant whatever the screen).
    Returns the chains and counters; n_full_builds_after_adapt and
    n_stage1_after_adapt count the steps after adaptation."""
    rng = np.random.default_rng(seed)
    th = np.array(theta0, dtype=np.float64)
    n_w, d = th.shape
    scale = step_frac * (np.asarray(hi) - np.asarray(lo))
    chi = builder.chi2(th)
    n_unconv = int((~getattr(builder, "last_converged", np.ones(n_w, dtype=bool))).sum())
    chi_s = surrogate.predict(th) if use_surrogate else chi.copy()
    chains = np.empty((n_steps, n_w, d))
    n_full, n_s1, n_acc = len(th), 0, 0
    built_th, built_chi = [th.copy()], [chi.copy()]
    full_at_adapt = s1_at_adapt = None
    t0 = time.perf_counter()
    for k in range(n_steps):
        if k == adapt_steps:
            full_at_adapt, s1_at_adapt = n_full, n_s1
        if refit is not None and use_surrogate and 0 < k < adapt_steps and k % refit_every == 0:
            refit(np.concatenate(built_th), np.concatenate(built_chi))
            chi_s = surrogate.predict(th)
        z = rng.normal(size=(n_w, d)) if normals is None else np.asarray(normals[k])
        u = rng.uniform(size=(n_w, 2)) if uniforms is None else np.asarray(uniforms[k])
        prop = th + scale * z
        inside = np.all((prop >= lo) & (prop <= hi), axis=1)
        if use_surrogate:
            cs = surrogate.predict(prop)
            # stage 1: ln L~ = -chi~ / dchi2
            s1 = inside & (np.log(u[:, 0]) < -(cs - chi_s) / dchi2)
        else:
            cs = None
            s1 = inside.copy()
        idx = np.flatnonzero(s1)
        n_s1 += len(idx)
        if len(idx):
            cf = builder.chi2(prop[idx])
            n_unconv += int((~getattr(builder, "last_converged", np.ones(len(idx), dtype=bool))).sum())
            n_full += len(idx)
            built_th.append(prop[idx].copy())
            built_chi.append(np.asarray(cf, dtype=np.float64).copy())
            for j, i in enumerate(idx):
                if use_surrogate:
                    a2 = -(cf[j] - chi[i]) / dchi2 + (cs[i] - chi_s[i]) / dchi2
                else:
                    a2 = -(cf[j] - chi[i]) / dchi2
                if np.log(u[i, 1 if use_surrogate else 0]) < a2:
                    th[i], chi[i] = prop[i], cf[j]
                    if use_surrogate:
                        chi_s[i] = cs[i]
                    n_acc += 1
        chains[k] = th
        if log and (k + 1) % max(1, n_steps // 10) == 0:
            log(f"mcmc step {k + 1}/{n_steps}: full builds {n_full}, accepted {n_acc}")
    el = time.perf_counter() - t0
    if full_at_adapt is None:
        full_at_adapt, s1_at_adapt = n_full, n_s1
    return {"chains": chains, "n_full_builds": n_full, "n_stage1": n_s1, "n_accepted": n_acc, "seconds": el,
            "proposals": n_steps * n_w, "models_per_s": n_steps * n_w / el, "n_unconverged_builds": n_unconv,
            "n_full_builds_after_adapt": n_full - full_at_adapt, "n_stage1_after_adapt": n_s1 - s1_at_adapt,
            "built": (np.concatenate(built_th), np.concatenate(built_chi))}
