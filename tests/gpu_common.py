"""Helpers shared by the GPU tests: run a workload through the HIP library
and through the oracle on identical seeded inputs."""
import numpy as np

import workloads as W


def lib():
    import paper_2607_00117_amd as P
    P.load()
    return P


def obs_small(spec=None):
    return dict(W.SMALL["obs"] if spec is None else spec)


def gpu_integrate(cfg, ics, dt, n_steps, dtype, obs=None, components=None, omega=None, euler=None):
    """Returns (A, overflow, drift, flags) as numpy arrays from integrate_and_bin."""
    import torch
    P = lib()
    comps = cfg["components"] if components is None else components
    pot = P.build_potential(comps, cfg["omega"] if omega is None else omega, cfg["euler"] if euler is None else euler)
    spec = dict(cfg["obs"] if obs is None else obs)
    o = P.obs_spec(spec)
    n = ics.shape[1]
    td = torch.float64 if dtype == "f64" else torch.float32
    dev = torch.device("cuda:0")
    ic_t = torch.from_numpy(np.ascontiguousarray(ics)).to(dev, td)
    dt_t = torch.from_numpy(np.ascontiguousarray(dt)).to(dev, td)
    nc = P.ncon(o)
    A = torch.empty((n, nc), dtype=td, device=dev)
    ov = torch.empty((n, 2), dtype=torch.float64, device=dev)
    dr = torch.empty(n, dtype=torch.float64, device=dev)
    fl = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = torch.empty(P.integrate_workspace_bytes(o, 1, n, n_steps, 1 if dtype == "f32" else 2), dtype=torch.uint8,
                     device=dev)
    P.integrate_and_bin(pot, [0, n], ic_t, dt_t, n_steps, o, A, ov, dr, fl, ws)
    torch.cuda.synchronize()
    return A.cpu().numpy(), ov.cpu().numpy(), dr.cpu().numpy(), fl.cpu().numpy()


def oracle_integrate(cfg, ics, dt, n_steps, obs=None, components=None, omega=None, euler=None, f32_state=False):
    import oracle as O
    comps = cfg["components"] if components is None else components
    pot = O.make_pot(comps, cfg["omega"] if omega is None else omega)
    R = O.euler_matrix(*(cfg["euler"] if euler is None else euler))
    ob = O.make_obs(dict(cfg["obs"] if obs is None else obs), R)
    return O.integrate_and_bin(pot, ob, ics, dt, n_steps, f32_state=f32_state)


def counts_from_fractions(A, n_steps, ncopy=4):
    c = np.rint(A.astype(np.float64) * (ncopy * n_steps))
    return c.astype(np.int64)
