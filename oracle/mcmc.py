"""Metropolis-Hastings and delayed-acceptance MH oracle (NumPy, FP64).

TEST INFRASTRUCTURE ONLY.

Delayed acceptance (Christen & Fox 2005) with a symmetric proposal: a proposal
theta' first passes a screen on the cheap density pi~ with probability
min(1, pi~(theta') / pi~(theta)); only then is the expensive density pi
evaluated and the move accepted with probability
min(1, pi(theta') pi~(theta) / (pi(theta) pi~(theta'))).  The chain leaves pi
invariant whatever pi~ is.  The random numbers are inputs: normals [n, d]
for the proposals and two uniforms [n, 2] for the two stages.
"""
import numpy as np


def mh(logp, theta0, chol, normals, uniforms):
    th = np.array(theta0, dtype=np.float64)
    lp = logp(th)
    out = np.empty((len(normals), th.size))
    n_eval = 1
    for k in range(len(normals)):
        prop = th + chol @ normals[k]
        lq = logp(prop)
        n_eval += 1
        if np.log(uniforms[k, 0]) < lq - lp:
            th, lp = prop, lq
        out[k] = th
    return out, n_eval


def da_mh(logp, logp_s, theta0, chol, normals, uniforms):
    """Returns (chain, number of expensive evaluations, stage-1 accepts)."""
    th = np.array(theta0, dtype=np.float64)
    lp, ls = logp(th), logp_s(th)
    out = np.empty((len(normals), th.size))
    n_eval, n_s1 = 1, 0
    for k in range(len(normals)):
        prop = th + chol @ normals[k]
        lsq = logp_s(prop)
        if np.log(uniforms[k, 0]) < lsq - ls:
            n_s1 += 1
            lq = logp(prop)
            n_eval += 1
            if np.log(uniforms[k, 1]) < (lq - lp) + (ls - lsq):
                th, lp, ls = prop, lq, lsq
        out[k] = th
    return out, n_eval, n_s1
