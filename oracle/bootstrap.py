"""Bootstrap realisations of the data and the bootstrap-marginalised chi^2
(Sec. 2.3-2.4, Eq. 6), plain NumPy in FP64.

TEST INFRASTRUCTURE ONLY.

Sec. 2.3: each realisation perturbs the observed maps by their measurement
errors and leaves the intrinsic density constraint (fixed by the potential)
alone; all realisations share the orbit library, so each is the weight problem
of Eq. 4 with a different data vector (its minimiser: `nnls.nnls_oracle`).

Eq. 6 as printed, ln sum_b exp((chi2_min - chi2_b)/2) + const, lies in
[0, ln B] whatever the fit, so it cannot rank models by itself; it is read as
the log-mean-exp marginalisation of the per-realisation likelihoods
exp(-chi2_b / 2):
    chi2_model = -2 ln[(1/B) sum_b exp(-chi2_b / 2)],
evaluated stably about chi2_min.  With B equal values it returns that value.
chi2_b is Eq. 5 (surface density and kinematics, the density block excluded)
for realisation b's weights against the observed data.
"""
import math

import numpy as np


def bootstrap_data(d, sigma, eps, col_begin, col_end):
    """Realisations out[b] = d + sigma * eps[b] on columns [col_begin, col_end)
    (the observed maps), d elsewhere.  eps: [B][C] standard normal deviates."""
    d = np.asarray(d, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    eps = np.atleast_2d(np.asarray(eps, dtype=np.float64))
    out = np.repeat(d[None, :], eps.shape[0], axis=0)
    for b in range(eps.shape[0]):
        for n in range(col_begin, col_end):
            out[b, n] = d[n] + sigma[n] * eps[b, n]
    return out


def chi2_model(chi2s):
    """-2 ln of the mean of exp(-chi2_b / 2) over the realisations, about the minimum."""
    x = [float(v) for v in chi2s]
    if not x:
        raise ValueError("chi2_model needs at least one value")
    lo = min(x)
    mean = sum(math.exp(-0.5 * (v - lo)) for v in x) / len(x)
    return lo - 2.0 * math.log(mean)
