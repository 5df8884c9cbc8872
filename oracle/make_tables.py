"""Writes the circular-speed tables the seeded initial conditions are built from.

For each workload potential it tabulates, on a radius grid in the midplane,
the azimuth-averaged potential Phi(R), circular speed v_c(R) with
v_c^2 = R <-dPhi/dR> and E_c = Phi + v_c^2 / 2, all from the FP64 oracle.
Output: workloads/tables/<name>.json.  Run: python -m oracle.make_tables
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def table(components, r_lo, r_hi, n, n_az):
    pot = O.make_pot(components, 0.0)
    R = np.geomspace(r_lo, r_hi, n)
    phi = np.zeros(n)
    vc2 = np.zeros(n)
    for i, r in enumerate(R):
        for k in range(n_az):
            a = 2 * math.pi * (k + 0.5) / n_az
            x = np.array([r * math.cos(a), r * math.sin(a), 0.0])
            g = O.accel(pot, x)
            phi[i] += O.phi(pot, x) / n_az
            vc2[i] += -r * (g[0] * math.cos(a) + g[1] * math.sin(a)) / n_az
    vc = np.sqrt(np.maximum(vc2, 0.0))
    return dict(R=R.tolist(), Phi=phi.tolist(), vc=vc.tolist(), Ec=(phi + 0.5 * vc2).tolist(),
                n_azimuths=n_az, components=[[k, list(p)] for k, p in components])


def main():
    out = os.path.join(ROOT, "workloads", "tables")
    os.makedirs(out, exist_ok=True)
    jobs = [(W.SMALL["table"], W.SMALL["components"], 1)]
    jobs.append((W.BARRED["table"], W.BARRED["components"], 32))
    for name, comps, naz in jobs:
        t = table(comps, 0.01, 30.0, 400, naz)
        with open(os.path.join(out, name + ".json"), "w") as f:
            json.dump(t, f)
        print(name, "written")


if __name__ == "__main__":
    main()
