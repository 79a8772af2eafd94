"""Writes dense16_rk4_1200.json: the oracle's RK4 trajectory end point for a
dense field of 16 overlapping vortices of order 5 (positions uniform in
[-1, 1]^2, circulations U[-1, 1], cores U[0.2, 0.5], Re 600, dt 1e-3, 1200
steps).  Calls only the oracle; takes about half an hour on 8 cores.

Over these steps the normalised higher moments of the field grow (the
truncated moment system of strongly overlapping vortices), which makes the end
point a pin of long-horizon stepping rather than of a single right-hand side."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1010_2475_amd import workloads as wl  # noqa: E402

STEPS = 1200


def config():
    w = wl.random_multi(N=16, M=5, Re=600.0, seed=7, steps=2000)
    w.x = np.random.default_rng(11).uniform(-1.0, 1.0, (16, 2))
    return w


def main():
    w = config()
    oracle.build()
    x, mom = oracle.rk4(w.M, w.nu, w.lam0, 0.0, w.dt, STEPS, w.x, w.mom)
    out = {"note": "oracle RK4 end point, see make_dense16.py", "steps": STEPS, "N": w.N, "M": w.M,
           "x": [[float(v) for v in r] for r in x], "mom": [[float(v) for v in r] for r in mom]}
    with open(os.path.join(HERE, "dense16_rk4_1200.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
