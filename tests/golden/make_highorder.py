"""Writes highorder_rk4.json: the oracle's RK4 end points for single vortices
of high order (17, 24 and 30), a few steps each from the seeded random
orthonormal state on a Lamb-Oseen core (order-40 workload recipe, own seeds).
Calls only the oracle.  The quad-precision right-hand side costs about M^8:
order 30 (one step) dominates, about 40 minutes on 8 cores; one order-40 step
would take hours, so order 40 is pinned through its right-hand side instead.

These pin the large-order stepping paths (matrix-core stepping with the stage
finished inside the next self kernel, graph replays, and the compensated
double-double contraction) to the oracle rather than to the library's own
right-hand side."""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1010_2475_amd import workloads as wl  # noqa: E402

# (order, Re, seed, t0, dt, steps)
CASES = [(17, 400.0, 17, 0.05, 2e-3, 4), (24, 700.0, 24, 0.05, 2e-3, 4), (30, 1000.0, 30, 0.05, 2e-3, 1)]


def config(M, Re, seed):
    return wl.single_random(M=M, Re=Re, seed=seed)


def main():
    oracle.build()
    path = os.path.join(HERE, "highorder_rk4.json")
    out = {"note": "oracle RK4 end points, see make_highorder.py", "cases": []}
    for (M, Re, seed, t0, dt, steps) in CASES:  # the file is rewritten after each case
        w = config(M, Re, seed)
        ta = time.time()
        x, mom = oracle.rk4(w.M, w.nu, w.lam0, t0, dt, steps, w.x, w.mom)
        print("order %d: %d steps in %.0f s" % (M, steps, time.time() - ta), flush=True)
        out["cases"].append({"M": M, "Re": Re, "seed": seed, "t0": t0, "dt": dt, "steps": steps,
                             "mom": [float(v) for v in mom[0]]})
        with open(path, "w") as f:
            json.dump(out, f)


if __name__ == "__main__":
    main()
