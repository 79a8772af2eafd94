"""Benchmark of the MMVM hot path on one MI355X.

Workload: the single-particle high-order case -- one vortex of order 40 (861
Hermite moments), seeded random orthonormal coefficients a~_k ~ N(0,1) 0.05
2^{-ord k/2} on top of a Lamb-Oseen core (lambda0 = 2), three independent
solves at Re = 1e2, 1e3, 1e4, classic RK4 with dt = 1e-3.  A step is one RK4
step of all three solves (stepped together as one batch of independent solves).  Metric: moment-updates/s
(one moment-update = one coefficient advanced one RK4 step), for the mixed
path (value) and the strict FP64 path (reported beside it), each with its
error against the FP64 oracle on sampled right-hand-side rows.  A served leg
replays the first requests of the seeded Poisson request stream through the
solve server and reports p50/p99 latency beside its throughput, at the stream's
own rate and at 1/20 of it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--serve-requests R] [--serve-slots S] [--no-configs]
       [--no-cpu-baseline] [--no-error] [--copy-calibration]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_FP64 = 78.6e12  # MI355X dense FP64, matrix cores and vector ALUs alike
ORDER = 40
RES = (1e2, 1e3, 1e4)


def stage2_flops(M):
    """Multiply-adds of the factorised contraction of one vortex (x2 flops)."""
    GM = max(2 * M, 1)
    macs = 0
    for k2 in range(M + 1):
        for g1 in range(GM + 1):
            for l2 in range(M + 1):
                macs += sum(1 for i in range(min(l2, k2) + 1) if g1 + k2 + l2 - 2 * i + 1 <= GM)
                macs += sum(1 for i in range(min(l2, k2 - 1) + 1) if 1 <= g1 + k2 + l2 - 2 * i - 1 <= GM)
        macs += 2 * (GM + 1) * sum(M - l1 + 1 for l1 in range(M + 1))
        for k1 in range(M - k2 + 1):
            for l1 in range(M + 1):
                macs += max(0, min(l1, k1 - 1) + 1)
                macs += sum(1 for i in range(min(l1, k1) + 1) if k1 + l1 - 2 * i + 1 <= GM)
    return 2 * macs


def self_flops(M):
    GM = max(2 * M, 1)
    macs = 0
    for s in range(1, GM + 1):
        for g2 in range(s + 1):
            g1 = s - g2
            macs += sum(1 for m2 in range(g2 & 1, M + 1, 2) for m1 in range(g1 & 1, M - m2 + 1, 2))
    return 2 * macs


# HBM traffic of the matrix-core stage-2 kernel (one launch = the 3 solves),
# from two rocprofv3 --pmc runs of this benchmark (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch) scaled by what the same counters read for a
# plain device copy of known size (bench.py --copy-calibration: 256 MiB read
# and written per launch; FETCH_SIZE read 131083 KiB, WRITE_SIZE 262146 KiB).
# Valid only for the kernel sources it was taken on.
TRAFFIC_STAGE2 = {"fetch_kib": 3243.8, "write_kib": 169.1, "fetch_scale": 262144.0 / 131084.6,
                  "write_scale": 262144.0 / 262146.5,
                  "sources_sha256": {"kernels.hip": "85f4cda03884d4dd1e8d30bb3f0718e51585ca86d4444e2e3a6db028798c9fb1",
                                     "kernels.hpp": "7eab1c200a65f53cc9b7280e7af9fff0a39ee427f48b7206bf1d854c16a9459a"}}


def stage2_traffic_bytes():
    """Calibrated bytes per launch, or None once the kernel sources changed."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1010_2475_amd", "csrc")
    for name, sha in TRAFFIC_STAGE2["sources_sha256"].items():
        with open(os.path.join(csrc, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != sha:
                return None
    t = TRAFFIC_STAGE2
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def serve_leg(mm, wl, n_req, budget, slots, prec, stretch=1.0):
    """Replays the first n_req requests of the seeded request stream at their
    arrival times (multiplied by stretch) through the solve server; latency =
    arrival -> result ready."""
    reqs = [(ta * stretch, w) for ta, w in wl.request_stream(n=n_req)]
    # a server loads the coefficient tables of the orders it serves at startup
    tp = time.perf_counter()
    for M in sorted({w.M for _, w in reqs}):
        mm.prepare(M)
    prep_s = time.perf_counter() - tp
    srv = mm.Server(budget, slots)
    t0 = time.perf_counter()
    pending = []
    for ta, w in reqs:
        delay = t0 + ta - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tk = srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, prec)
        pending.append((tk, w))
    lat, work, failed = [], 0, 0
    while pending:
        rest = []
        for tk, w in pending:
            try:
                r = srv.poll(tk, w.N, w.M)
            except mm.MMVMError as e:  # a solve whose state turned non-finite is reported, not retried
                if e.status != -8:
                    raise
                failed += 1
                st = e.stats
            else:
                if r is None:
                    rest.append((tk, w))
                    continue
                st = r[2]
            lat.append(1e3 * (st["t_done"] - st["t_arrive"]))
            work += w.N * w.K * st["steps"]
        pending = rest
        if pending:
            time.sleep(0.002)
    wall = time.perf_counter() - t0
    srv.close()
    window = reqs[-1][0]
    offered = sum(w.N * w.K * w.steps for _, w in reqs)
    return {"requests": n_req, "hbm_budget_bytes": budget, "slots": slots, "tables_prepared_s": prep_s,
            "offered_requests_per_s": n_req / window, "arrival_window_s": window,
            "offered_moment_updates_per_s": offered / window,
            "served_moment_updates_per_s": work / wall, "wall_s": wall, "nonfinite_requests": failed,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(max(lat))}}


def measure(mm, torch, works, prec, steps, warmup):
    """Steps the solves as one batch of independent single-vortex solves
    (mmvm_step_batch: one launch of each kernel for all of them)."""
    dev = torch.device("cuda:0")
    M, dt = works[0].M, works[0].dt
    nu = [w.nu for w in works]
    lam = [float(w.lam0[0]) for w in works]
    X = torch.tensor(np.concatenate([w.x for w in works]), device=dev)
    Mo = torch.tensor(np.concatenate([w.mom for w in works]), device=dev)
    st = torch.cuda.current_stream()
    mm.step_batch(M, nu, lam, 0.0, dt, warmup, X, Mo, prec, stream=st)
    mm.sync(st)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_a = time.perf_counter()
    start.record(st)
    mm.step_batch(M, nu, lam, warmup * dt, dt, steps, X, Mo, prec, stream=st)
    end.record(st)
    mm.sync(st)
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    states = [(X[i:i + 1].contiguous(), Mo[i:i + 1].contiguous()) for i in range(len(works))]
    return t_b - t_a, [start.elapsed_time(end)], states


def other_configs(mm, torch, wl):
    """The other workloads at their full sizes, both precisions: whole-run
    moment-updates/s with the state resident on the device (after 3 untimed
    steps); the two-cluster run is cut to 50 of its 200 steps."""
    dev = torch.device("cuda:0")
    cases = (("single_quadrupole_M10_Re1000", wl.single_quadrupole(), 1000),
             ("random_multi_N64_M6_Re500", wl.random_multi(), 500),
             ("two_clusters_N4096_M4_Re2000", wl.two_clusters(), 50))
    out = {}
    for name, w, steps in cases:
        r = {"N": w.N, "M": w.M, "steps": steps}
        for pname, prec in (("mixed", mm.MIXED), ("fp64", mm.FP64)):
            X = torch.tensor(w.x, device=dev)
            Mo = torch.tensor(w.mom, device=dev)
            mm.step(w.M, w.nu, w.lam0, 0.0, w.dt, 3, X, Mo, prec)
            mm.sync()
            t_a = time.perf_counter()
            mm.step(w.M, w.nu, w.lam0, 3 * w.dt, w.dt, steps, X, Mo, prec)
            mm.sync()
            secs = time.perf_counter() - t_a
            r[pname] = {"moment_updates_per_s": w.N * w.K * steps / secs, "ms_per_step": 1e3 * secs / steps}
        out[name] = r
    return out


def rhs_error(mm, torch, orc, w, x, mom, prec, t, rows):
    dev = torch.device("cuda:0")
    X = torch.tensor(x, device=dev)
    Mo = torch.tensor(mom, device=dev)
    dX, dM = torch.zeros_like(X), torch.zeros_like(Mo)
    mm.rhs(w.M, w.nu, w.lam0, t, X, Mo, dX, dM, prec)
    mm.sync()
    g = dM.cpu().numpy()[0]
    ref, _ = orc.rhs_rows(w.M, w.nu, w.lam0, t, x, mom, [0] * len(rows), rows)
    from paper_1010_2475_amd import workloads as wl
    n = wl.orthonormal_scale(w.M, math.sqrt(w.lam0[0] ** 2 + 4 * w.nu * t))
    return max(abs(g[r] - ref[i]) * n[r] for i, r in enumerate(rows)) / np.abs(g * n).max()


ONLY = {"single_quadrupole": "single_quadrupole", "single_random": "single_random",
        "random_multi": "random_multi", "two_clusters": "two_clusters"}


def only_leg(args):
    """One workload alone, stepped with the state resident on the device: W
    warmup steps, then K timed steps (for kernel traces and counters)."""
    import torch
    from paper_1010_2475_amd import mmvm as mm
    from paper_1010_2475_amd import workloads as wl
    w = getattr(wl, ONLY[args.only])()
    dev = torch.device("cuda:0")
    precs = [args.precision] if args.precision else ["mixed", "fp64"]
    out = {"workload": args.only, "N": w.N, "M": w.M, "steps": args.steps, "warmup": args.warmup}
    for pname in precs:
        prec = mm.MIXED if pname == "mixed" else mm.FP64
        X = torch.tensor(w.x, device=dev)
        Mo = torch.tensor(w.mom, device=dev)
        print("%s %s: %d warmup + %d steps" % (args.only, pname, args.warmup, args.steps), file=sys.stderr,
              flush=True)
        if args.warmup:
            mm.step(w.M, w.nu, w.lam0, 0.0, w.dt, args.warmup, X, Mo, prec)
        mm.sync()
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        mm.step(w.M, w.nu, w.lam0, args.warmup * w.dt, w.dt, args.steps, X, Mo, prec)
        mm.sync()
        torch.cuda.synchronize()
        secs = time.perf_counter() - t_a
        out[pname] = {"moment_updates_per_s": w.N * w.K * args.steps / secs, "ms_per_step": 1e3 * secs / args.steps}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip timing the other workloads")
    ap.add_argument("--serve-requests", type=int, default=100)
    ap.add_argument("--serve-budget-mb", type=int, default=256)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy (y = 1.0 * x over 256 MiB, five launches), the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters to bytes, and exit")
    ap.add_argument("--only", choices=sorted(ONLY), default=None,
                    help="time one workload alone (both precisions unless --precision) and print its line; for "
                         "profiling one path under rocprofv3")
    ap.add_argument("--precision", choices=("mixed", "fp64"), default=None)
    args = ap.parse_args()
    if args.only:
        only_leg(args)
        return
    if args.copy_calibration:
        import torch
        n = 32 * 1024 * 1024  # doubles: 256 MiB read and 256 MiB written per launch
        x = torch.ones(n, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(5):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 5}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the workload's solves are independent and this build "
              "measures one MI355X; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1010_2475_amd import mmvm as mm
    from paper_1010_2475_amd import workloads as wl

    mm.lib()
    works = [wl.single_random(M=ORDER, Re=Re) for Re in RES]
    K = works[0].K
    res = {}
    for name, prec in (("mixed", mm.MIXED), ("fp64", mm.FP64)):
        print("timing %s: %d warmup + %d steps" % (name, args.warmup, args.steps), file=sys.stderr, flush=True)
        secs, lat, states = measure(mm, torch, works, prec, args.steps, args.warmup)
        res[name] = {"secs": secs, "lat_ms": lat, "states": states,
                     "value": len(works) * K * args.steps / secs, "ms_per_step": 1e3 * secs / args.steps}

    # per-kernel durations with HIP events on the launch streams (separate pass)
    kt_steps = min(args.steps, 200)
    kernels = {}
    for name, prec in (("mixed", mm.MIXED), ("fp64", mm.FP64)):
        mm.timing_enable(True)
        measure(mm, torch, works, prec, kt_steps, 0)
        kernels[name] = {k: mm.timing_get(k) for k in ("prep", "self", "stage2", "emit", "apply")}
        mm.timing_enable(False)
    # algorithmic flops per launch: every launch processes all the solves of the batch
    nb = len(works)
    flops = {"prep": 0, "self": nb * self_flops(ORDER), "stage2": nb * stage2_flops(ORDER), "emit": 0, "apply": 0}
    kern = kernels["mixed"]
    dom = max(("self", "stage2"), key=lambda k: kern[k][0])
    avg_ms = kern[dom][0] / max(kern[dom][1], 1)
    achieved = flops[dom] / (avg_ms * 1e-3)

    out = {
        "metric": "moment-updates/s (mixed path; strict FP64 path beside it) at stated error vs the FP64 oracle",
        "value": res["mixed"]["value"],
        "unit": "moment-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["mixed"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single vortex, order 40 (861 moments), seeded random orthonormal "
                               "coefficients on a Lamb-Oseen core, Re 1e2/1e3/1e4 (3 solves stepped as one "
                               "batch of independent solves), RK4 dt 1e-3",
                   "solves": len(works), "order": ORDER, "moments_per_solve": K},
        "fp64": {"value": res["fp64"]["value"], "ms_per_step": res["fp64"]["ms_per_step"],
                 "dtype": "f64 state, double-double self contraction"},
        "timed_batch_gpu_ms": res["mixed"]["lat_ms"][0],
        "kernels_ms_per_launch": {p: {k: (v[0] / v[1] if v[1] else None) for k, v in kernels[p].items()}
                                  for p in kernels},
        "roofline": {"kernel": dom, "bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64,
                     "traffic": stage2_traffic_bytes() if dom == "stage2" else None,
                     "flops_per_launch": flops[dom], "avg_launch_ms": avg_ms,
                     "note": "algorithmic flops of the factorised contraction of the 3 vortices of one launch (the "
                             "matrix-core kernel also multiplies the zero padding of its operands); duration "
                             "from runtime-stamped start/end events of each launch on its stream; traffic = "
                             "calibrated FETCH_SIZE + WRITE_SIZE bytes per launch (null once the kernel sources "
                             "differ from the profiled ones), about 45x the algorithmic bytes: every launch "
                             "refills the L2 of each of the 8 XCDs with the constant operand tables"},
    }

    if not args.no_configs:
        print("timing the other workloads", file=sys.stderr, flush=True)
        out["other_configs"] = other_configs(mm, torch, wl)

    if args.serve_requests > 0:
        print("serving %d requests" % args.serve_requests, file=sys.stderr, flush=True)
        out["serve"] = serve_leg(mm, wl, args.serve_requests, args.serve_budget_mb << 20, args.serve_slots, mm.MIXED)
        out["serve"]["workload"] = ("first requests of the seeded served stream: Poisson arrivals (mean gap "
                                    "5 ms), half single-particle orders 10-40, half multi-vortex N 16-1024 "
                                    "orders 2-6, 200-2000 RK4 steps, mixed precision")
        # the same requests at 1/20 of the arrival rate, a load one GPU keeps up with
        print("serving %d requests at 1/20 of the rate" % args.serve_requests, file=sys.stderr, flush=True)
        out["serve_light"] = serve_leg(mm, wl, args.serve_requests, args.serve_budget_mb << 20, args.serve_slots,
                                       mm.MIXED, stretch=20.0)
        out["serve_light"]["workload"] = "the same requests with arrival times stretched 20x (mean gap 100 ms)"

    if not args.no_error or not args.no_cpu_baseline:
        import oracle
        oracle.build()
    if not args.no_error:
        rows = [wl.index(1, 1), wl.index(6, 5), wl.index(10, 14), wl.index(20, 20), wl.index(0, 39),
                wl.index(33, 7)]
        w = works[1]
        t_end = (args.warmup + args.steps) * w.dt
        for name, prec in (("mixed", mm.MIXED), ("fp64", mm.FP64)):
            X, Mo = res[name]["states"][1]
            err = rhs_error(mm, torch, oracle, w, X.cpu().numpy(), Mo.cpu().numpy(), prec, t_end, rows)
            (out if name == "mixed" else out["fp64"])["err_vs_oracle"] = err
        out["err_note"] = ("normwise error of dM/dt in orthonormal coefficients on %d sampled rows at the "
                           "final state of the Re=1e3 solve" % len(rows))

    if not args.no_cpu_baseline:
        # the oracle as it stands, on a bounded sample: 32 right-hand-side rows
        # spread over all shells of one solve; 4 rows = one moment-update
        w = works[1]
        rows = list(range(0, K, max(1, K // 64)))[:64]
        t0 = time.perf_counter()
        oracle.rhs_rows(w.M, w.nu, w.lam0, 0.0, w.x, w.mom, [0] * len(rows), rows)
        dt_cpu = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = {"value": len(rows) / (4.0 * dt_cpu), "unit": "moment-updates/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "%d rows of one order-40 right-hand side (quad-precision oracle), "
                                         "%.1f s; 4 rows = 1 moment-update" % (len(rows), dt_cpu)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
