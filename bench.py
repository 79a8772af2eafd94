"""Benchmark of the MMVM hot path on one MI355X.

Headline workload: the single-particle high-order case -- one vortex of order
40 (861 Hermite moments), seeded random orthonormal coefficients
a~_k ~ N(0,1) 0.05 2^{-ord k/2} on top of a Lamb-Oseen core (lambda0 = 2), three
independent solves at Re = 1e2, 1e3, 1e4, classic RK4 with dt = 1e-3, stepped
together as one batch of independent solves.  A step is one RK4 step of all
three solves.  Metric: moment-updates/s (one moment-update = one coefficient
advanced one RK4 step) of the MMVM_MIXED path (`value`; for a single vortex it
contracts in plain FP64 on the matrix cores) and of the MMVM_FP64 path (the
compensated double-double contraction) beside it, each with its error against
the oracle at the final state.

Also measured, each at its full size and step count, both precisions, with the
error against the oracle at its final state: the order-10 quadrupole (1000
steps), 64 random vortices of order 6 (500 steps), two clusters of 4096
vortices of order 4 (200 steps; with the pair kernel's roofline); the served
stream (all 2000 seeded Poisson requests, p50/p99 latency, offered vs served
load); and the oracle on the host cores (1 thread and all threads).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--serve-requests R] [--serve-slots S]
       [--no-configs] [--no-cpu-baseline] [--no-error] [--serve-light] [--copy-calibration]
       [--only WORKLOAD [--precision mixed|fp64]]
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
PEAK_FP32 = 157.3e12  # MI355X FP32 vector (the published figure; packed FP32 instructions are not used here)
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


def pair_flops(M):
    """Algorithmic flops of one ordered pair in the pair kernel (its own count;
    an FMA is 2): the contraction S[g] += sum_m alpha'_m Psi'(m + g) over every
    (m, g), 1 <= |g| <= 2M (2 K (KG - 1)); per shell n = 1..P = 3M the complex
    power, the edges (2 (n - 1) kappa-weighted FMAs each over n - 1 Gaussian
    products), the Laplacian relation (n - 1) and the lambda scaling (n + 1),
    8n + 7 in all; the incomplete-gamma start (56-term series, 112) and its
    downward recurrence (2P); the 1-D Gaussian derivatives (6P); the source
    moments' scaling (K + M) and the pair set-up (20)."""
    K = (M + 1) * (M + 2) // 2
    GM = max(2 * M, 1)
    KG = (GM + 1) * (GM + 2) // 2
    P = max(3 * M, 1)
    return 2 * K * (KG - 1) + sum(8 * n + 7 for n in range(1, P + 1)) + 112 + 2 * P + 6 * P + K + M + 20


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


# ---------------------------------------------------------------------------
# errors against the oracle (normwise, orthonormal coefficients; the scale of a
# vortex is the oracle's largest value on the sampled rows)
# ---------------------------------------------------------------------------
def gpu_rhs(mm, torch, w, x, mom, t, prec):
    dev = torch.device("cuda:0")
    X = torch.tensor(x, device=dev)
    Mo = torch.tensor(mom, device=dev)
    dX, dM = torch.zeros_like(X), torch.zeros_like(Mo)
    mm.rhs(w.M, w.nu, w.lam0, t, X, Mo, dX, dM, prec)
    mm.sync()
    return dX.cpu().numpy(), dM.cpu().numpy()


def rhs_error(mm, torch, orc, wl, w, x, mom, t, prec, js, ks):
    """Normwise error of dM/dt on rows (j in js, k in ks) and of dx/dt of those
    vortices, at the state (x, mom) and time t."""
    dx_g, dm_g = gpu_rhs(mm, torch, w, x, mom, t, prec)
    rj = [j for j in js for _ in ks]
    rk = [k for _ in js for k in ks]
    d, dxr = orc.rhs_rows(w.M, w.nu, w.lam0, t, x, mom, rj, rk)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t)
    err = 0.0
    for i, j in enumerate(js):
        n = wl.orthonormal_scale(w.M, lam_t[j])[ks]
        ref = d[i * len(ks):(i + 1) * len(ks)]
        scale = np.abs(ref * n).max()
        err = max(err, np.abs((dm_g[j, ks] - ref) * n).max() / scale)
    out = {"dmdt": float(err)}
    if w.N > 1:
        dx_r = dxr.reshape(len(js), len(ks), 2)[:, 0, :]
        out["dxdt"] = float(np.abs(dx_g[js] - dx_r).max() / max(1e-300, np.abs(dx_r).max()))
    return out


def serve_leg(mm, wl, n_req, budget, slots, prec, stretch=1.0):
    """Replays the first n_req requests of the seeded request stream at their
    arrival times (multiplied by stretch) through the solve server; latency =
    arrival -> result ready.  Requests whose state turns non-finite (the
    truncated moment system of strongly overlapping vortices) are counted
    apart: not in the latency percentiles, not in the served work."""
    reqs = [(ta * stretch, w) for ta, w in wl.request_stream(n=n_req)]
    # a server loads the coefficient tables of the orders it serves at startup
    tp = time.perf_counter()
    for M in sorted({w.M for _, w in reqs}):
        mm.prepare(M)
    prep_s = time.perf_counter() - tp
    srv = mm.Server(budget, slots)
    t0 = time.perf_counter()
    pending = []
    last_print = t0
    for i, (ta, w) in enumerate(reqs):
        delay = t0 + ta - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tk = srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, prec)
        pending.append((i, tk, w))
    lat, work, failed, done = [], 0, [], 0
    while pending:
        rest = []
        for i, tk, w in pending:
            try:
                r = srv.poll(tk, w.N, w.M)
            except mm.MMVMError as e:  # a solve whose state turned non-finite is reported, not retried
                if e.status != -8:
                    raise
                failed.append({"request": i, "N": w.N, "M": w.M, "steps": w.steps})
                done += 1
                continue
            if r is None:
                rest.append((i, tk, w))
                continue
            st = r[2]
            lat.append(1e3 * (st["t_done"] - st["t_arrive"]))
            work += w.N * w.K * st["steps"]
            done += 1
        pending = rest
        if pending:
            time.sleep(0.002)
            now = time.perf_counter()
            if now - last_print > 20.0:
                print("  served %d of %d requests (%.0f s)" % (done, n_req, now - t0), file=sys.stderr, flush=True)
                last_print = now
    wall = time.perf_counter() - t0
    srv.close()
    window = reqs[-1][0]
    offered = sum(w.N * w.K * w.steps for _, w in reqs)
    return {"requests": n_req, "hbm_budget_bytes": budget, "slots": slots, "tables_prepared_s": prep_s,
            "offered_requests_per_s": n_req / window, "arrival_window_s": window,
            "offered_moment_updates_per_s": offered / window,
            "served_moment_updates_per_s": work / wall, "wall_s": wall,
            "nonfinite_requests": len(failed), "nonfinite": failed[:50],
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(max(lat)), "of_requests": len(lat)}}


def measure(mm, torch, works, prec, steps, warmup):
    """Steps the solves as one batch of independent single-vortex solves
    (mmvm_step_batch: one launch of each kernel for all of them).  The warmup
    call is the first of its key: it builds the tables and captures the
    stepping graph, which the timed call replays."""
    dev = torch.device("cuda:0")
    M, dt = works[0].M, works[0].dt
    nu = [w.nu for w in works]
    lam = [float(w.lam0[0]) for w in works]
    X = torch.tensor(np.concatenate([w.x for w in works]), device=dev)
    Mo = torch.tensor(np.concatenate([w.mom for w in works]), device=dev)
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t_w = time.perf_counter()
    mm.step_batch(M, nu, lam, 0.0, dt, warmup, X, Mo, prec, stream=st)
    mm.sync(st)
    torch.cuda.synchronize()
    first_ms = 1e3 * (time.perf_counter() - t_w)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_a = time.perf_counter()
    start.record(st)
    mm.step_batch(M, nu, lam, warmup * dt, dt, steps, X, Mo, prec, stream=st)
    end.record(st)
    mm.sync(st)
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    return t_b - t_a, start.elapsed_time(end), first_ms, (X.cpu().numpy(), Mo.cpu().numpy())


def run_workload(mm, torch, w, steps, prec, warmup=3):
    """Whole-run moment-updates/s of one solve with its state resident on the
    device (after `warmup` untimed steps); returns the rate, ms per step, and
    the final state and time."""
    dev = torch.device("cuda:0")
    X = torch.tensor(w.x, device=dev)
    Mo = torch.tensor(w.mom, device=dev)
    mm.step(w.M, w.nu, w.lam0, 0.0, w.dt, warmup, X, Mo, prec)
    mm.sync()
    torch.cuda.synchronize()
    t_a = time.perf_counter()
    mm.step(w.M, w.nu, w.lam0, warmup * w.dt, w.dt, steps, X, Mo, prec)
    mm.sync()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t_a
    return (w.N * w.K * steps / secs, 1e3 * secs / steps, X.cpu().numpy(), Mo.cpu().numpy(),
            (warmup + steps) * w.dt)


def kernel_times(mm, torch, w, prec, steps=4):
    """Average duration per launch of each kernel over a few directly launched
    steps (runtime-stamped start/end events of every launch on its stream)."""
    dev = torch.device("cuda:0")
    X = torch.tensor(w.x, device=dev)
    Mo = torch.tensor(w.mom, device=dev)
    mm.timing_enable(True)
    try:
        mm.step(w.M, w.nu, w.lam0, 0.0, w.dt, steps, X, Mo, prec)
        mm.sync()
        out = {}
        for k in ("prep", "self", "pair", "stage2", "emit", "apply", "solo"):
            ms, n = mm.timing_get(k)
            if n:
                out[k] = {"avg_ms": ms / n, "launches": n}
    finally:
        mm.timing_enable(False)
    return out


def other_configs(mm, torch, wl, orc):
    """The other workloads at their full sizes and step counts, both precisions;
    error against the oracle at the final state of each run."""
    cases = (("single_quadrupole_M10_Re1000", wl.single_quadrupole()),
             ("random_multi_N64_M6_Re500", wl.random_multi()),
             ("two_clusters_N4096_M4_Re2000", wl.two_clusters()))
    out = {}
    for name, w in cases:
        r = {"N": w.N, "M": w.M, "steps": w.steps}
        for pname, prec in (("mixed", mm.MIXED), ("fp64", mm.FP64)):
            print("  %s %s: %d steps" % (name, pname, w.steps), file=sys.stderr, flush=True)
            rate, ms, x, mom, t_end = run_workload(mm, torch, w, w.steps, prec)
            e = {"moment_updates_per_s": rate, "ms_per_step": ms,
                 "circulation_drift": float(abs(mom[:, 0].sum() - w.mom[:, 0].sum()))}
            if orc is not None:
                js = list(range(w.N)) if w.N <= 3 else [0, w.N // 2, w.N - 1]
                ks = list(range(w.K))
                e["err_vs_oracle"] = rhs_error(mm, torch, orc, wl, w, x, mom, t_end, prec, js, ks)
            if w.N > 1:
                kt = kernel_times(mm, torch, w, prec)
                e["kernels_ms_per_launch"] = {k: v["avg_ms"] for k, v in kt.items()}
                if "pair" in kt:
                    pairs = w.N * (w.N - 1)
                    fl = pairs * pair_flops(w.M)
                    ach = fl / (kt["pair"]["avg_ms"] * 1e-3)
                    peak = PEAK_FP32 if prec == mm.MIXED and w.M <= 6 else PEAK_FP64
                    e["pair_roofline"] = {"bound": "alu", "achieved": ach / 1e12, "peak": peak / 1e12,
                                          "unit": "TFLOP/s", "frac": ach / peak, "pairs": pairs,
                                          "flops_per_pair": pair_flops(w.M), "avg_launch_ms": kt["pair"]["avg_ms"]}
            r[pname] = e
        out[name] = r
    return out


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def cpu_baseline(orc, wl, w):
    """The oracle as it stands on a bounded sample of the headline workload:
    rows of one order-40 right-hand side (4 rows = one moment-update: a row is
    evaluated once per RK4 stage), with one thread and with all threads."""
    K = w.K
    model, ncpu, avail = cpu_info()
    res = {}
    for label, threads, nrows in (("1_thread", 1, 8), ("all_threads", orc.max_threads(), 64)):
        orc.set_threads(threads)
        rows = list(range(0, K, max(1, K // nrows)))[:nrows]
        t0 = time.perf_counter()
        orc.rhs_rows(w.M, w.nu, w.lam0, 0.0, w.x, w.mom, [0] * len(rows), rows)
        secs = time.perf_counter() - t0
        res[label] = {"value": len(rows) / (4.0 * secs), "threads": threads, "rows": len(rows), "secs": secs}
    orc.set_threads(orc.max_threads())
    allt = res["all_threads"]
    return {"value": allt["value"], "unit": "moment-updates/s", "cores": allt["threads"], "kind": "oracle",
            "sample": "%d rows of one order-40 right-hand side of the headline workload (quad-precision oracle, "
                      "%.1f s on %d threads); 4 rows = 1 moment-update" % (allt["rows"], allt["secs"],
                                                                           allt["threads"]),
            "one_thread": res["1_thread"], "cpu_model": model, "nproc": ncpu, "cpus_available": avail}


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
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-budget-mb", type=int, default=256)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-light", action="store_true",
                    help="also replay the first 200 requests at 1/20 of the arrival rate")
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
        secs, gpu_ms, first_ms, state = measure(mm, torch, works, prec, args.steps, args.warmup)
        res[name] = {"secs": secs, "gpu_ms": gpu_ms, "first_ms": first_ms, "state": state,
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
        "metric": "moment-updates/s (MMVM_MIXED path; MMVM_FP64 path beside it) at stated error vs the FP64 oracle",
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
        "precision_note": "a single vortex has no pair term, so the MMVM_MIXED path (value) is plain FP64 "
                          "arithmetic on the matrix cores (uncompensated contraction); MMVM_FP64 (fp64) "
                          "accumulates the self table and stage 2 in compensated double-double",
        "first_call_ms": res["mixed"]["first_ms"],
        "fp64": {"value": res["fp64"]["value"], "ms_per_step": res["fp64"]["ms_per_step"],
                 "first_call_ms": res["fp64"]["first_ms"],
                 "dtype": "f64 state, double-double self table and stage 2"},
        "timed_batch_gpu_ms": res["mixed"]["gpu_ms"],
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
                             "differ from the profiled ones)"},
    }

    orc = None
    if not args.no_error or not args.no_cpu_baseline:
        import oracle
        oracle.build()
        orc = oracle
    if not args.no_error:
        rows = [wl.index(1, 1), wl.index(2, 0), wl.index(6, 5), wl.index(10, 14), wl.index(20, 20),
                wl.index(0, 39), wl.index(33, 7)]
        t_end = (args.warmup + args.steps) * works[0].dt
        for name, prec in (("mixed", mm.MIXED), ("fp64", mm.FP64)):
            X, Mo = res[name]["state"]
            err = 0.0
            for i, w in enumerate(works):
                e = rhs_error(mm, torch, orc, wl, w, X[i:i + 1], Mo[i:i + 1], t_end, prec, [0], rows)
                err = max(err, e["dmdt"])
            (out if name == "mixed" else out["fp64"])["err_vs_oracle"] = err
        out["err_note"] = ("normwise error of dM/dt in orthonormal coefficients on %d sampled rows at the final "
                           "state of each of the three solves (scale: the oracle's rows)" % len(rows))

    if not args.no_configs:
        print("timing the other workloads", file=sys.stderr, flush=True)
        out["other_configs"] = other_configs(mm, torch, wl, None if args.no_error else orc)

    if args.serve_requests > 0:
        print("serving %d requests" % args.serve_requests, file=sys.stderr, flush=True)
        out["serve"] = serve_leg(mm, wl, args.serve_requests, args.serve_budget_mb << 20, args.serve_slots, mm.MIXED)
        out["serve"]["workload"] = ("the seeded served stream: Poisson arrivals (mean gap 5 ms), half "
                                    "single-particle orders 10-40, half multi-vortex N 16-1024 orders 2-6, "
                                    "200-2000 RK4 steps, mixed precision")
        if args.serve_light:
            print("serving 200 requests at 1/20 of the rate", file=sys.stderr, flush=True)
            out["serve_light"] = serve_leg(mm, wl, 200, args.serve_budget_mb << 20, args.serve_slots, mm.MIXED,
                                           stretch=20.0)
            out["serve_light"]["workload"] = "the first 200 requests with arrival times stretched 20x"

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(orc, wl, works[1])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
