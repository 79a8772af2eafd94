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
PEAK_HBM = 8.0e12  # MI355X HBM3E, bytes/s
PEAK_FP32 = 157.3e12  # MI355X FP32 vector, the published figure (packed FP32 instructions are not used here)
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
# and written per launch; FETCH_SIZE read 131084.8 KiB, WRITE_SIZE 262147.5 KiB).
# Valid only for the kernel sources it was taken on.
TRAFFIC_STAGE2 = {"fetch_kib": 3239.8, "write_kib": 169.1, "fetch_scale": 262144.0 / 131084.8,
                  "write_scale": 262144.0 / 262147.5,
                  "sources_sha256": {"kernels.hip": "8f022ac73420ed8a2e648137bffa0701a374aafb67440319d8608db3f54760d4",
                                     "kernels.hpp": "a0d7a78e1c6f36cd875dd4c34788830eaaf17b6e5eb04a464db3aa2561c309d2"}}


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
        for k in ("prep", "self", "pair", "pair_mp", "pair_far", "stage2", "emit", "apply", "solo"):
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
                    # the pair stage: the near kernel plus, when split off, the far kernel
                    pair_ms = kt["pair"]["avg_ms"] + sum(kt[k]["avg_ms"] for k in ("pair_mp", "pair_far") if k in kt)
                    ach = fl / (pair_ms * 1e-3)
                    # packed FP32 is kept out of the kernels, so FP32 and FP64 vector code
                    # share the 78.6 TFLOP/s rate (and the tuner often runs FP64 for the mixed path)
                    peak = PEAK_FP64
                    e["pair_roofline"] = {"bound": "alu", "achieved": ach / 1e12, "peak": peak / 1e12,
                                          "unit": "TFLOP/s", "frac": ach / peak, "pairs": pairs,
                                          "flops_per_pair": pair_flops(w.M), "avg_stage_ms": pair_ms,
                                          "note": "near-form flops for every pair (the far-field kernel does "
                                                  "fewer for the pairs it takes)"}
            r[pname] = e
        out[name] = r
    return out



# the paper's tab:error (section "Numerical convergence"), quoted as context
PAPER_TAB_ERROR = {1: (0.0125, 0.0034, 0.0113, 0.0028), 2: (0.0248, 0.0067, 0.0225, 0.0058),
                   4: (0.0488, 0.0138, 0.0443, 0.0123), 8: (0.0943, 0.0309, 0.0848, 0.0309),
                   16: (0.1742, 0.0821, 0.1532, 0.0956)}


def tripole_leg(mm, torch, wl, times=(1, 2, 4, 8, 16), n=256, half=4.0):
    """The coarse-grid tripole (section "Tripole Relaxation"): the 6 x 6 grid
    at orders 0 and 2 against the order-24 single particle, relative L2 and
    Linf errors of the vorticity on an n x n grid over [-half, half]^2 (as in
    tab:error).  FP64, RK4 dt 1e-3; each run stepped to the listed times and
    reconstructed there with mmvm_vorticity_grid."""
    dev = torch.device("cuda:0")
    h = 2.0 * half / (n - 1)
    runs = (("ref", wl.tripole_reference()), (0, wl.tripole_coarse(M=0)), (2, wl.tripole_coarse(M=2)))
    fields, wall = {}, {}
    for key, w in runs:
        print("  tripole %s: order %d, N %d, to t=%g" % (key, w.M, w.N, times[-1]), file=sys.stderr, flush=True)
        X = torch.tensor(w.x, device=dev)
        Mo = torch.tensor(w.mom, device=dev)
        om = torch.empty((n, n), dtype=torch.float64, device=dev)
        done, out = 0, []
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        for T in times:
            k = int(round(T / w.dt)) - done
            mm.step(w.M, w.nu, w.lam0, done * w.dt, w.dt, k, X, Mo, mm.FP64)
            done += k
            mm.vorticity_grid(w.M, w.nu, w.lam0, done * w.dt, X, Mo, -half, -half, h, n, n, om)
            out.append(om.cpu().numpy())
        wall[key] = time.perf_counter() - t_a
        fields[key] = out
    rows = []
    for i, T in enumerate(times):
        ref = fields["ref"][i]
        r = {"t": T}
        for M in (0, 2):
            d = fields[M][i] - ref
            r["e%d_L2" % M] = float(np.sqrt((d ** 2).sum() / (ref ** 2).sum()))
            r["e%d_Linf" % M] = float(np.abs(d).max() / np.abs(ref).max())
        r["ratio_L2"] = r["e0_L2"] / r["e2_L2"]
        if T in PAPER_TAB_ERROR:
            r["paper"] = dict(zip(("e0_L2", "e2_L2", "e0_Linf", "e2_Linf"), PAPER_TAB_ERROR[T]))
        rows.append(r)
    return {"grid": "%d x %d over [-%g, %g]^2" % (n, n, half, half), "errors": rows,
            "wall_s": {str(k): v for k, v in wall.items()},
            "workload": "omega_0 = phi00 + 4 delta (phi20 - phi02), lambda0 = 1, delta = 0.25, Re 1000; coarse: "
                        "6 x 6 vortices on [-1, 1]^2 of core lambda0, circulation omega_0(x_j) times the node "
                        "area; reference: that blurred field as one particle of order 24 (the moments of the 36 "
                        "Gaussians about the centre)"}


def shear_leg(mm, torch, wl, Res=(500, 800, 1000, 1500, 2000, 3000, 4000), M=24, delta=0.1, t_end=200.0,
              dt_out=1.0):
    """Shear diffusion (section "Shear diffusion / Results"): the perturbed
    Lamb-Oseen vortex eq:IC_sd (delta 0.1, lambda0 2) at order 24 for the
    paper's Reynolds numbers, stepped as one batch, with the non-axisymmetric
    enstrophy E(t) every dt_out.  The collapse of the early decay on t/Re^{1/3}
    is reported as the spread (max / min over Re) of the times at which E/E(0)
    first falls below 1/2 and 1/4, scaled by Re^{1/3} and by Re."""
    dev = torch.device("cuda:0")
    works = [wl.single_quadrupole(M=M, delta=delta, Re=Re) for Re in Res]
    dt = works[0].dt
    nu = [w.nu for w in works]
    lam = [float(w.lam0[0]) for w in works]
    X = torch.tensor(np.concatenate([w.x for w in works]), device=dev)
    Mo = torch.tensor(np.concatenate([w.mom for w in works]), device=dev)
    E = torch.zeros((len(works), 1), dtype=torch.float64, device=dev)
    nout = int(round(t_end / dt_out))
    kout = int(round(dt_out / dt))
    series = np.zeros((nout + 1, len(works)))
    t_enst = 0.0

    def enstrophy(step):
        t = step * dt
        for i, w in enumerate(works):
            lt = math.sqrt(lam[i] ** 2 + 4.0 * nu[i] * t)
            mm.enstrophy_nonaxi(M, nu[i], lam[i], t, X[i:i + 1], Mo[i:i + 1], 0.0, 0.0, 10.0 * lt, 512, 128, E[i])
        return E[:, 0].cpu().numpy()

    print("  shear diffusion: %d solves of order %d to t=%g" % (len(works), M, t_end), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_a = time.perf_counter()
    series[0] = enstrophy(0)
    for o in range(1, nout + 1):
        mm.step_batch(M, nu, lam, (o - 1) * kout * dt, dt, kout, X, Mo, mm.MIXED)
        te = time.perf_counter()
        series[o] = enstrophy(o * kout)
        t_enst += time.perf_counter() - te
    wall = time.perf_counter() - t_a
    ts = dt_out * np.arange(nout + 1)
    rel = series / series[0]

    def first_below(col, f):
        idx = np.nonzero(col <= f)[0]
        if len(idx) == 0:
            return None
        i = idx[0]
        # log-linear interpolation between the bracketing outputs
        a, b = math.log(col[i - 1]), math.log(col[i])
        return float(ts[i - 1] + (math.log(f) - a) / (b - a) * dt_out)

    coll = {}
    for f in (0.5, 0.25):
        tf = [first_below(rel[:, i], f) for i in range(len(works))]
        if any(v is None for v in tf):
            coll["E/E0=%g" % f] = {"t": tf}
            continue
        s13 = [t / Re ** (1.0 / 3.0) for t, Re in zip(tf, Res)]
        s1 = [t / Re for t, Re in zip(tf, Res)]
        coll["E/E0=%g" % f] = {"t": tf, "t_over_Re13": s13, "t_over_Re": s1,
                               "spread_Re13": max(s13) / min(s13), "spread_Re": max(s1) / min(s1)}
    keep = list(range(0, nout + 1, max(1, nout // 50)))
    return {"Re": list(Res), "order": M, "delta": delta, "t_end": t_end, "E0": series[0].tolist(),
            "E_over_E0": {"t": ts[keep].tolist(), "by_Re": {str(Re): rel[keep, i].tolist()
                                                           for i, Re in enumerate(Res)}},
            "collapse": coll, "wall_s": wall, "enstrophy_wall_s": t_enst,
            "quadrature": "512 Gauss-Legendre nodes in r^2 on [0, (10 lambda(t))^2], 128 angles"}


def adaptive_leg(mm, torch, wl):
    """The runs of the paper's implementation note, with the adaptive
    Dormand-Prince 5(4) integrator at RelTol = AbsTol = 1e-8 (as its ode45):
    eq:IC_sd (delta 0.1, lambda0 2) at Re 1000 from t = 0 to 2000 at orders 2,
    18 and 22, and the 6 x 6 coarse tripole at order 2 from t = 0 to 50 (the
    last also against fixed-step RK4 at dt 1e-3)."""
    dev = torch.device("cuda:0")
    cases = [("IC_sd_order2_t2000", wl.single_quadrupole(M=2, delta=0.1, Re=1000.0), 2000.0, "< 1 s"),
             ("IC_sd_order18_t2000", wl.single_quadrupole(M=18, delta=0.1, Re=1000.0), 2000.0, "3.35 min"),
             ("IC_sd_order22_t2000", wl.single_quadrupole(M=22, delta=0.1, Re=1000.0), 2000.0, "10.65 min"),
             ("tripole_coarse_order2_t50", wl.tripole_coarse(M=2), 50.0, "about 6 min")]
    out = {}
    for name, w, T, paper in cases:
        print("  adaptive %s" % name, file=sys.stderr, flush=True)
        X = torch.tensor(w.x, device=dev)
        Mo = torch.tensor(w.mom, device=dev)
        mm.prepare(w.M)
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        st = mm.integrate_adaptive(w.M, w.nu, w.lam0, 0.0, T, 1e-8, 1e-8, 1e-3, X, Mo, mm.FP64)
        mm.sync()
        secs = time.perf_counter() - t_a
        r = dict(st)
        r.update({"wall_s": secs, "t_end": T, "N": w.N, "M": w.M, "paper_ode45_wall": paper})
        if w.N > 1:
            X2 = torch.tensor(w.x, device=dev)
            M2 = torch.tensor(w.mom, device=dev)
            mm.step(w.M, w.nu, w.lam0, 0.0, 1e-3, int(round(T / 1e-3)), X2, M2, mm.FP64)
            mm.sync()
            a, b = Mo.cpu().numpy(), M2.cpu().numpy()
            r["max_abs_diff_vs_rk4_dt1e-3"] = {"mom": float(np.abs(a - b).max()),
                                               "x": float(np.abs(X.cpu().numpy() - X2.cpu().numpy()).max())}
        out[name] = r
    return out


def recon_leg(mm, torch, w, X, Mo, t, n=2048, reps=5):
    """Reconstruction of the order-40 state on an n x n grid (mmvm_vorticity_grid)
    and its non-axisymmetric enstrophy: per-launch durations with HIP events,
    against the grid write (HBM) and the FP64 product (2 (M+1) flops per point)."""
    dev = torch.device("cuda:0")
    om = torch.empty((n, n), dtype=torch.float64, device=dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    lam_t = math.sqrt(float(w.lam0[0]) ** 2 + 4.0 * w.nu * t)
    half = 8.0 * lam_t
    h = 2.0 * half / (n - 1)
    mm.vorticity_grid(w.M, w.nu, w.lam0, t, X, Mo, -half, -half, h, n, n, om)  # workspace, first launch
    mm.sync()
    mm.timing_enable(True)
    try:
        for _ in range(reps):
            mm.vorticity_grid(w.M, w.nu, w.lam0, t, X, Mo, -half, -half, h, n, n, om)
            mm.enstrophy_nonaxi(w.M, w.nu, w.lam0, t, X, Mo, 0.0, 0.0, 10.0 * lam_t, 512, 128, E)
        mm.sync()
        rec_ms, rec_n = mm.timing_get("recon")
        ens_ms, ens_n = mm.timing_get("enstrophy")
    finally:
        mm.timing_enable(False)
    avg = rec_ms / max(rec_n, 1)
    M1 = w.M + 1
    write_b = 8.0 * n * n
    table_b = 8.0 * M1 * 2 * n
    flops = 2.0 * M1 * n * n
    ach_bw = (write_b + table_b) / (avg * 1e-3)
    return {"grid": "%d x %d" % (n, n), "order": w.M, "avg_launch_ms": avg, "launches": rec_n,
            "roofline": {"kernel": "k_recon_grid", "bound": "hbm", "achieved": ach_bw / 1e9, "peak": PEAK_HBM / 1e9,
                         "unit": "GB/s", "frac": ach_bw / PEAK_HBM, "bytes_per_launch": write_b + table_b,
                         "fp64_tflops": flops / (avg * 1e-3) / 1e12,
                         "fp64_frac": flops / (avg * 1e-3) / PEAK_FP64},
            "enstrophy_avg_launch_ms": ens_ms / max(ens_n, 1),
            "enstrophy_quadrature": "512 x 128 nodes, %d vorticity evaluations per launch" % (512 * 128)}


def dilute_leg(mm, torch, wl, orc):
    """The dilute field (N 4096, order 4, mean spacing 2: most source chunks
    in a target's far field), both precisions: rate, kernel durations, the
    launch shape the tuner chose (far=1: the far chunks go to the multipole
    kernel) and the error against the oracle on sampled rows."""
    w = wl.dilute_multi()
    r = {"N": w.N, "M": w.M, "steps": w.steps}
    for pname, prec in (("mixed", mm.MIXED), ("fp64", mm.FP64)):
        print("  dilute_multi %s: %d steps" % (pname, w.steps), file=sys.stderr, flush=True)
        rate, ms, x, mom, t_end = run_workload(mm, torch, w, w.steps, prec)
        e = {"moment_updates_per_s": rate, "ms_per_step": ms}
        if orc is not None:
            e["err_vs_oracle"] = rhs_error(mm, torch, orc, wl, w, x, mom, t_end, prec, [0, w.N // 2, w.N - 1],
                                           list(range(w.K)))
        kt = kernel_times(mm, torch, w, prec)
        e["kernels_ms_per_launch"] = {k: v["avg_ms"] for k, v in kt.items()}
        r[pname] = e
    r["tuned_shapes"] = [ln for ln in mm.autotune_report().splitlines() if "order=4 " in ln]
    return r


STUDIES = ("dilute_far_field", "tripole", "shear_diffusion", "adaptive", "reconstruction")


def run_studies(mm, torch, wl, orc, recon_state, which=STUDIES):
    out = {}
    for name in which:
        print("study %s" % name, file=sys.stderr, flush=True)
        t_a = time.perf_counter()
        if name == "dilute_far_field":
            r = dilute_leg(mm, torch, wl, orc)
        elif name == "tripole":
            r = tripole_leg(mm, torch, wl)
        elif name == "shear_diffusion":
            r = shear_leg(mm, torch, wl)
        elif name == "adaptive":
            r = adaptive_leg(mm, torch, wl)
        else:
            r = recon_leg(mm, torch, *recon_state)
        r["leg_wall_s"] = time.perf_counter() - t_a
        out[name] = r
    return out


def study_leg(name):
    """One study alone (the reconstruction on the order-40 headline state
    after 200 steps), as one JSON line."""
    import torch
    from paper_1010_2475_amd import mmvm as mm
    from paper_1010_2475_amd import workloads as wl
    mm.lib()
    orc = None
    if name == "dilute_far_field":
        import oracle
        oracle.build()
        orc = oracle
    state = None
    if name == "reconstruction":
        w = wl.single_random(M=ORDER, Re=RES[1])
        dev = torch.device("cuda:0")
        X = torch.tensor(w.x, device=dev)
        Mo = torch.tensor(w.mom, device=dev)
        mm.step(w.M, w.nu, w.lam0, 0.0, w.dt, 200, X, Mo, mm.MIXED)
        mm.sync()
        state = (w, X, Mo, 200 * w.dt)
    print(json.dumps(run_studies(mm, torch, wl, orc, state, (name,))))


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


ONLY = {"single_quadrupole": lambda wl: wl.single_quadrupole(), "single_random": lambda wl: wl.single_random(),
        "dilute_multi": lambda wl: wl.dilute_multi(), "random_multi": lambda wl: wl.random_multi(),
        "two_clusters": lambda wl: wl.two_clusters(),
        "dilute_multi_16384": lambda wl: wl.dilute_multi(N=16384, steps=20)}


def only_leg(args):
    """One workload alone, stepped with the state resident on the device: W
    warmup steps, then K timed steps (for kernel traces and counters)."""
    import torch
    from paper_1010_2475_amd import mmvm as mm
    from paper_1010_2475_amd import workloads as wl
    w = ONLY[args.only](wl)
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
        if w.N > 1:
            out[pname]["kernels_ms_per_launch"] = {k: v["avg_ms"] for k, v in kernel_times(mm, torch, w, prec).items()}
    out["tuned_shapes"] = mm.autotune_report().splitlines()
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
    ap.add_argument("--no-studies", action="store_true",
                    help="skip the paper's studies (dilute far field, tripole errors, shear diffusion, adaptive "
                         "runs, reconstruction)")
    ap.add_argument("--study", choices=sorted(STUDIES), default=None,
                    help="run one of the paper's studies alone and print its line")
    args = ap.parse_args()
    if args.only:
        only_leg(args)
        return
    if args.study:
        study_leg(args.study)
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

    if not args.no_studies:
        X0, M0 = res["mixed"]["state"]
        dev = torch.device("cuda:0")
        t_end = (args.warmup + args.steps) * works[0].dt
        out["studies"] = run_studies(mm, torch, wl, None if args.no_error else orc,
                                     (works[0], torch.tensor(X0[:1], device=dev), torch.tensor(M0[:1], device=dev),
                                      t_end))

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
