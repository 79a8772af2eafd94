// RK4 stepping on the device: nsteps x 4 stages.  The state is read once by
// the prep kernel; afterwards every stage's last kernel writes the next
// stage's inputs (double-buffered), so a stage costs its compute kernels only.
#include <cstdlib>
#include <cstring>

#include "api_internal.hpp"

namespace mmvm {

// One vortex on the matrix-core path: each stage's self kernel first finishes
// the previous stage (see ApplyArgs); the state alternates between the two
// ystate buffers and reaches the caller's moments with the last stage.
//
// Steps 1 .. nsteps-1 repeat with period two (the state buffer alternates by
// step; the stage buffers return to buffer 0 after four stages), so they run
// as replays of one captured graph of kGraphSteps steps (an even number) when
// there are enough of them.  The replays take their stage times from a device
// clock (t0, n) that the graph's last node advances by kGraphSteps; the graph
// is kept in the workspace and reused by later calls with the same order,
// batch and dt.  Several steps per graph leave fewer gaps between replays.
static const double kStageC[5] = {0.0, 0.5, 0.5, 1.0, 1.0};
constexpr int kGraphSteps = 8;
static_assert(kGraphSteps % 2 == 0, "the state buffers alternate by step");
constexpr int64_t kGraphMinSteps = 8;

// MMVM_GRAPHS=0 in the environment keeps every step on direct launches
static bool graphs_enabled()
{
    const char* e = std::getenv("MMVM_GRAPHS");
    return !(e && e[0] == '0');
}

// The launches of step n (n >= 1; step 0 starts without a previous stage).
// With clock set, the stage times come from the device clock: n is then an
// offset from clock.n, and the last stage 2 advances the clock when bump.
static hipError_t launch_step(const DevTables& T, Workspace& W, StageArgs A, double t0, int64_t n,
                              DevClock* clock, bool bump, hipStream_t st)
{
    ApplyArgs P{};
    P.dt = A.dt;
    int cur = 0;
    for (int s = 0; s < 4; ++s) {
        const double ts = t0 + ((double)n + kStageC[s]) * A.dt;
        const int64_t pn = s == 0 ? n - 1 : n;
        const int ps = s == 0 ? 3 : s - 1;
        P.stage = ps;
        P.t_prev = t0 + ((double)pn + kStageC[ps]) * A.dt;
        P.t_next = ts;
        P.clock = clock;
        P.n_prev = (int)pn;
        P.n_next = (int)n;
        P.c_prev = kStageC[ps];
        P.c_next = kStageC[s];
        // with a clock, n is relative to an odd clock.n: parities are fixed
        P.ycur = (int)((clock ? pn + 1 : pn) & 1);
        void* tk = timing_begin(st);
        hipError_t e = launch_self_apply(T, W.bufs, cur, P, st);
        timing_end(tk, "self", st);
        if (e != hipSuccess) return e;
        A.stage = s;
        A.cur = cur;
        A.t_stage = ts;
        A.t_next = t0 + ((double)n + kStageC[s + 1]) * A.dt;
        A.clock_bump = (bump && s == 3) ? clock : nullptr;
        A.clock_steps = kGraphSteps;
        tk = timing_begin(st);
        e = launch_stage2(T, W.bufs, A, false, st);
        timing_end(tk, "stage2", st);
        if (e != hipSuccess) return e;
        cur ^= 1;
    }
    return hipSuccess;
}

// One step of the double-double path (self, stage 2 and emit kernels of each
// stage; the stage buffers return to buffer 0 after the four stages) with its
// stage times taken from the device clock: the step's first kernel advances
// clock.n by one, and the emit kernels, the only ones that read a time, come
// after it.  The emits update the caller's state (A.x, A.mom) in place.
static hipError_t launch_dd_step(const DevTables& T, Workspace& W, StageArgs A, hipStream_t st)
{
    int cur = 0;
    for (int s = 0; s < 4; ++s) {
        A.stage = s;
        A.cur = cur;
        A.clock = W.clock;
        A.n_rel = 0;
        A.c_next = kStageC[s + 1];
        hipError_t e = launch_self(T, W.bufs, cur, true, st, s == 0 ? W.clock : nullptr);
        if (e == hipSuccess) e = launch_stage2(T, W.bufs, A, true, st);
        if (e == hipSuccess) e = launch_emit(T, W.bufs, A, true, st);
        if (e != hipSuccess) return e;
        cur ^= 1;
    }
    return hipSuccess;
}

// One step of interacting vortices of the small orders (pair kernels, then
// the fused stage-2 / RK4 kernel of each stage; the stage buffers return to
// buffer 0 after the four stages), q steps after the graph's first: the fused
// kernel, the only one that reads a time, takes it from the device clock.  Its
// RK4 update writes the caller's state in place.
static hipError_t launch_small_step(const DevTables& T, Workspace& W, StageArgs A, int q, mmvm_precision prec,
                                    hipStream_t st)
{
    int cur = 0;
    for (int s = 0; s < 4; ++s) {
        A.stage = s;
        A.cur = cur;
        A.clock = W.clock;
        A.n_rel = q;
        A.c_next = kStageC[s + 1];
        if (run_stage_bufs(T, W.bufs, prec, A, st, nullptr) != MMVM_OK) return hipErrorUnknown;
        cur ^= 1;
    }
    return hipSuccess;
}

enum { kGraphMFMA = 0, kGraphDD = 1, kGraphSmall = 2 };
constexpr int kDDGraphSteps = 4;     // steps per graph of the double-double path
constexpr int kSmallGraphSteps = 8;  // steps per graph of interacting small orders

// The workspace's stepping graph of this kind for this (order, batch, dt, and
// for the double-double path the caller's state), captured on first use; null
// if capture is not possible here.
static hipGraphExec_t stepping_graph(const DevTables& T, Workspace& W, const StageArgs& A, int kind, hipStream_t st,
                                     mmvm_precision prec = MMVM_FP64)
{
    const bool own_state = kind == kGraphDD || kind == kGraphSmall;  // the graph updates the caller's state
    const void* gx = own_state ? (const void*)A.x : nullptr;
    const void* gm = own_state ? (const void*)A.mom : nullptr;
    const int gp = kind == kGraphSmall ? (int)prec : -1;  // the pair kernels differ by precision
    if (W.graph && W.graph_kind == kind && W.graph_M == T.M && W.graph_N == W.bufs.N && W.graph_dt == A.dt &&
        W.graph_tables == &T && W.graph_x == gx && W.graph_mom == gm && W.graph_prec == gp)
        return W.graph;
    // an older graph may still be queued: it is retired behind the event of
    // its last replays and destroyed once that has fired
    W.retire_graph();
    // captured on the workspace's own stream (the caller's may be the null
    // stream, which cannot be captured); nothing runs during a capture, and
    // the replays go to the caller's stream
    if (!W.cap_stream && hipStreamCreateWithFlags(&W.cap_stream, hipStreamNonBlocking) != hipSuccess) {
        W.cap_stream = nullptr;
        (void)hipGetLastError();
        return nullptr;
    }
    hipStream_t cs = W.cap_stream;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    hipError_t e;
    if (kind == kGraphDD) {
        e = hipSuccess;
        for (int q = 0; q < kDDGraphSteps && e == hipSuccess; ++q) e = launch_dd_step(T, W, A, cs);
    } else if (kind == kGraphSmall) {
        e = hipSuccess;
        for (int q = 0; q < kSmallGraphSteps && e == hipSuccess; ++q) e = launch_small_step(T, W, A, q, prec, cs);
        if (e == hipSuccess) e = launch_advance_clock(W.clock, kSmallGraphSteps, cs);
    } else {
        e = hipSuccess;
        for (int q = 0; q < kGraphSteps && e == hipSuccess; ++q)
            e = launch_step(T, W, A, 0.0, q, W.clock, q == kGraphSteps - 1, cs);
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &g);
    hipGraphExec_t x = nullptr;
    if (e == hipSuccess && ec == hipSuccess && g) {
        if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) x = nullptr;
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (!x) return nullptr;
    if (!W.graph_done && hipEventCreateWithFlags(&W.graph_done, hipEventDisableTiming) != hipSuccess) {
        W.graph_done = nullptr;
        (void)hipGraphExecDestroy(x);
        return nullptr;
    }
    W.graph = x;
    W.graph_kind = kind;
    W.graph_prec = gp;
    W.graph_x = gx;
    W.graph_mom = gm;
    W.graph_M = T.M;
    W.graph_N = W.bufs.N;
    W.graph_dt = A.dt;
    W.graph_tables = &T;
    return x;
}

static mmvm_status run_steps_fused(const DevTables& T, Workspace& W, const StageArgs& A0, double t0, int64_t nsteps,
                                   hipStream_t st)
{
    StageArgs A = A0;
    A.clock_bump = nullptr;
    hipError_t e = hipSuccess;
    // step 0: its first stage has no previous stage to finish
    {
        void* tk = timing_begin(st);
        e = launch_self(T, W.bufs, 0, false, st);
        timing_end(tk, "self", st);
        int cur = 0;
        for (int s = 0; s < 4 && e == hipSuccess; ++s) {
            if (s > 0) {
                ApplyArgs P{};
                P.dt = A.dt;
                P.stage = s - 1;
                P.ycur = 0;
                P.t_prev = t0 + (0.0 + kStageC[s - 1]) * A.dt;
                P.t_next = t0 + (0.0 + kStageC[s]) * A.dt;
                tk = timing_begin(st);
                e = launch_self_apply(T, W.bufs, cur, P, st);
                timing_end(tk, "self", st);
                if (e != hipSuccess) break;
            }
            A.stage = s;
            A.cur = cur;
            A.t_stage = t0 + (0.0 + kStageC[s]) * A.dt;
            A.t_next = t0 + (0.0 + kStageC[s + 1]) * A.dt;
            tk = timing_begin(st);
            e = launch_stage2(T, W.bufs, A, false, st);
            timing_end(tk, "stage2", st);
            cur ^= 1;
        }
    }
    int64_t n = 1;
    // The graph is captured by the first call of its key whatever its length,
    // so that a short first call (a warmup, a server's first chunk) leaves the
    // capture behind it; it is replayed once a call has enough steps.
    if (e == hipSuccess && graphs_enabled() && !timing_on() && W.clock) {
        hipGraphExec_t g = stepping_graph(T, W, A, kGraphMFMA, st);
        const int64_t reps = (nsteps - 1) / kGraphSteps;
        if (g && reps > 0) {
            e = launch_set_clock(W.clock, t0, 1, st);
            for (int64_t r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(g, st);
            if (e == hipSuccess) e = hipEventRecord(W.graph_done, st);
            if (e == hipSuccess) count_graph_replays(reps);
            n += kGraphSteps * reps;
        }
    }
    for (; n < nsteps && e == hipSuccess; ++n) e = launch_step(T, W, A, t0, n, nullptr, false, st);
    if (e == hipSuccess) {
        ApplyArgs P{};
        P.dt = A.dt;
        P.stage = 3;
        P.ycur = (int)((nsteps - 1) & 1);
        P.t_prev = t0 + ((double)(nsteps - 1) + kStageC[3]) * A.dt;
        P.mom_out = A.mom;
        void* tk = timing_begin(st);
        e = launch_apply_final(T, W.bufs, P, st);
        timing_end(tk, "apply", st);
    }
    if (e != hipSuccess) {
        report_hip_error(e, "fused stepping launch");
        return MMVM_EDEVICE;
    }
    return MMVM_OK;
}

mmvm_status run_steps(const DevTables& T, Workspace& W, double t0, double dt, int64_t nsteps, double* x,
                      double* mom, mmvm_precision prec, hipStream_t st)
{
    static const double cst[5] = {0.0, 0.5, 0.5, 1.0, 1.0};
    StageArgs A;
    std::memset(&A, 0, sizeof(A));
    A.mode = MODE_RK4;
    A.dt = dt;
    A.x = x;
    A.mom = mom;
    A.want_pair = W.bufs.interact != 0;
    A.want_f32 = prec == MMVM_MIXED;
    if (!W.bufs.interact && solo_persistent(T.M, use_dd(T.M, prec))) {
        // small orders: every solve of the batch runs all its steps in one workgroup
        void* tk = timing_begin(st);
        hipError_t e = launch_solo_rk4(T, W.bufs.N, W.bufs.lam0sq, W.bufs.nuv, W.bufs.toff, t0, dt, nsteps, mom,
                                       W.bufs.flag, st);
        timing_end(tk, "solo", st);
        if (e != hipSuccess) {
            report_hip_error(e, "k_solo_rk4 launch");
            return MMVM_EDEVICE;
        }
        return MMVM_OK;
    }
    int cur = 0;
    mmvm_status r = run_prep(T, W, cur, x, mom, t0, prec, st);
    if (r != MMVM_OK) return r;
    if (stage2_fuses_emit(T.M, use_dd(T.M, prec), !W.bufs.interact)) return run_steps_fused(T, W, A, t0, nsteps, st);
    // the double-double path (single vortices): step 0 direct, then replays
    // of a kDDGraphSteps-step graph on a clock that starts at step 0, then
    // the remaining steps direct
    const bool dd_graph = use_dd(T.M, prec) && !W.bufs.interact && graphs_enabled() && !timing_on() && W.clock;
    if (dd_graph && nsteps - 1 < kGraphMinSteps) (void)stepping_graph(T, W, A, kGraphDD, st);  // captured for later calls
    // interacting vortices of the small orders: step 0 direct (it also tunes the
    // pair kernel's shape), then replays of a kSmallGraphSteps-step graph on a
    // clock that starts at step 1, then the remaining steps direct
    const bool small_graph = W.bufs.interact && stage2_fuses_self(T.M, use_dd(T.M, prec), false) &&
                             graphs_enabled() && !timing_on() && W.clock;
    for (int64_t n = 0; n < nsteps; ++n) {
        if (n == 1 && small_graph) {
            hipGraphExec_t g = stepping_graph(T, W, A, kGraphSmall, st, prec);
            const int64_t reps = (nsteps - 1) / kSmallGraphSteps;
            if (g && reps > 0) {
                hipError_t e = launch_set_clock(W.clock, t0, 1, st);
                for (int64_t q = 0; q < reps && e == hipSuccess; ++q) e = hipGraphLaunch(g, st);
                if (e == hipSuccess) e = hipEventRecord(W.graph_done, st);
                if (e != hipSuccess) {
                    report_hip_error(e, "small-order stepping graph replay");
                    return MMVM_EDEVICE;
                }
                count_graph_replays(reps);
                n += kSmallGraphSteps * reps;  // the rest is launched directly
                if (n >= nsteps) return MMVM_OK;
            }
        }
        if (n == 1 && dd_graph && nsteps - 1 >= kGraphMinSteps) {
            hipGraphExec_t g = stepping_graph(T, W, A, kGraphDD, st);
            if (g) {
                const int64_t reps = (nsteps - 1) / kDDGraphSteps;
                hipError_t e = launch_set_clock(W.clock, t0, 0, st);
                for (int64_t q = 0; q < reps && e == hipSuccess; ++q) e = hipGraphLaunch(g, st);
                if (e == hipSuccess) e = hipEventRecord(W.graph_done, st);
                if (e != hipSuccess) {
                    report_hip_error(e, "stepping graph replay");
                    return MMVM_EDEVICE;
                }
                count_graph_replays(reps);
                n += kDDGraphSteps * reps;  // the rest is launched directly
                if (n >= nsteps) return MMVM_OK;
            }
        }
        for (int s = 0; s < 4; ++s) {
            A.stage = s;
            A.cur = cur;
            A.t_stage = t0 + ((double)n + cst[s]) * dt;
            // the next stage's time: c_{s+1}, or the next step's first stage
            A.t_next = t0 + ((double)n + cst[s + 1]) * dt;
            r = run_stage(T, W, prec, A, st);
            if (r != MMVM_OK) return r;
            cur ^= 1;
        }
    }
    return MMVM_OK;
}

}  // namespace mmvm
