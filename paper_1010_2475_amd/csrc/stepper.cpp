// RK4 stepping on the device: nsteps x 4 stages.  The state is read once by
// the prep kernel; afterwards every stage's last kernel writes the next
// stage's inputs (double-buffered), so a stage costs its compute kernels only.
#include <cstring>

#include "api_internal.hpp"

namespace mmvm {

// One vortex on the matrix-core path: each stage's self kernel first finishes
// the previous stage (see ApplyArgs); the state alternates between the two
// ystate buffers and reaches the caller's moments with the last stage.
static mmvm_status run_steps_fused(const DevTables& T, Workspace& W, const StageArgs& A0, double t0, int64_t nsteps,
                                   hipStream_t st)
{
    static const double cst[5] = {0.0, 0.5, 0.5, 1.0, 1.0};
    StageArgs A = A0;
    ApplyArgs P{};
    P.dt = A.dt;
    int cur = 0;
    hipError_t e = hipSuccess;
    for (int64_t n = 0; n < nsteps && e == hipSuccess; ++n) {
        for (int s = 0; s < 4 && e == hipSuccess; ++s) {
            const double ts = t0 + ((double)n + cst[s]) * A.dt;
            void* tk = timing_begin(st);
            if (n == 0 && s == 0) {
                e = launch_self(T, W.bufs, cur, false, st);
            } else {
                // finish the previous stage: (n, s - 1), or the last stage of step n - 1
                const int64_t pn = s == 0 ? n - 1 : n;
                const int ps = s == 0 ? 3 : s - 1;
                P.stage = ps;
                P.ycur = (int)(pn & 1);
                P.t_prev = t0 + ((double)pn + cst[ps]) * A.dt;
                P.t_next = ts;
                e = launch_self_apply(T, W.bufs, cur, P, st);
            }
            timing_end(tk, "self", st);
            if (e != hipSuccess) break;
            A.stage = s;
            A.cur = cur;
            A.t_stage = ts;
            A.t_next = t0 + ((double)n + cst[s + 1]) * A.dt;
            tk = timing_begin(st);
            e = launch_stage2(T, W.bufs, A, false, st);
            timing_end(tk, "stage2", st);
            cur ^= 1;
        }
    }
    if (e == hipSuccess) {
        P.stage = 3;
        P.ycur = (int)((nsteps - 1) & 1);
        P.t_prev = t0 + ((double)(nsteps - 1) + cst[3]) * A.dt;
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
        hipError_t e = launch_solo_rk4(T, W.bufs.N, W.bufs.lam0sq, W.bufs.nuv, t0, dt, nsteps, mom, W.bufs.flag, st);
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
    for (int64_t n = 0; n < nsteps; ++n) {
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
