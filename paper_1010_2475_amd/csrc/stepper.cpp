// RK4 stepping on the device: nsteps x 4 stages.  The state is read once by
// the prep kernel; afterwards every stage's last kernel writes the next
// stage's inputs (double-buffered), so a stage costs its compute kernels only.
#include <cstring>

#include "api_internal.hpp"

namespace mmvm {

mmvm_status run_steps(const DevTables& T, Workspace& W, double nu, double t0, double dt, int64_t nsteps,
                      double* x, double* mom, mmvm_precision prec, hipStream_t st)
{
    static const double cst[5] = {0.0, 0.5, 0.5, 1.0, 1.0};
    StageArgs A;
    std::memset(&A, 0, sizeof(A));
    A.mode = MODE_RK4;
    A.dt = dt;
    A.nu = nu;
    A.x = x;
    A.mom = mom;
    A.want_pair = W.bufs.N > 1;
    A.want_f32 = prec == MMVM_MIXED;
    int cur = 0;
    mmvm_status r = run_prep(T, W, cur, x, mom, t0, nu, prec, st);
    if (r != MMVM_OK) return r;
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
