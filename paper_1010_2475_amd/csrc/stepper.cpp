// RK4 stepping on the device: nsteps x 4 stages, each one right-hand side.
#include <cstring>

#include "api_internal.hpp"

namespace mmvm {

mmvm_status run_steps(const DevTables& T, Workspace& W, double nu, double t0, double dt, int64_t nsteps,
                      double* x, double* mom, mmvm_precision prec, hipStream_t st)
{
    static const double cst[4] = {0.0, 0.5, 0.5, 1.0};
    StageArgs A;
    std::memset(&A, 0, sizeof(A));
    A.mode = MODE_RK4;
    A.dt = dt;
    A.nu = nu;
    A.x = x;
    A.mom = mom;
    for (int64_t n = 0; n < nsteps; ++n) {
        for (int s = 0; s < 4; ++s) {
            const double ts = t0 + ((double)n + cst[s]) * dt;
            A.stage = s;
            A.t_stage = ts;
            const bool first = (n == 0 && s == 0);
            const double* xin = first ? x : W.bufs.xs;
            const double* min_ = first ? mom : W.bufs.ys;
            mmvm_status r = run_rhs_core(T, W, xin, min_, ts, nu, prec, A, st);
            if (r != MMVM_OK) return r;
        }
    }
    return MMVM_OK;
}

}  // namespace mmvm
