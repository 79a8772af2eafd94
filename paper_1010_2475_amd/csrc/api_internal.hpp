// Internal interfaces shared by the C ABI, the stepper and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/mmvm.h"
#include "kernels.hpp"

namespace mmvm {

// Above this order the FP64 path runs the self velocity table and the stage-2
// contraction in double-double: their alternating sums lose ~1.45x per order
// to cancellation, and plain FP64 would exceed a 1e-12 normwise error.
constexpr int kDDThreshold = 24;

struct Workspace {
    std::mutex mu;
    char* base = nullptr;
    size_t bytes = 0;
    int N = 0, M = 0;
    StageBufs bufs{};
    int* flag_ptr = nullptr;
    double* lam0_dev = nullptr;
    std::vector<double> lam0_cache;
    int latched = 0;

    mmvm_status ensure(int N, int M, bool need_dd, hipStream_t st);
    static size_t bytes_for(int N, int M, bool need_dd);
    mmvm_status set_lambda0(const double* lambda0, int N, hipStream_t st);
    void release();
    ~Workspace() { release(); }
};

mmvm_status device_tables(int M, const DevTables** out);

// per-kernel timing (mmvm_timing_enable); no-ops when disabled
bool timing_on();
void* timing_begin(hipStream_t st);
void timing_end(void* tok, const char* name, hipStream_t st);
Workspace* workspace_for(hipStream_t st);
mmvm_status validate(const mmvm_problem* prob);
bool use_dd(int M, mmvm_precision prec);
mmvm_status run_prep(const DevTables& T, Workspace& W, int cur, const double* xin, const double* min_, double t,
                     double nu, mmvm_precision prec, hipStream_t st);
mmvm_status run_stage(const DevTables& T, Workspace& W, mmvm_precision prec, const StageArgs& A, hipStream_t st);
mmvm_status run_steps(const DevTables& T, Workspace& W, double nu, double t0, double dt, int64_t nsteps,
                      double* x, double* mom, mmvm_precision prec, hipStream_t st);

}  // namespace mmvm
