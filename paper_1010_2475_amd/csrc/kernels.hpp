// Device-side entry points (launchers) of the MMVM hot path.  All pointers are
// device pointers; all launches are asynchronous on `stream`.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mmvm {

// Device copies of the tables of one order (see tables.hpp), per device.
struct DevTables {
    int M, K, P, GM, KG, T0N;
    const double* t0_hi;   // [tri(T0N)]
    const double* t0_lo;
    const double* f0_hi;   // [M+1]^3
    const double* f0_lo;
    const double* f1_hi;
    const double* f1_lo;
    const double* c1_hi;   // [K]
    const double* c1_lo;
    const double* kap0;    // [P+1][P+1]
    const double* kap1;
    const double* hol;     // [P+1]
};

// Stage state and scratch of one solve of N vortices at order M.
struct StageBufs {
    int N;
    const double* lam0sq;  // [N] lambda_{j,0}^2
    double* xs;            // [N][2] stage input positions
    double* ys;            // [N][K] stage input moments
    double* accx;          // [N][2] RK4 accumulators
    double* accm;          // [N][K]
    double* lam2;          // [N] lambda_j(t_s)^2
    double* alpha;         // [N][K] scaled moments M_k / lambda^{|k|}
    double* alphaT;        // [K][N] the same, transposed (FP64 pair kernel)
    float* alphaT32;       // [K][N] FP32 copy (mixed pair kernel)
    double* s_self;        // [N][KG] self velocity-derivative table (lambda units)
    double* s_self_lo;     // [N][KG] its low part (double-double path), or null
    double* s_pair;        // [N][KG] pair velocity-derivative table
    int* flag;             // device error flag (bit 0: zero circulation, bit 1: non-finite)
};

enum StageMode { MODE_RHS = 0, MODE_RK4 = 1 };

struct StageArgs {
    int mode;
    int stage;         // RK4 stage 0..3
    double t_stage;    // time of this stage
    double t_next;     // time of the next stage input (for lambda)
    double dt;
    double nu;
    // RK4 state (in place) / RHS outputs
    double* x;         // user positions  [N][2]
    double* mom;       // user moments    [N][K]
    double* dx;        // RHS output      [N][2]
    double* dmom;      // RHS output      [N][K]
};

// prep: stage input (xs, ys) -> lam2, alpha, alphaT; checks circulation/finiteness
hipError_t launch_prep(const DevTables& T, const StageBufs& B, const double* xin, const double* min_,
                       double t, double nu, bool need_pair, bool need_f32, hipStream_t st);
// self velocity-derivative table; dd = use double-double
hipError_t launch_self(const DevTables& T, const StageBufs& B, bool dd, hipStream_t st);
// pair velocity-derivative table (N > 1); f32 = mixed precision
hipError_t launch_pair(const DevTables& T, const StageBufs& B, bool f32, int lanes_per_pair,
                       hipStream_t st);
// stage-2 contraction + drift + RK4 bookkeeping
hipError_t launch_stage2(const DevTables& T, const StageBufs& B, const StageArgs& A, bool dd,
                         hipStream_t st);

// the pair kernel is compiled for orders 0..kMaxPairOrder
constexpr int kMaxPairOrder = 6;
bool pair_order_supported(int M);

// prints a HIP error with its location to stderr (unless MMVM_QUIET is set)
void report_hip_error(hipError_t e, const char* where);

}  // namespace mmvm
