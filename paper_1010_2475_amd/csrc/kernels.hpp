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
    const double* rcp;     // [128] rcp[i] = 1/i (rcp[0] = 0)
};

// Stage state and scratch of one solve of N vortices at order M.  The scaled
// moments, their source-major copies and lambda^2 are double-buffered: a
// stage reads buffer `cur` and its last kernel writes the next stage's inputs
// into buffer 1 - cur.
struct StageBufs {
    int N;
    const double* lam0sq;  // [N] lambda_{j,0}^2
    double* xs;            // [N][2] stage input positions
    double* ys;            // [N][K] stage input moments
    double* accx;          // [N][2] RK4 accumulators
    double* accm;          // [N][K]
    double* lam2[2];       // [N] lambda_j(t_s)^2
    double* alpha[2];      // [N][K] scaled moments M_k / lambda^{|k|}
    double* alphaT[2];     // [K][N] the same, source-major (FP64 pair kernel)
    float* alphaT32[2];    // [K][N] FP32 copy (mixed pair kernel)
    double* s_self;        // [N][KG] self velocity-derivative table (lambda units)
    double* s_self_lo;     // [N][KG] its low part (double-double path), or null
    double* s_pair;        // [N][KG] pair velocity-derivative table
    double* gpart;         // [N][4][K][2] partial contractions of the large-order stage 2 (hi, lo)
    unsigned* done;        // [N] workgroup counters of the large-order stage 2 (self-resetting)
    int* flag;             // device error flag (bit 0: zero circulation, bit 1: non-finite)
};

enum StageMode { MODE_RHS = 0, MODE_RK4 = 1 };

struct StageArgs {
    int mode;
    int stage;         // RK4 stage 0..3
    int cur;           // buffer holding this stage's inputs
    int want_pair;     // the next stage runs the pair kernel (write alphaT)
    int want_f32;      // ... in FP32
    double t_stage;    // time of this stage
    double t_next;     // time of the next stage (lambda of the next inputs)
    double dt;
    double nu;
    // RK4 state (in place) / RHS outputs
    double* x;         // user positions  [N][2]
    double* mom;       // user moments    [N][K]
    double* dx;        // RHS output      [N][2]
    double* dmom;      // RHS output      [N][K]
};

// prep: stage input (xin, min_) -> lam2[cur], alpha[cur], alphaT[cur]; checks
// circulation/finiteness; copies the state into (xs, ys) when they differ
hipError_t launch_prep(const DevTables& T, const StageBufs& B, int cur, const double* xin, const double* min_,
                       double t, double nu, bool need_pair, bool need_f32, hipStream_t st);
// self velocity-derivative table (orders without a fused self term); dd = double-double
hipError_t launch_self(const DevTables& T, const StageBufs& B, int cur, bool dd, hipStream_t st);
// pair velocity-derivative table (N > 1); f32 = mixed precision
hipError_t launch_pair(const DevTables& T, const StageBufs& B, int cur, bool f32, hipStream_t st);
// orders whose stage-2 kernel computes the self table itself
constexpr int kMaxSmallOrder = 10;
bool stage2_fuses_self(int M, bool dd);
// stage-2 contraction + drift + RK4 bookkeeping
hipError_t launch_stage2(const DevTables& T, const StageBufs& B, const StageArgs& A, bool dd,
                         hipStream_t st);

// the pair kernel is compiled for orders 0..kMaxPairOrder
constexpr int kMaxPairOrder = 6;
bool pair_order_supported(int M);

// prints a HIP error with its location to stderr (unless MMVM_QUIET is set)
void report_hip_error(hipError_t e, const char* where);

}  // namespace mmvm
