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
    double* par_dev = nullptr;       // [3N]: lambda_{j,0}^2, the viscosity and the time offset of each vortex
    std::vector<double> par_cache;
    hipEvent_t par_event = nullptr;    // the upload from par_cache has completed
    int latched = 0;
    // captured stepping graph (eight RK4 steps of the matrix-core path, or four
    // of the double-double path), reused while its key (kind, order, batch, dt,
    // tables, the caller's state for the double-double path) holds; see stepper.cpp
    DevClock* clock = nullptr;
    hipStream_t cap_stream = nullptr;  // where the graph is captured
    hipGraphExec_t graph = nullptr;
    hipEvent_t graph_done = nullptr;   // recorded after the replays of a call
    int graph_kind = -1, graph_M = -1, graph_N = -1, graph_prec = -1;
    double graph_dt = 0.0;
    const void* graph_tables = nullptr;
    const void* graph_x = nullptr;
    const void* graph_mom = nullptr;
    // graphs replaced while possibly queued, each with an event after its last replays
    std::vector<std::pair<hipGraphExec_t, hipEvent_t>> retired;
    void drop_graph();    // the graph is not in flight (the stream was synchronised)
    void retire_graph();  // the graph may be in flight; also destroys retired ones that finished

    // solo: the vortices do not interact (N = 1, or a batch of independent solves)
    mmvm_status ensure(int N, int M, bool need_dd, bool solo, hipStream_t st);
    static size_t bytes_for(int N, int M, bool need_dd, bool solo);
    // lambda0 [N]; viscosity nu[N], or the scalar nu0 for every vortex when nu is null;
    // toff [N]: each vortex's time offset (null: zero)
    mmvm_status set_params(const double* lambda0, const double* nu, double nu0, int N, hipStream_t st,
                           const double* toff = nullptr);
    void release();
    ~Workspace();
};

mmvm_status device_tables(int M, const DevTables** out);
// the tables of order M on the current device if they were built, else null (builds nothing)
const DevTables* find_device_tables(int M);
// Lays out the workspace regions of one solve of N vortices at order M from
// `base` (256-byte aligned regions; the error flag first) and binds them to
// *bufs, *clock and *par ([3N]: lambda_{j,0}^2, nu_j, time offsets); returns the bytes
// needed.  With base == nullptr it only returns the size.
size_t stage_layout(char* base, int N, int M, bool need_dd, bool solo, StageBufs* bufs, DevClock** clock,
                    double** par);

// per-kernel timing (mmvm_timing_enable): timing_on, timing_begin, timing_end in kernels.hpp
// replays of captured stepping graphs since the process started
void count_graph_replays(int64_t n);
int64_t graph_replays();
Workspace* workspace_for(hipStream_t st);
mmvm_status validate(const mmvm_problem* prob);
bool use_dd(int M, mmvm_precision prec);
mmvm_status run_prep(const DevTables& T, Workspace& W, int cur, const double* xin, const double* min_, double t,
                     mmvm_precision prec, hipStream_t st);
mmvm_status run_stage(const DevTables& T, Workspace& W, mmvm_precision prec, const StageArgs& A, hipStream_t st);
// the same on explicit buffers; shape fixes the pair kernel's launch shape (null: the autotuner's)
mmvm_status run_prep_bufs(const DevTables& T, const StageBufs& B, int cur, const double* xin, const double* min_,
                          double t, mmvm_precision prec, hipStream_t st);
mmvm_status run_stage_bufs(const DevTables& T, const StageBufs& B, mmvm_precision prec, const StageArgs& A,
                           hipStream_t st, const PairShape* shape);
// the pair-kernel shape already chosen for (order, precision, N) in this process, or the default (never tunes)
PairShape pair_shape_known(int M, bool f32, int N);
mmvm_status run_steps(const DevTables& T, Workspace& W, double t0, double dt, int64_t nsteps, double* x,
                      double* mom, mmvm_precision prec, hipStream_t st);

}  // namespace mmvm
