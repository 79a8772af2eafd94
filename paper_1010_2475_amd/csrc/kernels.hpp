// Device-side entry points (launchers) of the MMVM hot path.  All pointers are
// device pointers; all launches are asynchronous on `stream`.
#pragma once
#include <hip/hip_ext.h>
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
    const double* binom;   // [M+1][M+1] C(l, i)
    const double* fd0;     // [M+1][M+1] f0[k][i][i]
    const double* fd1;     // [M+1][M+1] f1[k][i][i]
    const double* fd0_lo;  // low parts of fd0, fd1 (double-double)
    const double* fd1_lo;
    const int* dd_la;      // double-double stage 2: task lists of steps A and C per (k2, pass, parity)
    const int* dd_lc;
    const double* wpad;    // matrix-core stage 2: banded factor operand [M+1][2][KA][LP] (k2, pass, g2, l2)
    const double* cpad;    // matrix-core stage 2: C(l, i) zero-padded [LP][LP]
    const double* t0d;     // matrix-core self table: Psi0 dense [T0R][TP] (a, b), zero beyond a + b <= T0N
    const double* c1d;     // matrix-core path: c1 dense [LP][LP] (k1, k2)
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
    int interact;          // the vortices interact (N > 1 and not a batch of independent solves)
    const double* lam0sq;  // [N] lambda_{j,0}^2
    const double* nuv;     // [N] viscosity of the solve each vortex belongs to
    const double* toff;    // [N] time offset of each vortex: lambda_j(t) is evaluated at t + toff[j]
                           // (zero except for a server batch of solves at different times)
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
    double* p_part;        // [N][groups][KG] partial pair tables of split source groups (or null)
    int pair_groups;       // > 1: the pair table is the sum of these partial tables (set per stage)
    unsigned char* far_mask;  // [N][pair_mask_stride(N)] far-field chunks of the pair kernel (or null)
    // the pair kernels' sources in spatial order (from kPairFarAlwaysN vortices):
    // source p is vortex perm[p], vortex j is source rank[j] (null: caller order)
    const int* rank;
    const int* perm;
    double* xsS;           // [N][2] stage positions of the sources (= xs when not sorted)
    double* lam2S[2];      // [N] lambda^2 of the sources (= lam2 when not sorted)
    // alphaT / alphaT32 hold the sources in the same order
    double* chunk_mp;      // [far_records(N)][kChunkRec] multipole expansions of the sorted source chunks, then of their cells (or null)
    double* s_pad;         // [N][2][KA][RP] self table of each parity by columns g2, rows r, zero-padded (matrix-core path)
    double* alphaD[2];     // [N][LP + 16][LP] alpha[m1][m2] dense, zero beyond the triangle (matrix-core path)
    double* alphaS[2];     // [N][LP][LP] (-1)^{|l|} alpha[l1][l2] stored at (l2, l1), zero beyond the triangle
    // matrix-core path, dense (k1, k2) layouts [N][LP][LP]:
    double* gpartD;        // [N][4][LP][LP] partial contractions of stage 2
    double* ystate[2];     // RK4 state y_n, alternating by step (single-vortex stepping)
    double* accD;          // RK4 accumulator (single-vortex stepping)
    double* gpart;         // [N][4][K][2] partial contractions of the large-order stage 2 (hi, lo)
    int* flag;             // device error flag (bit 0: zero circulation, bit 1: non-finite)
};

enum StageMode { MODE_RHS = 0, MODE_RK4 = 1 };

// Device-side clock of a captured stepping graph: the stage times are
// t0 + (n + c) dt with n = clock.n + a step offset baked into each node.
struct DevClock {
    double t0;
    long long n;
};
struct StageArgs {
    int mode;
    int stage;         // RK4 stage 0..3
    int cur;           // buffer holding this stage's inputs
    int want_pair;     // the next stage runs the pair kernel (write alphaT)
    int want_f32;      // ... in FP32
    double t_stage;    // time of this stage
    double t_next;     // time of the next stage (lambda of the next inputs)
    double dt;
    // RK4 state (in place) / RHS outputs
    double* x;         // user positions  [N][2]
    double* mom;       // user moments    [N][K]
    double* dx;        // RHS output      [N][2]
    double* dmom;      // RHS output      [N][K]
    DevClock* clock_bump;  // graph replay: the matrix-core stage 2 advances clock.n by clock_steps
    int clock_steps;
    // graph replay of the double-double path and of interacting small orders:
    // when clock is set the emit kernel (double-double) or the fused stage-2
    // kernel (small orders) takes t_next = t0 + (clock.n + n_rel + c_next) dt
    // (the double-double step's first self kernel advances clock.n, see
    // launch_self; the small-order graph's last node does)
    const DevClock* clock;
    int n_rel;
    double c_next;
};

// prep: stage input (xin, min_) -> lam2[cur], alpha[cur], alphaT[cur]; checks
// circulation/finiteness; copies the state into (xs, ys) when they differ
hipError_t launch_prep(const DevTables& T, const StageBufs& B, int cur, const double* xin, const double* min_,
                       double t, bool need_pair, bool need_f32, hipStream_t st);
// self velocity-derivative table (orders without a fused self term); dd = double-double.
// bump (graph replay): the kernel first advances bump->n by one
hipError_t launch_self(const DevTables& T, const StageBufs& B, int cur, bool dd, hipStream_t st,
                       DevClock* bump = nullptr);

// Matrix-core RK4 stepping of one vortex: the self kernel of stage t + 1 first
// finishes stage t from its partial contractions (RK4 update of the state held
// in ystate[ycur], scaled moments of stage t + 1 built in LDS; the row-0
// workgroups write the state, the accumulators and the signed moments of
// stage2); the last stage of a call is finished by launch_apply_final.
struct ApplyArgs {
    int stage;         // RK4 stage t whose partial sums are applied
    int ycur;          // ystate[ycur] holds y_n
    double t_prev;     // time of stage t
    double t_next;     // time of stage t + 1
    double dt;
    double* mom_out;   // launch_apply_final: y_{n+1} -> the caller's moments
    // graph replay: when clock is set, t_prev = t0 + (clock.n + n_prev + c_prev) dt
    // and t_next likewise (the host's expression, evaluated on the device)
    const DevClock* clock;
    int n_prev, n_next;
    double c_prev, c_next;
};
// sets a stepping clock (one thread; a kernel, so it may precede graph replays)
hipError_t launch_set_clock(DevClock* clock, double t0, long long n, hipStream_t st);
// advances a stepping clock by `by` steps (one thread; the last node of a graph
// whose kernels read the clock)
hipError_t launch_advance_clock(DevClock* clock, long long by, hipStream_t st);
bool stage2_fuses_emit(int M, bool dd, bool solo);
hipError_t launch_self_apply(const DevTables& T, const StageBufs& B, int cur, const ApplyArgs& P, hipStream_t st);
hipError_t launch_apply_final(const DevTables& T, const StageBufs& B, const ApplyArgs& P, hipStream_t st);
// pair velocity-derivative table (N > 1); f32 = mixed precision.  Launch
// shape: split wavefronts per target (they share its sources), tpb targets
// per workgroup; launch_pair takes the shape the autotuner picked for
// (order, precision, N).
// kind 0: the unrolled kernel, one pair per lane (split, tpb as above; for the
// mixed precision f64 = 1 runs its FP64 variant);
// kind 1: the few-vortex kernel, one pair per 16 lanes, a target's sources
// split over pair_split_groups(N) workgroups whose partial tables the stage-2
// kernel adds (pair_split.hpp); `groups` records the count at tuning time.
struct PairShape {
    int split = 1, tpb = 4;
    int kind = 0, groups = 1;
    int f64 = 0;
    int far = 0;  // kind 0: chunks of far pairs go to the multipole kernel k_pair_far
};
// the far-field split needs a mask of N x ceil(N / 64) bytes: offered up to this N
constexpr int kPairFarMaxN = 16384;
// highest order whose mixed-precision pair kernel keeps FP32 shells: there the
// normwise error stays below 1e-6 for every spectrum measured, flat included
// (6e-7); at orders 5 and 6 the FP32 shells reach 3e-6 (decaying spectra) to
// 3.5e-5 (flat), so the mixed path runs them in FP64
constexpr int kPairF32MaxOrder = 4;
// from this N the tuner only offers shapes with the far split, and the sources
// are sorted in space
constexpr int kPairFarAlwaysN = 1024;
// Multipole expansion of a chunk of 64 sorted sources about its centre, for
// the targets far from the whole chunk: terms n = 0 .. kFarPM; one record per
// chunk = centre (2), radius, pad, then the complex coefficients B_n
constexpr int kFarPM = 40;
constexpr int kChunkRec = 4 + 2 * (kFarPM + 1);
// Cells of kFarCellChunks consecutive chunks carry an expansion of their own
// (translated from their chunks'), taken for targets far from the whole cell;
// their records follow the chunk records
constexpr int kFarCellChunks = 4;
// chunk and cell records of N sorted sources
constexpr int far_records(int N)
{
    return ((N + 63) >> 6) + (((N + 63) >> 6) + kFarCellChunks - 1) / kFarCellChunks;
}
// bytes of one target's row of the far-chunk mask (chunks of 64 sources, rows
// padded to 8 bytes for 64-bit loads)
constexpr int pair_mask_stride(int N) { return (((N + 63) >> 6) + 7) & ~7; }
// sorts the sources of a stage in space (rank, perm) from the call's positions
hipError_t launch_sort_sources(const StageBufs& B, const double* x, hipStream_t st);
constexpr int kPairMaxThreads = 256;  // the kernel keeps up to 256 VGPRs + AGPRs per lane
// largest N * groups of a split launch with groups > 1
constexpr int kPairSplitMaxPartials = 1024;
inline bool pair_shape_valid(PairShape s)
{
    if (s.kind == 1) return s.groups >= 1 && s.groups <= kPairSplitMaxPartials;
    return s.kind == 0 && s.split >= 1 && s.tpb >= 1 && (s.split & (s.split - 1)) == 0 &&
           64 * s.split * s.tpb <= kPairMaxThreads;
}
// source groups of the few-vortex kernel for N vortices: at least 16 sources
// per group and about 512 workgroups in all
inline int pair_split_groups(int N)
{
    int g = (512 + N - 1) / N;
    const int cap = (N + 15) / 16;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    while (g > 1 && (long)N * g > kPairSplitMaxPartials) --g;
    return g;
}

hipError_t launch_pair(const DevTables& T, const StageBufs& B, int cur, bool f32, hipStream_t st,
                       PairShape* used = nullptr);
hipError_t launch_pair_shape(const DevTables& T, const StageBufs& B, int cur, bool f32, PairShape sh, hipStream_t st);
// the autotuner's shape for this launch (times the candidates on first use of a key)
PairShape pair_shape_for(const DevTables& T, const StageBufs& B, int cur, bool f32, hipStream_t st);
// orders whose stage-2 kernel computes the self table itself
constexpr int kMaxSmallOrder = 10;
// Persistent RK4 of independent single vortices (one workgroup per solve, all
// steps in one launch) for orders 0..kMaxSoloOrder, FP64 arithmetic.
constexpr int kMaxSoloOrder = 11;
constexpr int kSoloThreads = 1024;
bool solo_persistent(int M, bool dd);
hipError_t launch_solo_rk4(const DevTables& T, int nb, const double* lam0sq, const double* nuv, const double* toff,
                           double t0, double dt, int64_t nsteps, double* mom, int* flag, hipStream_t st);
bool stage2_fuses_self(int M, bool dd, bool solo);
// stage-2 contraction; at small orders also the drift and the RK4 bookkeeping
hipError_t launch_stage2(const DevTables& T, const StageBufs& B, const StageArgs& A, bool dd,
                         hipStream_t st);
// large orders: the contraction writes four partial sums per moment and a
// second kernel adds them and applies the drift and the RK4 bookkeeping
bool stage2_needs_emit(int M, bool dd, bool solo);
hipError_t launch_emit(const DevTables& T, const StageBufs& B, const StageArgs& A, bool dd, hipStream_t st);

// Matrix-core stage 2 (FP64, single vortex, orders kMaxSmallOrder + 1 .. kS2MaxOrder):
// shapes of its zero-padded operands.  Rows r of the velocity-derivative table
// hold g1 = par + 2r; l is padded to LP, g2 (the contraction index of the first
// product) to KA, l of the second and third products to KBP <= LP.
constexpr int kS2Threads = 512;
constexpr int kS2Waves = kS2Threads / 64;
constexpr int kS2MaxOrder = 47;
constexpr int kS2TPad = 18;  // zero rows on either side of T
constexpr int kMinMfmaOrder = 7;  // a single vortex uses the matrix-core path from this order on
// the order has matrix-core tables; the path runs for (M, precision, solo), where
// solo = the vortices do not interact (one vortex, or a batch of independent solves)
bool mfma_order(int M);
bool stage2_uses_mfma(int M, bool dd, bool solo);

struct S2Shape {
    int nrp, LP, RP, KA, KBP, LDS, LDY, LDT, NTR;
    int t, y, ps, total;  // LDS regions of the stage-2 kernel (doubles, multiples of 4)
    __host__ __device__ S2Shape(int M, int par)
    {
        const int M1 = M + 1, GM = 2 * M;
        nrp = (GM - par) / 2 + 1;
        LP = 16 * ((M1 + 15) / 16);
        RP = LP;                       // nrp <= M + 1 for either parity
        KA = 4 * ((GM >> 2) + 1);
        KBP = 4 * ((M >> 2) + 1);
        LDS = KA + 1;                  // row stride of the padded self table
        LDY = LP + 1;                  // odd strides spread the rows over the LDS banks
        LDT = LP + 1;
        NTR = GM + 1 + 2 * kS2TPad;
        const int u = (2 * M + 1) * M1;  // U of the third product, at most
        t = 0;                                        // T, sheared-friendly (second -> third product)
        y = up4(NTR * LDT);                           // Y (first -> second product), then U
        ps = y + up4(RP * LDY > u ? RP * LDY : u);    // partial sums of the last step
        total = ps + up4(kS2Waves * 64);
    }
    __host__ __device__ static int up4(int n) { return (n + 3) & ~3; }
    // per-vortex size of the padded self table (both parities)
    __host__ __device__ int spad() const { return 2 * RP * KA; }
    // rows of the dense alpha layout (zero rows beyond LP cover the k-steps of the self product)
    __host__ __device__ int LA() const { return LP + 16; }
};

// Dense Psi0 operand of the matrix-core self table: columns b < TP, rows a < T0R.
// The product for row g1 reads rows ceil(g1 / 2) .. ceil(g1 / 2) + 4 kSelfKS - 1.
constexpr int kSelfKS = (kS2MaxOrder / 2 + 4) / 4;  // k-steps over m1 of one parity
struct T0Shape {
    int T0N, TP, T0R;
    __host__ __device__ explicit T0Shape(int M)
    {
        T0N = (3 * M + 1) / 2 + 1;
        TP = 16 * ((T0N + 1 + 15) / 16);
        T0R = (2 * M + 1) / 2 + 4 * kSelfKS + 1;
    }
};

// the unrolled pair kernel is compiled for orders 0..kMaxPairOrder; above, up to
// MMVM_MAX_PAIR_ORDER, the runtime-order kernel (pair_gen.hip) runs, in FP64 for
// both precisions
constexpr int kMaxPairOrder = 6;
bool pair_order_supported(int M);
hipError_t launch_pair_gen(const DevTables& T, const StageBufs& B, int cur, hipStream_t st);
// interacting vortices above the small orders: S_pair added into the operand of
// the matrix-core (padded) or double-double stage 2
hipError_t launch_pair_into_stage2(const DevTables& T, const StageBufs& B, bool dd, hipStream_t st);
// raises a kernel's dynamic-LDS limit to `bytes`, once per (kernel, device)
hipError_t lds_limit_once(const void* fn, size_t bytes, const char* what);

// Kernel timing: while a slot is set on the calling thread, the next kernel
// launched through launch_kernel carries the slot's events, which the runtime
// stamps at that kernel's start and end (hipExtLaunchKernel).
struct TimingSlot {
    hipEvent_t start = nullptr, stop = nullptr;
    bool used = false;
};
TimingSlot*& timing_slot();
// per-kernel timing (mmvm_timing_enable); no-ops when disabled: the first kernel
// launched between begin and end is timed under `name`
bool timing_on();
void* timing_begin(hipStream_t st);
void timing_end(void* tok, const char* name, hipStream_t st);

template <typename F, typename... Args>
inline void launch_kernel(F kernel, const dim3& grid, const dim3& block, std::uint32_t shmem, hipStream_t st,
                          Args... args)
{
    TimingSlot* ts = timing_slot();
    if (ts && !ts->used) {
        ts->used = true;
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, ts->start, ts->stop, 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
    }
}

// prints a HIP error with its location to stderr (unless MMVM_QUIET is set)
void report_hip_error(hipError_t e, const char* where);

}  // namespace mmvm
