// HIP kernels (gfx950) of the MMVM hot path.
//
// Per right-hand side (one RK4 stage) the path runs these kernels:
//   k_prep    stage input -> lambda_j(t)^2, scaled moments alpha = M_k / lambda^{|k|}
//             (row-major and source-major copies), circulation/finiteness checks
//   k_self    self velocity-derivative table  S_self[g] = sum_m alpha_m Psi0(m + g)
//   k_pair    pair velocity-derivative table  S_pair[g] = sum_{j'} sum_m ... Psi(m + g; s_jj')
//             (one wavefront per target, lanes over sources, wavefront-shuffle reduction)
//   k_stage2  the factorised contraction of eq:FinalSingleI/II (self + pair share it);
//             at small orders also the drift term, the centre velocity and the RK4
//             bookkeeping, which at large orders a fifth kernel (k_emit) does
// All quantities are in "lambda units" of the target vortex: with
// alpha_l = M_l lambda^{-|l|} and S in units lambda^{|g|}, eq:moment_evolutionFinish
// becomes dM_k/dt = lambda^{|k|-2} G_k(alpha, S) with lambda-free tables.
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "../../include/mmvm.h"
#include "dd.hpp"
#include "kernels.hpp"
#include "util.hpp"

namespace mmvm {

// Raises a kernel's dynamic-LDS limit to `bytes`, once per (kernel, device): the
// runtime keeps the attribute per device.  Later calls only look the result
// up, so a launch that a caller captures into a graph makes no attribute call
// once an uncaptured launch on that device has made it.
hipError_t lds_limit_once(const void* fn, size_t bytes, const char* what)
{
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, hipError_t> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_pair(fn, dev);
    auto it = done.find(key);
    if (it != done.end()) return it->second;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        report_hip_error(e, what);
    }
    done[key] = e;
    return e;
}

// t0 + (n + c) dt as the host evaluates it, with separate roundings: HIP's
// __dmul_rn / __dadd_rn are plain operations that -ffp-contract fuses into one
// fused multiply-add, so contraction is switched off here
__device__ __forceinline__ double clock_time(double t0, long long n, double c, double dt)
{
#pragma clang fp contract(off)
    const double a = (double)n + c;
    const double p = a * dt;
    return t0 + p;
}

// ---------------------------------------------------------------------------
// prep
// ---------------------------------------------------------------------------
// x^s by binary exponentiation (at most 2 log2(s) dependent products)
__device__ __forceinline__ double pow_uint(double x, int s)
{
    double r = 1.0;
    while (s) {
        if (s & 1) r *= x;
        x *= x;
        s >>= 1;
    }
    return r;
}

// lambda^{-s} from lambda^2
__device__ __forceinline__ double inv_lambda_pow(double l2, int s) { return pow_uint(1.0 / sqrt(l2), s); }

// The two dense layouts of the scaled moments read by the matrix-core kernels
// (only allocated on that path): alphaD[m1][m2] and (-1)^{|l|} alpha at (l2, l1).
__device__ __forceinline__ void store_dense_alpha(const StageBufs& B, int buf, int M, int j, int k1, int k2, double a)
{
    if (!B.alphaD[buf]) return;
    const int LP = 16 * ((M + 16) / 16), LA = LP + 16;
    B.alphaD[buf][(long)j * LA * LP + k1 * LP + k2] = a;
    B.alphaS[buf][(long)j * LP * LP + k2 * LP + k1] = ((k1 + k2) & 1) ? -a : a;
}

// zeros of the dense layouts outside the triangle, in both buffers
__global__ __launch_bounds__(256) void k_alpha_dense_clear(StageBufs B, int M)
{
    const int LP = 16 * ((M + 16) / 16), LA = LP + 16;
    const long per = (long)LA * LP, total = (long)B.N * per;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int j = (int)(idx / per), pos = (int)(idx - (long)j * per);
        const int m1 = pos / LP, m2 = pos - m1 * LP;
        if (m1 + m2 <= M) continue;
        for (int b = 0; b < 2; ++b) {
            B.alphaD[b][idx] = 0.0;
            if (m1 < LP) B.alphaS[b][(long)j * LP * LP + m2 * LP + m1] = 0.0;
        }
    }
}

// Spatial order of the pair kernels' sources: the vortices of one call
// sorted along a Hilbert curve through their positions at the call's start, so
// that consecutive chunks of 64 sources are compact (a target's near chunks are
// few, its far chunks are skipped as wholes, and the expansions of chunks and
// cells converge close to them).  A Morton (Z) order jumps across quadrant
// edges, so chunks straddling a jump span two distant clumps: on a uniform
// field the Hilbert order halves the mean chunk radius.  One workgroup:
// bounding box of the finite positions, one scale for both axes onto a 16-bit
// grid, the curve index (32 bits) with the vortex index below it (unique keys:
// a deterministic order), bitonic sort of NP (a power of two >= N) keys in
// LDS.  Positions move within a call; the order only has to stay good, not
// exact.
constexpr int kSortThreads = 1024;

// Index of grid point (q1, q2) along the Hilbert curve of the 2^16 x 2^16 grid,
// by the curve's recursive construction read from the top level down: at each
// level the quadrant holding the point contributes (its rank along the curve)
// x (points per quadrant), and the point is mapped into the frame in which that
// quadrant's sub-curve has the standard orientation (a transpose, preceded by
// a reflection in the last quadrant of the bottom row).
__device__ __forceinline__ unsigned hilbert_index16(unsigned q1, unsigned q2)
{
    unsigned d = 0;
    for (unsigned s = 1u << 15; s > 0; s >>= 1) {
        const unsigned r1 = (q1 & s) ? 1u : 0u, r2 = (q2 & s) ? 1u : 0u;
        d += s * s * ((3u * r1) ^ r2);
        if (r2 == 0) {
            if (r1 == 1) {
                q1 = 0xFFFFu - q1;
                q2 = 0xFFFFu - q2;
            }
            const unsigned t = q1;
            q1 = q2;
            q2 = t;
        }
    }
    return d;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_sources(int N, int NP, const double* __restrict__ x,
                                                               int* __restrict__ rank, int* __restrict__ perm)
{
    extern __shared__ unsigned long long skey[];  // [NP]
    __shared__ double red[4][kSortThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double lo1 = INFINITY, hi1 = -INFINITY, lo2 = INFINITY, hi2 = -INFINITY;
    for (int j = tid; j < N; j += kSortThreads) {
        const double a = x[2 * j], b = x[2 * j + 1];
        if (isfinite(a) && isfinite(b)) {
            lo1 = fmin(lo1, a);
            hi1 = fmax(hi1, a);
            lo2 = fmin(lo2, b);
            hi2 = fmax(hi2, b);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo1 = fmin(lo1, __shfl_xor(lo1, off, 64));
        hi1 = fmax(hi1, __shfl_xor(hi1, off, 64));
        lo2 = fmin(lo2, __shfl_xor(lo2, off, 64));
        hi2 = fmax(hi2, __shfl_xor(hi2, off, 64));
    }
    if (lane == 0) {
        red[0][wv] = lo1;
        red[1][wv] = hi1;
        red[2][wv] = lo2;
        red[3][wv] = hi2;
    }
    __syncthreads();
    lo1 = red[0][0];
    hi1 = red[1][0];
    lo2 = red[2][0];
    hi2 = red[3][0];
    for (int w = 1; w < kSortThreads / 64; ++w) {
        lo1 = fmin(lo1, red[0][w]);
        hi1 = fmax(hi1, red[1][w]);
        lo2 = fmin(lo2, red[2][w]);
        hi2 = fmax(hi2, red[3][w]);
    }
    // one scale for both axes: grid cells are squares (compact chunks on elongated fields too)
    const double span = fmax(hi1 - lo1, hi2 - lo2);
    const double sc = span > 0.0 ? 65535.0 / span : 0.0;
    for (int p = tid; p < NP; p += kSortThreads) {
        unsigned long long key = ~0ull;
        if (p < N) {
            const double a = x[2 * p], b = x[2 * p + 1];
            unsigned q1 = 0, q2 = 0;
            if (isfinite(a) && isfinite(b)) {
                q1 = (unsigned)fmin(65535.0, fmax(0.0, (a - lo1) * sc));
                q2 = (unsigned)fmin(65535.0, fmax(0.0, (b - lo2) * sc));
            }
            const unsigned code = hilbert_index16(q1, q2);
            key = ((unsigned long long)code << 32) | (unsigned)p;
        }
        skey[p] = key;
    }
    __syncthreads();
    // bitonic network: each pass compare-exchanges NP/2 disjoint pairs (i, i + jj)
    for (int k = 2; k <= NP; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int t = tid; t < (NP >> 1); t += kSortThreads) {
                const int i = 2 * jj * (t / jj) + (t % jj), l = i + jj;
                const unsigned long long a = skey[i], b = skey[l];
                if ((a > b) == ((i & k) == 0)) {
                    skey[i] = b;
                    skey[l] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int p = tid; p < N; p += kSortThreads) {
        const int j = (int)(skey[p] & 0xffffffffull);
        perm[p] = j;
        rank[j] = p;
    }
}

hipError_t launch_sort_sources(const StageBufs& B, const double* x, hipStream_t st)
{
    if (!B.rank || !B.perm || B.N > kPairFarMaxN) return hipErrorInvalidValue;
    int NP = 1;
    while (NP < B.N) NP <<= 1;
    const size_t shmem = sizeof(unsigned long long) * (size_t)NP;
    // the limit is set once per device: for the largest sort (kPairFarMaxN keys, 128 KB)
    const hipError_t e = lds_limit_once((const void*)k_sort_sources,
                                        sizeof(unsigned long long) * (size_t)kPairFarMaxN, "k_sort_sources");
    if (e != hipSuccess) return e;
    launch_kernel(k_sort_sources, dim3(1), dim3(kSortThreads), (std::uint32_t)shmem, st, B.N, NP, x,
                  (int*)B.rank, (int*)B.perm);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_prep(StageBufs B, int cur, int M, int N, int K, const double* __restrict__ xin,
                                              const double* __restrict__ min_, const double* __restrict__ lam0sq,
                                              double t, double* __restrict__ xs, double* __restrict__ ys,
                                              double* __restrict__ lam2, double* __restrict__ alpha,
                                              double* __restrict__ alphaT, float* __restrict__ alphaT32,
                                              int* __restrict__ flag, int copy_state)
{
    const long total = (long)N * K;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        int j = (int)(idx / K), k = (int)(idx - (long)j * K);
        double l2 = lam0sq[j] + 4.0 * B.nuv[j] * __dadd_rn(t, B.toff[j]);
        double mk = min_[idx];
        const int sk = shell_of(k);
        double a = mk * inv_lambda_pow(l2, sk);
        if (copy_state) ys[idx] = mk;
        if (B.ystate[0]) {
            const int LP = 16 * ((M + 16) / 16), k2 = k - sk * (sk + 1) / 2;
            B.ystate[0][(long)j * LP * LP + (sk - k2) * LP + k2] = mk;
        }
        alpha[idx] = a;
        store_dense_alpha(B, cur, M, j, sk - (k - sk * (sk + 1) / 2), k - sk * (sk + 1) / 2, a);
        const int src = B.rank ? B.rank[j] : j;  // the pair kernels' source index
        if (alphaT) alphaT[(long)k * N + src] = a;
        if (alphaT32) alphaT32[(long)k * N + src] = (float)a;
        if (!isfinite(mk)) atomicOr(flag, 2);
        if (k == 0) {
            lam2[j] = l2;
            double x0 = xin[2 * j], x1 = xin[2 * j + 1];
            xs[2 * j] = x0;
            xs[2 * j + 1] = x1;
            if (B.rank) {
                B.lam2S[cur][src] = l2;
                B.xsS[2 * src] = x0;
                B.xsS[2 * src + 1] = x1;
            }
            if (B.interact && mk == 0.0) atomicOr(flag, 1);
            if (!isfinite(x0) || !isfinite(x1)) atomicOr(flag, 2);
        }
    }
}

hipError_t launch_prep(const DevTables& T, const StageBufs& B, int cur, const double* xin, const double* min_,
                       double t, bool need_pair, bool need_f32, hipStream_t st)
{
    if (B.rank) {
        const hipError_t e = launch_sort_sources(B, xin, st);
        if (e != hipSuccess) return e;
    }
    long total = (long)B.N * T.K;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    bool copy = (min_ != B.ys);
    launch_kernel(k_prep, dim3(blocks), dim3(256), 0, st, B, cur, T.M, B.N, T.K, xin, min_, B.lam0sq, t, B.xs,
                       B.ys, B.lam2[cur], B.alpha[cur], need_pair ? B.alphaT[cur] : (double*)nullptr,
                       need_pair && need_f32 ? B.alphaT32[cur] : (float*)nullptr, B.flag, copy ? 1 : 0);
    if (B.alphaD[0]) {  // zeros of the dense layouts (disjoint from what k_prep writes)
        const int LP = 16 * ((T.M + 16) / 16);
        long nz = (long)B.N * (LP + 16) * LP;
        int zb = (int)((nz + 255) / 256);
        if (zb > 4096) zb = 4096;
        launch_kernel(k_alpha_dense_clear, dim3(zb), dim3(256), 0, st, B, T.M);
    }
    return hipGetLastError();
}

// RK4 bookkeeping of one state component (moment or position coordinate):
// stage s contributes w_s * val to the accumulator; the next stage's input is
// y_n + c_{s+1} dt val, and the last stage writes y_{n+1} = y_n + dt * acc.
__device__ __forceinline__ double rk4_update(int stage, double dt, double* y, double* acc, double val)
{
    const double wts[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const double cn[3] = {0.5, 0.5, 1.0};
    const double yn = *y;
    if (stage == 0) *acc = wts[0] * val;
    else if (stage < 3) *acc += wts[stage] * val;
    if (stage < 3) return yn + cn[stage] * dt * val;
    const double ynew = yn + dt * (*acc + wts[3] * val);
    *y = ynew;
    return ynew;
}

// Emits dM^j_k/dt: RHS output, or the RK4 update plus the next stage's scaled
// moment (and its source-major copies for the pair kernel).
__device__ __forceinline__ void emit_moment(const StageBufs& B, const StageArgs& S, int M, int j, int k, int s,
                                            int K, double val, double lam2_next)
{
    const long o = (long)j * K + k;
    if (S.mode == MODE_RHS) {
        S.dmom[o] = val;
        return;
    }
    const double yn = rk4_update(S.stage, S.dt, S.mom + o, B.accm + o, val);
    B.ys[o] = yn;
    const int nx = 1 - S.cur;
    const double a = yn * inv_lambda_pow(lam2_next, s);
    B.alpha[nx][o] = a;
    if (B.alphaD[nx]) {
        const int k2 = k - s * (s + 1) / 2;
        store_dense_alpha(B, nx, M, j, s - k2, k2, a);
    }
    if (S.want_pair) {
        // FP64 always (the mixed path may run the FP64 pair kernel), FP32 for the mixed kernel
        const int src = B.rank ? B.rank[j] : j;
        B.alphaT[nx][(long)k * B.N + src] = a;
        if (S.want_f32) B.alphaT32[nx][(long)k * B.N + src] = (float)a;
    }
}

__device__ __forceinline__ void emit_position(const StageBufs& B, const StageArgs& S, int j, double xd1,
                                              double xd2, double lam2_next)
{
    if (S.mode == MODE_RHS) {
        S.dx[2 * j] = xd1;
        S.dx[2 * j + 1] = xd2;
        return;
    }
    const double x0 = rk4_update(S.stage, S.dt, S.x + 2 * j, B.accx + 2 * j, xd1);
    const double x1 = rk4_update(S.stage, S.dt, S.x + 2 * j + 1, B.accx + 2 * j + 1, xd2);
    B.xs[2 * j] = x0;
    B.xs[2 * j + 1] = x1;
    B.lam2[1 - S.cur][j] = lam2_next;
    if (B.rank) {
        const int src = B.rank[j];
        B.xsS[2 * src] = x0;
        B.xsS[2 * src + 1] = x1;
        B.lam2S[1 - S.cur][src] = lam2_next;
    }
}

// ---------------------------------------------------------------------------
// self velocity-derivative table: S_self[j][g] = sum_m alpha_m Psi0(m + g), c = 2
// (the target's own Gaussian convolved with itself: Lambda^2 = 2 lambda^2).
// Psi0 is nonzero only for even-even arguments.
// ---------------------------------------------------------------------------
hipError_t launch_self_pad(const DevTables& T, const StageBufs& B, int cur, hipStream_t st);

// Compensated accumulation (Ogita, Rump and Oishi's Dot2, extended to
// double-double operands): the running sum s carries a second word c that
// collects the exact rounding error of every product (TwoProd) and of every
// addition (TwoSum), plus the cross terms of the low words.  The result s + c
// is as accurate as a sum computed in twice the working precision, at about
// twelve operations per multiply-add (a double-double multiply-add costs
// about twenty-eight).
struct Acc2 {
    double s, c;
};

// acc += (xh + xl)(yh + yl), the xl yl term dropped
__device__ __forceinline__ void dot2(Acc2& a, double xh, double xl, double yh, double yl)
{
#pragma clang fp contract(off)
    const double p = xh * yh;
    double t = fma(xh, yh, -p);
    t = fma(xl, yh, t);
    t = fma(xh, yl, t);
    const double s = a.s + p;
    const double bb = s - a.s;
    const double es = (a.s - (s - bb)) + (p - bb);
    a.s = s;
    a.c += es + t;
}

// acc += x (yh + yl)
__device__ __forceinline__ void dot2(Acc2& a, double x, double yh, double yl)
{
#pragma clang fp contract(off)
    const double p = x * yh;
    double t = fma(x, yh, -p);
    t = fma(x, yl, t);
    const double s = a.s + p;
    const double bb = s - a.s;
    const double es = (a.s - (s - bb)) + (p - bb);
    a.s = s;
    a.c += es + t;
}

// a += b (two partial sums of one compensated sum)
__device__ __forceinline__ void acc2_merge(Acc2& a, const Acc2& b)
{
    const dd t = two_sum(a.s, b.s);
    a.s = t.hi;
    a.c += b.c + t.lo;
}

// the accumulated value as a normalised double-double
__device__ __forceinline__ dd acc2_value(const Acc2& a) { return two_sum(a.s, a.c); }

constexpr int kSelfVThreads = 256;  // workgroup size of k_self
constexpr int kSelfFillA = ((MMVM_MAX_ORDER + 1) * (MMVM_MAX_ORDER + 2) / 2 + kSelfVThreads - 1) / kSelfVThreads;
constexpr int kSelfT0NMax = (3 * MMVM_MAX_ORDER + 1) / 2 + 1;
constexpr int kSelfFillT = ((kSelfT0NMax + 1) * (kSelfT0NMax + 2) / 2 + kSelfVThreads - 1) / kSelfVThreads;

template <bool DD>
__global__ __launch_bounds__(kSelfVThreads) void k_self(int N, int M, int K, int GM, int KG, int T0N,
                                              const double* __restrict__ alpha, const double* __restrict__ t0h,
                                              const double* __restrict__ t0l, double* __restrict__ sself,
                                              double* __restrict__ sself_lo, DevClock* bump)
{
    // graph replay: the first kernel of a replayed step advances its clock (no
    // kernel of the step has read it yet; they all run after this one)
    if (bump && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) bump->n += 1;
    // LDS: alpha of the vortex [K] and the Psi0 table [tri(T0N)] (hi, lo).
    // Four lanes share one entry g, each summing every fourth even-step m2.
    extern __shared__ double sm_self[];
    const int nt0 = (T0N + 1) * (T0N + 2) / 2;
    double* sa = sm_self;
    double* th = sa + K;
    double* tl = th + nt0;
    const int j = blockIdx.y;
    const double* a = alpha + (long)j * K;
    {
        // every load is issued before the first LDS store (indices clamped
        // into the arrays; the stores past their ends are skipped)
        const int tid = threadIdx.x;
        double va[kSelfFillA], vh[kSelfFillT], vl[kSelfFillT];
#pragma unroll
        for (int u = 0; u < kSelfFillA; ++u) va[u] = a[min(tid + u * kSelfVThreads, K - 1)];
#pragma unroll
        for (int u = 0; u < kSelfFillT; ++u) {
            const int i = min(tid + u * kSelfVThreads, nt0 - 1);
            vh[u] = t0h[i];
            if constexpr (DD) vl[u] = t0l[i];
        }
#pragma unroll
        for (int u = 0; u < kSelfFillA; ++u)
            if (tid + u * kSelfVThreads < K) sa[tid + u * kSelfVThreads] = va[u];
#pragma unroll
        for (int u = 0; u < kSelfFillT; ++u) {
            const int i = tid + u * kSelfVThreads;
            if (i < nt0) {
                th[i] = vh[u];
                if constexpr (DD) tl[i] = vl[u];
            }
        }
    }
    __syncthreads();
    // four lanes share one entry g (eight for the compensated sums)
    constexpr int LANES = DD ? 8 : 4;
    const int gt = blockIdx.x * kSelfVThreads + threadIdx.x;
    const int g = gt / LANES, q = gt % LANES;
    const bool live = g < KG && g > 0;
    int g1 = 0, g2 = 0;
    if (live) {
        const int gs = shell_of(g);
        g2 = g - gs * (gs + 1) / 2;
        g1 = gs - g2;
    }
    if constexpr (!DD) {
        double acc = 0.0;
        if (live)
            for (int m2 = (g2 & 1) + 2 * q; m2 <= M; m2 += 8) {
                const int b2 = (m2 + g2) >> 1;
                for (int m1 = g1 & 1; m1 + m2 <= M; m1 += 2)
                    acc = fma(sa[ctri(m1, m2)], th[ctri((m1 + g1) >> 1, b2)], acc);
            }
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        if (q == 0 && g < KG) sself[(long)j * KG + g] = live ? acc : 0.0;
    } else {
        // compensated accumulation of alpha_m (Psi0_hi + Psi0_lo)
        Acc2 acc{0.0, 0.0};
        if (live)
            for (int m2 = (g2 & 1) + 2 * q; m2 <= M; m2 += 2 * LANES) {
                const int b2 = (m2 + g2) >> 1;
                for (int m1 = g1 & 1; m1 + m2 <= M; m1 += 2) {
                    const int ti = ctri((m1 + g1) >> 1, b2);
                    dot2(acc, sa[ctri(m1, m2)], th[ti], tl[ti]);
                }
            }
        for (int off = 1; off < LANES; off <<= 1) {
            const double os = __shfl_xor(acc.s, off, 64), oc = __shfl_xor(acc.c, off, 64);
            const dd t = two_sum(acc.s, os);
            acc.s = t.hi;
            acc.c += oc + t.lo;
        }
        if (q == 0 && g < KG) {
            const dd v = acc2_value(acc);
            sself[(long)j * KG + g] = live ? v.hi : 0.0;
            sself_lo[(long)j * KG + g] = live ? v.lo : 0.0;
        }
    }
}

hipError_t launch_self(const DevTables& T, const StageBufs& B, int cur, bool dd, hipStream_t st, DevClock* bump)
{
    if (stage2_uses_mfma(T.M, dd, !B.interact)) return bump ? hipErrorInvalidValue : launch_self_pad(T, B, cur, st);
    const int threads = kSelfVThreads;
    dim3 grid(((dd ? 8 : 4) * T.KG + threads - 1) / threads, B.N);
    const int nt0 = (T.T0N + 1) * (T.T0N + 2) / 2;
    // the fill covers at most kSelfFillA and kSelfFillT rounds of the workgroup
    if (T.K > kSelfFillA * threads || nt0 > kSelfFillT * threads) return hipErrorInvalidValue;
    size_t shmem = sizeof(double) * ((size_t)T.K + (dd ? 2 : 1) * (size_t)nt0);
    if (dd)
        launch_kernel(k_self<true>, grid, dim3(threads), shmem, st, B.N, T.M, T.K, T.GM, T.KG, T.T0N,
                           B.alpha[cur], T.t0_hi, T.t0_lo, B.s_self, B.s_self_lo, bump);
    else
        launch_kernel(k_self<false>, grid, dim3(threads), shmem, st, B.N, T.M, T.K, T.GM, T.KG, T.T0N,
                           B.alpha[cur], T.t0_hi, T.t0_lo, B.s_self, (double*)nullptr, bump);
    return hipGetLastError();
}

template <int M>
hipError_t launch_pair_M(const DevTables& T, const StageBufs& B, int cur, bool f32, PairShape sh, hipStream_t st);

bool pair_order_supported(int M) { return M >= 0 && M <= MMVM_MAX_PAIR_ORDER; }

hipError_t launch_pair_shape(const DevTables& T, const StageBufs& B, int cur, bool f32, PairShape sh, hipStream_t st)
{
    if (T.M > kMaxPairOrder) return launch_pair_gen(T, B, cur, st);  // any order, FP64
    switch (T.M) {
    case 0: return launch_pair_M<0>(T, B, cur, f32, sh, st);
    case 1: return launch_pair_M<1>(T, B, cur, f32, sh, st);
    case 2: return launch_pair_M<2>(T, B, cur, f32, sh, st);
    case 3: return launch_pair_M<3>(T, B, cur, f32, sh, st);
    case 4: return launch_pair_M<4>(T, B, cur, f32, sh, st);
    case 5: return launch_pair_M<5>(T, B, cur, f32, sh, st);
    case 6: return launch_pair_M<6>(T, B, cur, f32, sh, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pair(const DevTables& T, const StageBufs& B, int cur, bool f32, hipStream_t st, PairShape* used)
{
    if (T.M > kMaxPairOrder) {
        if (used) *used = PairShape();
        return launch_pair_gen(T, B, cur, st);
    }
    const PairShape sh = pair_shape_for(T, B, cur, f32, st);
    if (used) *used = sh;
    return launch_pair_shape(T, B, cur, f32, sh, st);
}

// The pair table joins the self table as the operand of the large-order stage
// 2 (interacting vortices): S = S_self + S_pair.
//   padded matrix-core layout: s_pad[j][par][g2][r] with g1 = par + 2r;
//   double-double layout: (s_self, s_self_lo) += s_pair, an exact two-sum plus
//   the low word.
__global__ __launch_bounds__(256) void k_pair_into_pad(StageBufs B, int GM, int KG, int KA, int RP)
{
    const long total = (long)B.N * KG;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int j = (int)(idx / KG), g = (int)(idx - (long)j * KG);
        if (g == 0) continue;
        const int gs = shell_of(g), g2 = g - gs * (gs + 1) / 2, g1 = gs - g2;
        double* o = B.s_pad + (((long)j * 2 + (g1 & 1)) * KA + g2) * RP + (g1 >> 1);
        *o += B.s_pair[idx];
    }
}

__global__ __launch_bounds__(256) void k_pair_into_dd(StageBufs B, int KG)
{
    const long total = (long)B.N * KG;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        if (idx - (idx / KG) * KG == 0) continue;
        const dd t = two_sum(B.s_self[idx], B.s_pair[idx]);
        const dd v = quick_two_sum(t.hi, t.lo + B.s_self_lo[idx]);
        B.s_self[idx] = v.hi;
        B.s_self_lo[idx] = v.lo;
    }
}

hipError_t launch_pair_into_stage2(const DevTables& T, const StageBufs& B, bool dd, hipStream_t st)
{
    const long total = (long)B.N * T.KG;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (dd) {
        if (!B.s_self_lo) return hipErrorInvalidValue;
        launch_kernel(k_pair_into_dd, dim3(blocks), dim3(256), 0, st, B, T.KG);
    } else {
        if (!B.s_pad) return hipErrorInvalidValue;
        const S2Shape sh(T.M, 0);
        launch_kernel(k_pair_into_pad, dim3(blocks), dim3(256), 0, st, B, T.GM, T.KG, sh.KA, sh.RP);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stage 2: the factorised contraction.
//   G_k = c1_k sum_l (-1)^{|l|} alpha_l sum_g [ -X[k1][l1][g1] Y[k2][l2][g2]
//                                              + Y[k1][l1][g1] X[k2][l2][g2] ] S[g]
// with X[k][l][k+l-2i-1] = f1[k][l][i] (Gamma^I's first-axis factor, paired with
// H_1 = -Psi(. + e2)) and Y[k][l][k+l-2i+1] = f0[k][l][i] (paired with
// H_2 = Psi(. + e1)); dM_k/dt = lambda^{|k|-2} G_k + drift.  For every k2 the
// second axis is contracted first (A), then l2 against the moments (B), then
// the first axis (C); the Y- and X- halves run as two passes to bound LDS.
// ---------------------------------------------------------------------------
struct ArithF64 {
    typedef double T;
    __device__ static T zero() { return 0.0; }
    __device__ static T ld(const double* h, const double*, long i) { return h[i]; }
    __device__ static T mk(double v) { return v; }
    __device__ static T madd(T acc, T a, T b) { return fma(a, b, acc); }
    __device__ static T add(T a, T b) { return a + b; }
    __device__ static T neg(T a) { return -a; }
    __device__ static double hi(T a) { return a; }
    __device__ static void st(double* p, T a) { p[0] = a; p[1] = 0.0; }
    __device__ static T ldst(const double* p) { return p[0]; }
};
struct ArithDD {
    typedef dd T;
    __device__ static T zero() { return dd_make(0.0); }
    __device__ static T ld(const double* h, const double* l, long i) { return dd_make(h[i], l[i]); }
    __device__ static T mk(double v) { return dd_make(v); }
    __device__ static T madd(T acc, T a, T b) { return dd_add(acc, dd_mul(a, b)); }
    __device__ static T add(T a, T b) { return dd_add(a, b); }
    __device__ static T neg(T a) { return dd_neg(a); }
    __device__ static double hi(T a) { return a.hi + a.lo; }
    __device__ static void st(double* p, T a) { p[0] = a.hi; p[1] = a.lo; }
    __device__ static T ldst(const double* p) { return dd_make(p[0], p[1]); }
};

// centre velocity (eq:xjdot_Final) from the pair table, block-wide:
//   xdot_1 = -(1/(Gamma lambda)) sum_m (-1)^{|m|} alpha_m S_pair[m + e2]
//   xdot_2 = +(1/(Gamma lambda)) sum_m (-1)^{|m|} alpha_m S_pair[m + e1]
__device__ void centre_velocity(const double* al, const double* sp, int K, double lam, double* red, double& xd1,
                                double& xd2)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    double p1 = 0.0, p2 = 0.0;
    for (int m = tid; m < K; m += nt) {
        int s = shell_of(m);
        int m2 = m - s * (s + 1) / 2, m1 = s - m2;
        double a = (s & 1) ? -al[m] : al[m];
        p1 += a * sp[ctri(m1, m2 + 1)];
        p2 += a * sp[ctri(m1 + 1, m2)];
    }
    for (int off = 32; off > 0; off >>= 1) {
        p1 += __shfl_xor(p1, off, 64);
        p2 += __shfl_xor(p2, off, 64);
    }
    if ((tid & 63) == 0) {
        red[(tid >> 6) * 2] = p1;
        red[(tid >> 6) * 2 + 1] = p2;
    }
    __syncthreads();
    p1 = p2 = 0.0;
    for (int w = 0; w < (nt + 63) / 64; ++w) {
        p1 += red[2 * w];
        p2 += red[2 * w + 1];
    }
    const double gam = al[0];
    xd1 = -p1 / (gam * lam);
    xd2 = p2 / (gam * lam);
}

// ---------------------------------------------------------------------------
// Large orders on the strict FP64 path (above the double-double threshold).
// The contraction's alternating sums cancel, so every sum is accumulated in a
// compensated form (Acc2 / dot2 above), with double-double operands and
// results.
// ---------------------------------------------------------------------------
// LDS layout of the double-double stage 2 (doubles; double-double values as
// (hi, lo) pairs).  Rows r of the velocity-derivative table hold g1 = par + 2r
// with g2 = 0 .. GM - g1 (row-packed); step B overwrites it with T.
// With ctab (one workgroup per CU, 134.8 KB at order 40) the second-axis factor
// slice is a full [M+1][M+1] rectangle and step C's binomials and first-axis
// diagonals are staged in LDS too; without (two workgroups per CU, 79.4 KB),
// the slice keeps only its band i <= min(l2, k2) and step C reads its tables
// from L2.
struct DDShape {
    int M1, nrp;
    int s, f, y, ar, bin, fd, total;
    __host__ __device__ DDShape(int M, int par, bool ctab)
    {
        M1 = M + 1;
        nrp = (2 * M - par) / 2 + 1;
        const int m2 = M1 * M1;
        s = 0;                      // S, then T: nrp * M1 <= M1^2 pairs
        f = s + 2 * m2;             // f[k2][l2][i]: [M1][M1] pairs (ctab), else its band i <= min(l2, k2)
        y = f + (ctab ? 2 * m2 : M1 * (M1 + 1));  // Y, then the partials of step C: [M1][M1] pairs
        ar = y + 2 * m2;            // (-1)^{|l|} alpha at (l1, l2), zero beyond the triangle: [M1 + 1][M1]
        bin = ar + (M1 + 1) * M1;   // C(l, i): [M1][M1] (ctab)
        fd = bin + (ctab ? m2 : 0);  // f[k1][i][i] of the first axis: [M1][M1] pairs (ctab)
        total = fd + (ctab ? 2 * m2 : 0);
    }
    // start of row r (in pairs): rows have GM - par - 2r + 1 entries
    __host__ __device__ static int row_off(int M, int par, int r) { return r * (2 * M - par + 1) - r * (r - 1); }
    // start of row l2 of the factor band (in pairs): rows have min(l2, k2) + 1 entries
    __host__ __device__ static int band_off(int k2, int l2)
    {
        return l2 <= k2 + 1 ? l2 * (l2 + 1) / 2 : (k2 + 1) * (k2 + 2) / 2 + (l2 - k2 - 1) * (k2 + 1);
    }
};

constexpr int kDDThreads = 1024;
constexpr int kDDOneRound = 256;  // compute units of an MI355X
// task-list entries per thread: steps A (rows x l2 <= (M+1)^2) and C (k1 x l1 slots)
constexpr int kDDTA = ((MMVM_MAX_ORDER + 1) * (MMVM_MAX_ORDER + 1) + kDDThreads - 1) / kDDThreads;
constexpr int kDDTC = ((MMVM_MAX_ORDER + 1) * ((MMVM_MAX_ORDER + 2) / 2) + kDDThreads - 1) / kDDThreads;

// blockIdx.x = (k2, pass, par): pass 0 = Y half (f0 on the second axis, f1 on
// the first, minus sign), pass 1 = X half; par = parity of the rows g1 this
// workgroup owns (step C of (k1, l1) reads rows of parity k1 + l1 + 1 only).
// Each workgroup writes its partial sum over l1 for every k1 of its k2; the
// emit kernel adds the four partials.  Single vortices only (the interacting
// path stops far below the double-double orders).
template <bool CTAB>
__global__ __launch_bounds__(kDDThreads) void k_stage2_dd(DevTables T, StageBufs B, StageArgs S)
{
    const int M = T.M, K = T.K, GM = T.GM, M1 = M + 1;
    const int j = blockIdx.y;
    const int k2 = blockIdx.x >> 2, pass = (blockIdx.x >> 1) & 1, par = blockIdx.x & 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    const DDShape L(M, par, CTAB);
    const int nrp = L.nrp;
    extern __shared__ double smem[];
    double* sS = smem + L.s;
    double* sF = smem + L.f;
    double* sY = smem + L.y;
    double* sAR = smem + L.ar;
    double* sBin = smem + L.bin;
    double* sFd = smem + L.fd;

    // this workgroup's task lists of steps A and C (longest sums first)
    const int H = (M1 + 1) >> 1;
    const int* la = T.dd_la + (long)blockIdx.x * M1 * M1;
    const int* lc = T.dd_lc + (long)blockIdx.x * M1 * H;
    int codeA[kDDTA], codeC[kDDTC];
    // fills: S rows of parity par, the band of the second-axis factor slice
    // and signed alpha.  Every global load of a thread is issued before its
    // first LDS store (clamped addresses, zeros selected afterwards), so the
    // fill costs about one L2 round trip.
    {
        constexpr int MM1 = MMVM_MAX_ORDER + 1;
        constexpr int NS = (MM1 * (2 * MMVM_MAX_ORDER + 1) + kDDThreads - 1) / kDDThreads;
        constexpr int NQ = (MM1 * MM1 + kDDThreads - 1) / kDDThreads;
        constexpr int NA = ((MM1 + 1) * MM1 + kDDThreads - 1) / kDDThreads;
        const double* ssh = B.s_self + (long)j * T.KG;
        const double* ssl = B.s_self_lo + (long)j * T.KG;
        const double* fh = (pass == 0 ? T.f0_hi : T.f1_hi) + (long)k2 * M1 * M1;
        const double* fl = (pass == 0 ? T.f0_lo : T.f1_lo) + (long)k2 * M1 * M1;
        const double* al = B.alpha[S.cur] + (long)j * K;
        const double* dh = pass == 0 ? T.fd1 : T.fd0;
        const double* dl = pass == 0 ? T.fd1_lo : T.fd0_lo;
        const int nS = nrp * (GM + 1), nQ = M1 * M1, nA = (M1 + 1) * M1;
        double vsh[NS], vsl[NS], vfh[NQ], vfl[NQ], va[NA];
        double vbn[CTAB ? NQ : 1], vdh[CTAB ? NQ : 1], vdl[CTAB ? NQ : 1];
#pragma unroll
        for (int u = 0; u < kDDTA; ++u) codeA[u] = la[min(tid + u * kDDThreads, M1 * M1 - 1)];
#pragma unroll
        for (int u = 0; u < kDDTC; ++u) codeC[u] = lc[min(tid + u * kDDThreads, M1 * H - 1)];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int e = tid + u * kDDThreads;
            const int r = e / (GM + 1), g2 = e - r * (GM + 1);
            const int g1 = par + 2 * r;
            const int g = (e < nS && g1 + g2 <= GM) ? ctri(g1, g2) : 0;
            vsh[u] = ssh[g];
            vsl[u] = ssl[g];
        }
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int e = tid + u * kDDThreads;
            const int ec = e < nQ ? e : 0;
            vfh[u] = fh[ec];
            vfl[u] = fl[ec];
            if constexpr (CTAB) {
                vbn[u] = T.binom[ec];
                vdh[u] = dh[ec];
                vdl[u] = dl[ec];
            }
        }
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + u * kDDThreads;
            const int l1 = e / M1, l2 = e - l1 * M1;
            va[u] = al[(e < nA && l1 + l2 <= M) ? ctri(l1, l2) : 0];
        }
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int e = tid + u * kDDThreads;
            const int r = e / (GM + 1), g2 = e - r * (GM + 1);
            const int g1 = par + 2 * r;
            if (e < nS && g1 + g2 <= GM) {
                const int o = DDShape::row_off(M, par, r) + g2;
                const bool z = g1 + g2 == 0;
                sS[2 * o] = z ? 0.0 : vsh[u];
                sS[2 * o + 1] = z ? 0.0 : vsl[u];
            }
        }
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int e = tid + u * kDDThreads;
            const int l2 = e / M1, i = e - l2 * M1;
            if (e < nQ && (CTAB || (i <= l2 && i <= k2))) {
                const int o = CTAB ? e : DDShape::band_off(k2, l2) + i;
                sF[2 * o] = vfh[u];
                sF[2 * o + 1] = vfl[u];
            }
            if constexpr (CTAB) {
                if (e < nQ) {
                    sBin[e] = vbn[u];
                    sFd[2 * e] = vdh[u];
                    sFd[2 * e + 1] = vdl[u];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + u * kDDThreads;
            const int l1 = e / M1, l2 = e - l1 * M1;
            if (e < nA) sAR[e] = l1 + l2 <= M ? (((l1 + l2) & 1) ? -va[u] : va[u]) : 0.0;
        }
    }
    __syncthreads();
    // (A) second axis: Y[r][l2] = sum_i f[k2][l2][i] S[g1][k2 + l2 - 2i +- 1]
    // over the i whose g2 stays inside row g1 (lanes over rows)
    {
        const int off = pass == 0 ? 1 : -1;
#pragma unroll
        for (int u = 0; u < kDDTA; ++u) {
            if (tid + u * kDDThreads >= M1 * nrp) break;
            const int r = codeA[u] >> 8, l2 = codeA[u] & 255;
            const int g1 = par + 2 * r;
            const int imax = pass == 0 ? (l2 < k2 ? l2 : k2) : (l2 < k2 - 1 ? l2 : k2 - 1);
            const int over = k2 + l2 + off + g1 - GM;  // g2 <= GM - g1  <=>  2i >= over
            const int ilo = over > 0 ? (over + 1) >> 1 : 0;
            const double* fr = sF + 2 * (CTAB ? l2 * M1 : DDShape::band_off(k2, l2));
            const double* sr = sS + 2 * (DDShape::row_off(M, par, r) + k2 + l2 + off);
            // two independent chains (even and odd i) keep more loads in flight
            Acc2 a{0.0, 0.0}, b{0.0, 0.0};
            int i = ilo;
            for (; i < imax; i += 2) {
                dot2(a, fr[2 * i], fr[2 * i + 1], sr[-4 * i], sr[-4 * i + 1]);
                dot2(b, fr[2 * i + 2], fr[2 * i + 3], sr[-4 * i - 4], sr[-4 * i - 3]);
            }
            if (i == imax) dot2(a, fr[2 * i], fr[2 * i + 1], sr[-4 * i], sr[-4 * i + 1]);
            acc2_merge(a, b);
            const dd v = acc2_value(a);
            sY[2 * (r * M1 + l2)] = v.hi;
            sY[2 * (r * M1 + l2) + 1] = v.lo;
        }
    }
    __syncthreads();
    // (B) T[r][l1] = sum_{l2 <= M - l1} (-1)^{|l|} alpha_l Y[r][l2], two l1 per thread
    {
        const int npair = (M1 + 1) >> 1;
        for (int task = tid; task < npair * nrp; task += nt) {
            const int q = task / nrp, r = task - q * nrp;
            const int l1 = 2 * q;
            const double* yr = sY + 2 * (r * M1);
            const double* a0 = sAR + l1 * M1;
            const double* a1 = a0 + M1;  // zero where l1 + 1 + l2 > M (a zero row past M)
            // even and odd l2 in separate chains
            Acc2 u{0.0, 0.0}, v{0.0, 0.0}, u1{0.0, 0.0}, v1{0.0, 0.0};
            int l2 = 0;
            for (; l2 < M - l1; l2 += 2) {
                const double yh = yr[2 * l2], yl = yr[2 * l2 + 1];
                const double zh = yr[2 * l2 + 2], zl = yr[2 * l2 + 3];
                dot2(u, a0[l2], yh, yl);
                dot2(v, a1[l2], yh, yl);
                dot2(u1, a0[l2 + 1], zh, zl);
                dot2(v1, a1[l2 + 1], zh, zl);
            }
            if (l2 == M - l1) {
                const double yh = yr[2 * l2], yl = yr[2 * l2 + 1];
                dot2(u, a0[l2], yh, yl);
                dot2(v, a1[l2], yh, yl);
            }
            acc2_merge(u, u1);
            acc2_merge(v, v1);
            const dd tu = acc2_value(u), tv = acc2_value(v);
            sS[2 * (r * M1 + l1)] = tu.hi;
            sS[2 * (r * M1 + l1) + 1] = tu.lo;
            if (l1 + 1 <= M) {
                sS[2 * (r * M1 + l1 + 1)] = tv.hi;
                sS[2 * (r * M1 + l1 + 1) + 1] = tv.lo;
            }
        }
    }
    __syncthreads();
    // (C) first axis for the (k1, l1) whose rows have parity par:
    //   pass 0: - sum_i f1[k1][l1][i] T[k1 + l1 - 2i - 1][l1]
    //   pass 1: + sum_i f0[k1][l1][i] T[k1 + l1 - 2i + 1][l1]
    // with f[k1][l1][i] = C(l1, i) f[k1][i][i]; one task per (k1, l1 of that parity)
    const int nk1 = M - k2 + 1;
#pragma unroll
    for (int u = 0; u < kDDTC; ++u) {
        if (tid + u * kDDThreads >= nk1 * H) break;
        const int k1 = codeC[u] >> 8, q = codeC[u] & 255;
        const int task = k1 * H + q;
        const int l1 = 2 * q + ((par + k1 + 1) & 1);
        if (l1 > M) {
            sY[2 * task] = 0.0;
            sY[2 * task + 1] = 0.0;
            continue;
        }
        // binomials and diagonals: LDS (CTAB) or the L2-resident tables
        Acc2 a{0.0, 0.0};
        const double* bn = (CTAB ? sBin : T.binom) + l1 * M1;
        const double* fdh;
        const double* fdl;
        int fs;  // stride between hi and lo words, and between entries
        if constexpr (CTAB) {
            fdh = sFd + 2 * (k1 * M1);
            fdl = fdh + 1;
            fs = 2;
        } else {
            fdh = (pass == 0 ? T.fd1 : T.fd0) + k1 * M1;
            fdl = (pass == 0 ? T.fd1_lo : T.fd0_lo) + k1 * M1;
            fs = 1;
        }
        if (pass == 0) {
            const int imax = l1 < k1 - 1 ? l1 : k1 - 1;
            // unrolled: the table loads of two terms issue together (same order of sums)
#pragma unroll 2
            for (int i = 0; i <= imax; ++i) {
                const int r = (k1 + l1 - 2 * i - 1 - par) >> 1;
                const dd f = dd_mul_d(dd_make(fdh[fs * i], fdl[fs * i]), bn[i]);
                dot2(a, f.hi, f.lo, sS[2 * (r * M1 + l1)], sS[2 * (r * M1 + l1) + 1]);
            }
            a.s = -a.s;
            a.c = -a.c;
        } else {
            const int imax = l1 < k1 ? l1 : k1;
            const int i0 = k1 + l1 + 1 > GM ? 1 : 0;
#pragma unroll 2
            for (int i = i0; i <= imax; ++i) {
                const int r = (k1 + l1 - 2 * i + 1 - par) >> 1;
                const dd f = dd_mul_d(dd_make(fdh[fs * i], fdl[fs * i]), bn[i]);
                dot2(a, f.hi, f.lo, sS[2 * (r * M1 + l1)], sS[2 * (r * M1 + l1) + 1]);
            }
        }
        const dd v = acc2_value(a);
        sY[2 * task] = v.hi;
        sY[2 * task + 1] = v.lo;
    }
    __syncthreads();
    // partial over l1 for every k1 of this k2 -> global (hi, lo)
    double* gp = B.gpart + ((long)j * 4 + (pass * 2 + par)) * K * 2;
    for (int k1 = tid; k1 < nk1; k1 += nt) {
        Acc2 a{0.0, 0.0};
        for (int q = 0; q < H; ++q) dot2(a, 1.0, sY[2 * (k1 * H + q)], sY[2 * (k1 * H + q) + 1]);
        const dd g = acc2_value(a);
        const int k = ctri(k1, k2);
        gp[2 * k] = g.hi;
        gp[2 * k + 1] = g.lo;
    }
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// A strided LDS matrix: element (i, j) at p[i * rs + j * cs].
struct View {
    const double* p;
    int rs, cs;
};

// One 16x16 output tile over the k-steps [s0, s1) (s1 - s0 <= KS).  Lane l
// supplies A[row0 + l%16][4s + l/16] and B[4s + l/16][col0 + l%16]; it receives
// D[row0 + l/16 + 4q][col0 + l%16] in component q.  All operands are loaded
// first, then two accumulator chains alternate k-steps.
template <int KS>
struct TileOps {
    double a[KS], b[KS];
    int s0, s1;
};

template <int KS>
__device__ __forceinline__ void tile_load(TileOps<KS>& o, int lane, int row0, int col0, int s0, int s1, const View& A,
                                          const View& B)
{
    const int lk = lane >> 4;
    const double* pa = A.p + (row0 + (lane & 15)) * A.rs + (4 * s0 + lk) * A.cs;
    const double* pb = B.p + (4 * s0 + lk) * B.rs + (col0 + (lane & 15)) * B.cs;
    const int sa = 4 * A.cs, sb = 4 * B.rs;
#pragma unroll
    for (int q = 0; q < KS; ++q) {
        if (s0 + q < s1) {
            o.a[q] = pa[q * sa];
            o.b[q] = pb[q * sb];
        } else {
            o.a[q] = 0.0;
            o.b[q] = 0.0;
        }
    }
    o.s0 = s0;
    o.s1 = s1;
}

template <int KS>
__device__ __forceinline__ dbl4 tile_mfma(const TileOps<KS>& o)
{
    dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < KS; ++q) {
        if (o.s0 + q < o.s1) {
            if (q & 1) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(o.a[q], o.b[q], acc1, 0, 0, 0);
            else acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(o.a[q], o.b[q], acc0, 0, 0, 0);
        }
    }
    return acc0 + acc1;
}

template <int KS>
__device__ __forceinline__ dbl4 mfma_tile(int lane, int row0, int col0, int s0, int s1, const View& A, const View& B)
{
    TileOps<KS> o;
    tile_load(o, lane, row0, col0, s0, s1, A, B);
    return tile_mfma(o);
}

// largest order of the matrix-core stage 2 and the per-wavefront bounds it implies
constexpr int kS2KA = ((2 * kS2MaxOrder) >> 2) + 1;        // k-steps of (A)
constexpr int kS2KB = kS2MaxOrder / 4 + 1;                 // k-steps of (B) and (C)
// k-steps of an (A) tile in the third row of tiles (g1 >= 64, so g2 <= 2 kS2MaxOrder - 64)
constexpr int kS2KA3 = ((2 * kS2MaxOrder - 64) >> 2) + 1;
static_assert(kS2Waves == 8 && 16 * ((kS2MaxOrder + 16) / 16) <= 48, "at most nine (A) tiles, three by three");
// k-steps of a (B) tile in the third column of tiles (l1 >= 32, so l2 <= kS2MaxOrder - 32)
constexpr int kS2KB3 = (kS2MaxOrder - 32) / 4 + 1;
// output tiles of (C) per wavefront: d over 2 (M - k2) + 1 <= 2 M + 1 rows, i over M + 1 columns
constexpr int kS2TilesC = (((2 * kS2MaxOrder + 1 + 15) / 16) * ((kS2MaxOrder + 1 + 15) / 16) + kS2Waves - 1) / kS2Waves;
static_assert(kS2MaxOrder < 64, "one lane per k1 in the last step");
static_assert(MMVM_MAX_ORDER <= kS2MaxOrder, "order");

__host__ __device__ inline int s2m_lds_doubles(int M)
{
    const S2Shape a(M, 0), b(M, 1);
    return a.total > b.total ? a.total : b.total;
}

bool mfma_order(int M) { return M >= kMinMfmaOrder && M <= kS2MaxOrder; }
bool stage2_uses_mfma(int M, bool dd, bool solo)
{
    return !dd && mfma_order(M) && (M > kMaxSmallOrder || solo);
}

// ---------------------------------------------------------------------------
// Large orders, FP64, on the matrix cores.  Same workgroup split as the
// double-double kernel; the three steps become products of zero-padded
// operands staged in LDS, computed with v_mfma_f64_16x16x4f64 (per wavefront
// D[16x16] += A[16x4] B[4x16]):
//   (A)  Y[r][l2]  = sum_{g2} S[g1(r)][g2] W[g2][l2],  W[g2][l2] = F[k2][l2][i]
//        at g2 = k2 + l2 - 2i +- 1 (the factor slice of this k2);
//   (B)  T[r][l1]  = sum_{l2} Y[r][l2] (-1)^{|l|} alpha[l1, l2]  (l1 + l2 <= M);
//   (C)  with F'[k1][l1][i] = C(l1, i) F'[k1][i][i]:
//        U[d][i]   = sum_{l1} T[d + l1][l1] C(l1, i),
//        G[k1]     = -+ sum_i F'[k1][i][i] U[k1 - 2i -+ 1][i].
// Rows r index g1 = par + 2r (the rows of this workgroup's parity).  The self
// kernel writes S zero-padded and by columns (the 16 rows of an operand
// fragment are one cache line), and W and C come padded from the tables, so
// the operands are read in place.  Every output tile runs
// only over the k-steps where its band of W, the triangle of alpha or the
// triangle of C is nonzero.  T is stored by (g1, l1) with zero rows for the
// other parity and kS2TPad zero rows on either side, so that the sheared
// operand of (C) is the strided view (d, l1) -> T[d + l1][l1].
// One vortex per workgroup row of the grid (no pair table).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kS2Threads) void k_stage2_mfma(DevTables T, StageBufs B, StageArgs S)
{
    const int M = T.M, GM = T.GM, M1 = M + 1;
    const int j = blockIdx.y;
    const int k2 = blockIdx.x >> 2, pass = (blockIdx.x >> 1) & 1, par = blockIdx.x & 1;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: tile loops branch on scalars
    const S2Shape sh(M, par);
    const int nrp = sh.nrp, LP = sh.LP, KA = sh.KA;
    const int nk1 = M - k2 + 1;
    const int dlo = k2 - M + 1;           // step C: d = g1 - l1 in [dlo, dlo + nd)
    const int nd = 2 * (M - k2) + 1;
    const int ni = M - k2 + 1;
    const int off2 = pass == 0 ? 1 : -1;
    const int imaxk = pass == 0 ? k2 : k2 - 1;

    // Operands read straight from global memory (L2-resident, rows contiguous;
    // every tile issues all its loads before its first product): the padded
    // self-table rows of this parity, the banded factor operand of this (k2,
    // pass), the signed moments and the padded binomials.  LDS holds only what
    // the products pass to each other.
    extern __shared__ double smem[];
    double* sT = smem + sh.t;             // T [NTR][LDT]                  (B -> C)
    double* sY = smem + sh.y;             // Y [RP][LDY]                   (A -> B)
    double* sU = smem + sh.y;             // U [nd][ni], over Y            (C -> last step)
    double* sP = smem + sh.ps;            // partial sums of the last step [8][64]
    const double* gS = B.s_pad + ((long)j * 2 + par) * sh.RP * sh.KA;  // column-major: 16 rows = one line
    const double* gW = T.wpad + ((long)k2 * 2 + pass) * KA * LP;
    const double* gA = B.alphaS[S.cur] + (long)j * LP * LP;
    const double* gD = pass == 0 ? T.fd1 : T.fd0;
    // graph replay: the last stage of the captured steps advances the clock
    // (every reader of it, a self kernel, has finished; the next one starts after)
    if (S.clock_bump && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) S.clock_bump->n += S.clock_steps;

    // T is zero except the rows of this parity written after (B)
    {
        double2* dT = reinterpret_cast<double2*>(sT);
        const double2 z2 = {0.0, 0.0};
        for (int e = tid; e < sh.NTR * sh.LDT / 2; e += kS2Threads) dT[e] = z2;
        if (tid == 0 && ((sh.NTR * sh.LDT) & 1)) sT[sh.NTR * sh.LDT - 1] = 0.0;
    }
    const int tr = sh.RP >> 4, tc = LP >> 4;
    // (A)
    {
        const View va = {gS, 1, sh.RP}, vb = {gW, LP, 1};
        // the k-steps of tile t: W[.][l2] is nonzero for g2 in [lo(l2), k2 + l2 + off2],
        // lo = 1 + |l2 - k2| (pass 0), |l2 - k2 + 1| (pass 1); row r0 ends at g2 = GM - par - 2 r0
        auto krange = [&](int t, int& r0, int& c0, int& s0, int& s1) {
            r0 = (t / tc) * 16;
            c0 = (t % tc) * 16;
            const int lhi = c0 + 15 < M ? c0 + 15 : M;
            const int dist = imaxk < c0 ? c0 - imaxk : (imaxk > lhi ? imaxk - lhi : 0);
            const int glo = (pass == 0 ? 1 : 0) + dist;
            int ghi = k2 + off2 + lhi;
            if (ghi > GM - par - 2 * r0) ghi = GM - par - 2 * r0;
            s0 = glo >> 2;
            s1 = (c0 <= M && glo <= ghi) ? (ghi >> 2) + 1 : s0;
        };
        auto put = [&](int r0, int c0, const dbl4& d) {
#pragma unroll
            for (int q = 0; q < 4; ++q) sY[(r0 + (lane >> 4) + 4 * q) * sh.LDY + c0 + (lane & 15)] = d[q];
        };
        if (tr * tc <= kS2Waves || wave < kS2Waves - 2) {
            // a tile per wavefront (the first six of nine)
            if (wave < tr * tc) {
                int r0, c0, s0, s1;
                krange(wave, r0, c0, s0, s1);
                put(r0, c0, mfma_tile<kS2KA>(lane, r0, c0, s0, s1, va, vb));
            }
        } else {
            // nine tiles (orders 32 and up): the last row of tiles (rows g1 >= 64,
            // where S is nonzero for g2 <= GM - 64 only) has at most kS2KA3
            // k-steps a tile.  Wavefront 6 takes tiles 6 and 8, with the operands
            // of both loaded first; wavefront 7 takes tile 7.
            TileOps<kS2KA3> o[2];
            int r0[2], c0[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                int s0, s1;
                krange(wave + 2 * u, r0[u], c0[u], s0, s1);
                if (u == 1 && wave != kS2Waves - 2) s1 = s0;
                tile_load(o[u], lane, r0[u], c0[u], s0, s1, va, vb);
            }
            put(r0[0], c0[0], tile_mfma(o[0]));
            if (wave == kS2Waves - 2) put(r0[1], c0[1], tile_mfma(o[1]));
        }
    }
    __syncthreads();
    // (B) T[r][l1] = sum_{l2} Y[r][l2] (-1)^{|l|} alpha[l1, l2]
    {
        const View va = {sY, sh.LDY, 1}, vb = {gA, LP, 1};
        auto put = [&](int t, const dbl4& d) {
            const int r0 = (t / tc) * 16, c0 = (t % tc) * 16;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int r = r0 + (lane >> 4) + 4 * u, l1 = c0 + (lane & 15);
                if (r < nrp) sT[(par + 2 * r + kS2TPad) * sh.LDT + l1] = d[u];
            }
        };
        // l2 <= M - l1 < M - c0 + 1
        auto steps = [&](int t) {
            const int c0 = (t % tc) * 16;
            return c0 <= M ? (M - c0) / 4 + 1 : 0;
        };
        if (tr * tc <= kS2Waves) {
            if (wave < tr * tc) put(wave, mfma_tile<kS2KB>(lane, (wave / tc) * 16, (wave % tc) * 16, 0, steps(wave), va, vb));
        } else if (wave < kS2Waves - 2) {
            // nine tiles: wavefronts 0..5 take the first two columns of tiles
            const int t = (wave >> 1) * 3 + (wave & 1);
            put(t, mfma_tile<kS2KB>(lane, (t / tc) * 16, (t % tc) * 16, 0, steps(t), va, vb));
        } else {
            // the third column (l1 >= 32) has at most kS2KB3 k-steps a tile:
            // wavefront 6 takes tiles 2 and 8 (the operands of both loaded
            // first), wavefront 7 takes tile 5
            const int ta = wave == kS2Waves - 2 ? 2 : 5;
            TileOps<kS2KB3> o[2];
            tile_load(o[0], lane, (ta / tc) * 16, (ta % tc) * 16, 0, steps(ta), va, vb);
            tile_load(o[1], lane, 32, 32, 0, wave == kS2Waves - 2 ? steps(8) : 0, va, vb);
            put(ta, tile_mfma(o[0]));
            if (wave == kS2Waves - 2) put(8, tile_mfma(o[1]));
        }
    }
    __syncthreads();
    // (C) U = T(sheared) x C; U overwrites Y, whose last reads preceded the barrier
    {
        // a wavefront takes tiles wave, wave + 8, ...; the operands of its next
        // tile load while the current one multiplies (two register buffers)
        const int td = (nd + 15) >> 4, ti = (ni + 15) >> 4, ntc = td * ti;
        const View va = {sT + (dlo + kS2TPad) * sh.LDT, sh.LDT, sh.LDT + 1}, vb = {T.cpad, LP, 1};
        TileOps<kS2KB> op[2];
        int r0[kS2TilesC], c0[kS2TilesC];
#pragma unroll
        for (int u = 0; u < kS2TilesC; ++u) {
            const int t = wave + u * kS2Waves;
            r0[u] = (t / ti) * 16;
            c0[u] = (t % ti) * 16;
        }
        // l1 >= i >= c0 and 0 <= d + l1 <= GM; no k-steps past the tiles of this wavefront
        auto load = [&](int u) {
            int llo = -(dlo + r0[u] + 15);
            if (llo < c0[u]) llo = c0[u];
            int lhi = GM - (dlo + r0[u]);
            if (lhi > M) lhi = M;
            const int s0 = llo >> 2;
            const int s1 = (wave + u * kS2Waves < ntc && llo <= lhi) ? (lhi >> 2) + 1 : s0;
            tile_load(op[u & 1], lane, r0[u], c0[u], s0, s1, va, vb);
        };
        load(0);
#pragma unroll
        for (int u = 0; u < kS2TilesC; ++u) {
            if (u + 1 < kS2TilesC) load(u + 1);
            const dbl4 d = tile_mfma(op[u & 1]);
            if (wave + u * kS2Waves < ntc) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int di = r0[u] + (lane >> 4) + 4 * q, i = c0[u] + (lane & 15);
                    if (di < nd && i < ni) sU[di * ni + i] = d[q];
                }
            }
        }
    }
    __syncthreads();
    // G[k1] = -+ sum_i F'[k1][i][i] U[k1 - 2i -+ 1][i]: lane = k1, wavefront w takes i = w mod 8
    {
        const int k1 = lane;
        double v = 0.0;
        if (k1 < nk1) {
            const int imax = pass == 0 ? k1 - 1 : k1;
            for (int i = wave; i <= imax; i += kS2Waves) {
                const int d = pass == 0 ? k1 - 2 * i - 1 : k1 - 2 * i + 1;
                v = fma(gD[k1 * M1 + i], sU[(d - dlo) * ni + i], v);
            }
        }
        sP[wave * 64 + lane] = v;
    }
    __syncthreads();
    if (tid < nk1) {  // partial G[k1 = tid][k2] of this (pass, parity), dense layout
        double g = 0.0;
        for (int w = 0; w < kS2Waves; ++w) g += sP[w * 64 + tid];
        B.gpartD[((long)j * 4 + (pass * 2 + par)) * LP * LP + tid * LP + k2] = pass == 0 ? -g : g;
    }
}

// ---------------------------------------------------------------------------
// Self velocity-derivative table of the matrix-core path, written zero-padded
// by columns for each parity: s_pad[j][par][c][r] = S_self[g1 = par + 2r][g2 = c]
// (zero beyond the triangle and at g = 0).  Workgroup = (row r, parity, vortex).
// With Psi0(2a, 2b) = t0[a][b] and m1 of the parity of g1 (m1 = p1 + 2 m1'):
//   Q[m2][b]  = sum_{m1'} alpha[p1 + 2 m1'][m2] t0[m1' + ceil(g1 / 2)][b]   (matrix cores)
//   S[g1][g2] = sum_{m2 = g2 mod 2} Q[m2][(m2 + g2) / 2].
// ---------------------------------------------------------------------------
constexpr int kSelfThreads = 512;
constexpr int kSelfWaves = kSelfThreads / 64;
template <bool APPLY>
__global__ __launch_bounds__(kSelfThreads) void k_self_mfma(DevTables T, StageBufs B, int cur, ApplyArgs P)
{
    const int M = T.M, GM = T.GM;
    // Workgroup ids are renumbered.  The rows with work (r < nrp of each
    // parity) come first, so that they take a CU each, and the rows beyond the
    // triangle, which only write zeros, are dispatched last.  The hardware
    // deals consecutive ids to the 8 XCDs in turn, and the rows of one
    // (vortex, parity) all read that vortex's partial sums and state of that
    // parity, so each XCD takes a contiguous run of rows (its L2 then fetches
    // those operands once).
    int r, par, j;
    {
        const int n0 = S2Shape(M, 0).nrp, n1 = S2Shape(M, 1).nrp, RPg = gridDim.x;
        const int per = n0 + n1, nwork = (gridDim.y >> 1) * per;
        const int lin = blockIdx.y * gridDim.x + blockIdx.x;
        if (lin < nwork) {
            const int xcd = lin & 7, q8 = nwork >> 3, r8 = nwork & 7;
            const int vid = xcd * q8 + (xcd < r8 ? xcd : r8) + (lin >> 3);
            j = vid / per;
            const int w = vid - j * per;
            par = w < n0 ? 0 : 1;
            r = par == 0 ? w : w - n0;
        } else {
            const int z = lin - nwork, perz = (RPg - n0) + (RPg - n1);
            j = z / perz;
            const int w = z - j * perz;
            par = w < RPg - n0 ? 0 : 1;
            r = par == 0 ? n0 + w : n1 + (w - (RPg - n0));
        }
    }
    const S2Shape sh(M, par);
    const T0Shape tz(M);
    const int LP = sh.LP, TP = tz.TP, LDA = LP + 2, LDB = TP + 2, LDQ = TP + 1;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g1 = par + 2 * r;
    const int len = r < sh.nrp ? GM - g1 + 1 : 0;
    const int p1 = g1 & 1, sh1 = (g1 + p1) >> 1;
    const int ks = (((M - p1) >> 1) + 4) >> 2;  // m1' < 4 ks covers m1 <= M
    double* out = B.s_pad + ((long)j * 2 + par) * sh.RP * sh.KA + r;  // column g2 at out[g2 * RP]
    if (len == 0 && r != 0) {  // rows beyond the triangle
        for (int c = tid; c < sh.KA; c += kSelfThreads) out[(long)c * sh.RP] = 0.0;
        return;
    }
    extern __shared__ double smem[];
    double* sAl = smem;                  // alpha rows m1 = p1 + 2 m1', [4 kSelfKS][LDA]
    double* sT0 = sAl + 4 * kSelfKS * LDA;  // t0 rows sh1 + m1', [4 kSelfKS][LDB]
    double* sQ = sT0 + 4 * kSelfKS * LDB;   // Q [LP][LDQ]
    constexpr int kRows = 4 * kSelfKS;
    constexpr int kRowSlots = kRows / kSelfWaves;
    static_assert(kRowSlots * kSelfWaves == kRows, "rows");
    static_assert(16 * ((kS2MaxOrder + 16) / 16) <= 64, "a row of alpha fits a wavefront");

    const double2* gT = reinterpret_cast<const double2*>(T.t0d);
    // Operand rows past the k-steps in use are never read by the products, so
    // their loads only need to stay inside the tables: the indices are clamped
    // (lane-dependent arithmetic, no branch around a load).
    const int capT = tz.T0R * (TP / 2) - 1;
    if constexpr (APPLY) {
        // finish the previous stage for the moments with m1 of this parity; the
        // row-0 workgroup of each parity writes their state and signed moments.
        // All loads first; the powers of lambda come from a per-workgroup table
        // (binary exponentiation: short dependency chains).
        // RK4 weight of this stage and node of the next one
        const double wst = (P.stage == 0 || P.stage == 3) ? 1.0 / 6.0 : 1.0 / 3.0;
        const double cnx = P.stage < 2 ? 0.5 : 1.0;
        const bool writer = r == 0;
        const double l0sq = B.lam0sq[j], nuj = B.nuv[j], tfj = B.toff[j];  // issued with the operand loads
        double2 vt2[kRowSlots];
        double pg[kRowSlots][4], pc[kRowSlots], py[kRowSlots], pa[kRowSlots];
        const long LL = (long)LP * LP;
        const double* gpj = B.gpartD + (long)j * 4 * LL;
        const double* yj = B.ystate[P.ycur] + (long)j * LL;
        const double* aj = B.accD + (long)j * LL;
#pragma unroll
        for (int q = 0; q < kRowSlots; ++q) {
            const int m1p = wave + kSelfWaves * q, m1 = p1 + 2 * m1p, m2 = lane;
            vt2[q] = gT[min((sh1 + m1p) * (TP / 2) + lane, capT)];
            const int d = m1 + m2 <= M ? m1 * LP + m2 : 0;  // dense (k1, k2) position
#pragma unroll
            for (int h = 0; h < 4; ++h) pg[q][h] = gpj[h * LL + d];
            pc[q] = T.c1d[d];
            py[q] = yj[d];
            pa[q] = aj[d];  // used from stage 1 on
        }
#pragma unroll
        for (int q = 0; q < kRowSlots; ++q) {
            const int m1p = wave + kSelfWaves * q;
            if (lane < TP / 2) reinterpret_cast<double2*>(sT0 + m1p * LDB)[lane] = vt2[q];
        }
        __shared__ double pw[2][MMVM_MAX_ORDER + 1];  // lambda_prev^s / lambda_prev^2, lambda_next^{-s}
        if (tid <= M) {
            double tp = P.t_prev, tn = P.t_next;
            if (P.clock) {
                const double t0 = P.clock->t0;
                const long long n = P.clock->n;
                tp = clock_time(t0, n + P.n_prev, P.c_prev, P.dt);
                tn = clock_time(t0, n + P.n_next, P.c_next, P.dt);
            }
            const double lam2p = l0sq + 4.0 * nuj * __dadd_rn(tp, tfj);
            const double lam2n = l0sq + 4.0 * nuj * __dadd_rn(tn, tfj);
            pw[0][tid] = pow_uint(sqrt(lam2p), tid) / lam2p;
            pw[1][tid] = pow_uint(1.0 / sqrt(lam2n), tid);
            if (writer && par == 0 && tid == 0) B.lam2[cur][j] = lam2n;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kRowSlots; ++q) {
            const int m1p = wave + kSelfWaves * q, m1 = p1 + 2 * m1p, m2 = lane;
            double a = 0.0;
            if (m1 + m2 <= M) {
                const int s = m1 + m2, k = ctri(m1, m2);
                double g = pg[q][0] + pg[q][1];
                g += pg[q][2];
                g += pg[q][3];
                const double val = k == 0 ? 0.0 : (pc[q] * g) * pw[0][s];  // circulation is conserved exactly
                double nxt;
                const long o = (long)j * LL + m1 * LP + m2;
                if (P.stage < 3) {
                    if (writer) B.accD[o] = P.stage == 0 ? wst * val : pa[q] + wst * val;
                    nxt = py[q] + cnx * P.dt * val;
                } else {
                    nxt = py[q] + P.dt * (pa[q] + wst * val);
                    if (writer) B.ystate[1 - P.ycur][o] = nxt;
                }
                a = nxt * pw[1][s];
                if (writer) B.alphaS[cur][(long)j * LP * LP + m2 * LP + m1] = (s & 1) ? -a : a;
            }
            if (lane < LP) sAl[m1p * LDA + lane] = a;
        }
    } else {
        // operands: rows copied as double2, all loads first
        const double2* gA = reinterpret_cast<const double2*>(B.alphaD[cur] + (long)j * sh.LA() * LP);
        const int capA = sh.LA() * (LP / 2) - 1;
        double2 va[kRowSlots], vt[kRowSlots];
#pragma unroll
        for (int q = 0; q < kRowSlots; ++q) {
            const int m1p = wave + kSelfWaves * q;
            va[q] = gA[min((p1 + 2 * m1p) * (LP / 2) + lane, capA)];
            vt[q] = gT[min((sh1 + m1p) * (TP / 2) + lane, capT)];
        }
#pragma unroll
        for (int q = 0; q < kRowSlots; ++q) {
            const int m1p = wave + kSelfWaves * q;
            if (lane < LP / 2) reinterpret_cast<double2*>(sAl + m1p * LDA)[lane] = va[q];
            if (lane < TP / 2) reinterpret_cast<double2*>(sT0 + m1p * LDB)[lane] = vt[q];
        }
    }
    __syncthreads();
    // Q tiles: rows m2 < LP, columns b <= bmax
    {
        const int bmax = (M + len - 1) >> 1;
        const int tr = LP >> 4, tc = (bmax >> 4) + 1;
        const View va_ = {sAl, 1, LDA}, vb_ = {sT0, LDB, 1};
        for (int t = wave; t < tr * tc; t += kSelfWaves) {
            const int r0 = (t / tc) * 16, c0 = (t % tc) * 16;
            // alpha[m1][m2] = 0 for m1 + m2 > M: rows m2 >= r0 need m1' <= (M - r0 - p1) / 2
            // only (the k-steps skipped would add exact zeros at the end of the sum)
            const int nm = M - r0 - p1 >= 0 ? ((M - r0 - p1) >> 1) + 1 : 0;
            const int kt = (nm + 3) >> 2;
            const dbl4 d = mfma_tile<kSelfKS>(lane, r0, c0, 0, kt < ks ? kt : ks, va_, vb_);
#pragma unroll
            for (int q = 0; q < 4; ++q) sQ[(r0 + (lane >> 4) + 4 * q) * LDQ + c0 + (lane & 15)] = d[q];
        }
    }
    __syncthreads();
    // S[g1][g2] = sum over m2 of the parity of g2; four lanes per entry
    for (int t = tid; t < 4 * sh.KA; t += kSelfThreads) {
        const int g2 = t >> 2, q = t & 3;
        double acc = 0.0;
        if (g2 < len)
            for (int m2 = (g2 & 1) + 2 * q; m2 <= M; m2 += 8) acc += sQ[m2 * LDQ + ((m2 + g2) >> 1)];
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        if (q == 0) out[(long)g2 * sh.RP] = (g2 < len && g1 + g2 > 0) ? acc : 0.0;
    }
}

static size_t self_mfma_lds(int M)
{
    const S2Shape sh(M, 0);
    const T0Shape tz(M);
    return sizeof(double) * (4 * (size_t)kSelfKS * ((sh.LP + 2) + (tz.TP + 2)) + (size_t)sh.LP * (tz.TP + 1));
}

bool stage2_fuses_emit(int M, bool dd, bool solo) { return stage2_uses_mfma(M, dd, solo) && solo; }

hipError_t launch_self_apply(const DevTables& T, const StageBufs& B, int cur, const ApplyArgs& P, hipStream_t st)
{
    const S2Shape sh(T.M, 0);
    launch_kernel(k_self_mfma<true>, dim3(sh.RP, 2 * B.N), dim3(kSelfThreads), self_mfma_lds(T.M), st, T, B,
                       cur, P);
    return hipGetLastError();
}

// the last stage of a stepping call: y_{n+1} into the caller's moments (the
// emit kernel's arithmetic)
__global__ __launch_bounds__(1024) void k_apply_final(DevTables T, StageBufs B, ApplyArgs P)
{
    const int j = blockIdx.x, K = T.K;
    const int LP = 16 * ((T.M + 16) / 16);
    const long LL = (long)LP * LP;
    const double lam2p = B.lam0sq[j] + 4.0 * B.nuv[j] * __dadd_rn(P.t_prev, B.toff[j]);
    const double lamp = sqrt(lam2p);
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const int s = shell_of(k);
        const int k2 = k - s * (s + 1) / 2, k1 = s - k2;
        const long o = (long)j * LL + k1 * LP + k2;
        const double* gp = B.gpartD + (long)j * 4 * LL + k1 * LP + k2;
        double g = gp[0] + gp[LL];
        g += gp[2 * LL];
        g += gp[3 * LL];
        const double lp = pow_uint(lamp, s) / lam2p;  // lambda^{s-2}
        const double val = k == 0 ? 0.0 : (T.c1d[k1 * LP + k2] * g) * lp;
        P.mom_out[(long)j * K + k] = B.ystate[P.ycur][o] + P.dt * (B.accD[o] + (1.0 / 6.0) * val);
    }
}

__global__ void k_set_clock(DevClock* clock, double t0, long long n)
{
    if (threadIdx.x == 0) {
        clock->t0 = t0;
        clock->n = n;
    }
}

hipError_t launch_set_clock(DevClock* clock, double t0, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(64), 0, st, clock, t0, n);
    return hipGetLastError();
}

__global__ void k_advance_clock(DevClock* clock, long long by)
{
    if (threadIdx.x == 0) clock->n += by;
}

hipError_t launch_advance_clock(DevClock* clock, long long by, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance_clock, dim3(1), dim3(64), 0, st, clock, by);
    return hipGetLastError();
}

hipError_t launch_apply_final(const DevTables& T, const StageBufs& B, const ApplyArgs& P, hipStream_t st)
{
    launch_kernel(k_apply_final, dim3(B.N), dim3(1024), 0, st, T, B, P);
    return hipGetLastError();
}

hipError_t launch_self_pad(const DevTables& T, const StageBufs& B, int cur, hipStream_t st)
{
    const S2Shape sh(T.M, 0);
    ApplyArgs none{};
    launch_kernel(k_self_mfma<false>, dim3(sh.RP, 2 * B.N), dim3(kSelfThreads), self_mfma_lds(T.M), st, T, B,
                       cur, none);
    return hipGetLastError();
}

constexpr int kEmitThreads = 1024;  // one moment per thread up to the largest order
static_assert((MMVM_MAX_ORDER + 1) * (MMVM_MAX_ORDER + 2) / 2 <= kEmitThreads, "emit");

template <class A>
__global__ __launch_bounds__(kEmitThreads) void k_emit(DevTables T, StageBufs B, StageArgs S)
{
    typedef typename A::T R;
    const int K = T.K, N = B.N, j = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    __shared__ double red[2 * kEmitThreads / 64];
    const double* al = B.alpha[S.cur] + (long)j * K;
    const double* sp = B.interact ? B.s_pair + (long)j * T.KG : nullptr;
    const double lam2 = B.lam2[S.cur][j];
    const double lam = sqrt(lam2);
    double tn = S.t_next;
    if (S.clock)  // graph replay: the stage time from the device clock
        tn = clock_time(S.clock->t0, S.clock->n + S.n_rel, S.c_next, S.dt);
    const double lam2n = B.lam0sq[j] + 4.0 * B.nuv[j] * __dadd_rn(tn, B.toff[j]);
    double xd1 = 0.0, xd2 = 0.0;
    if (B.interact) centre_velocity(al, sp, K, lam, red, xd1, xd2);
    const double* gj = B.gpart + (long)j * 4 * K * 2;
    const int LP = 16 * ((T.M + 16) / 16);
    for (int k = tid; k < K; k += nt) {
        const int s = shell_of(k);
        const int kk2 = k - s * (s + 1) / 2, k1 = s - kk2;
        R g = A::zero();
        if constexpr (std::is_same<A, ArithF64>::value) {  // the matrix-core contraction: dense partials
            const double* gd = B.gpartD + (long)j * 4 * LP * LP + k1 * LP + kk2;
            for (int q = 0; q < 4; ++q) g = A::add(g, gd[(long)q * LP * LP]);
        } else {
            for (int q = 0; q < 4; ++q) g = A::add(g, A::ldst(gj + ((long)q * K + k) * 2));
        }
        const double lp = pow_uint(lam, s) / lam2;  // lambda^{s-2}
        double val = A::hi(A::madd(A::zero(), A::ld(T.c1_hi, T.c1_lo, k), g)) * lp;
        if (B.interact) {  // drift, eq:last_termsimp: xdot_1 M_{k-e1} + xdot_2 M_{k-e2}
            double lq = lp * lam;  // lambda^{s-1}
            if (k1 >= 1) val += xd1 * al[ctri(k1 - 1, kk2)] * lq;
            if (kk2 >= 1) val += xd2 * al[ctri(k1, kk2 - 1)] * lq;
        }
        if (k == 0) val = 0.0;  // circulation is conserved exactly
        emit_moment(B, S, T.M, j, k, s, K, val, lam2n);
    }
    if (tid == 0) emit_position(B, S, j, xd1, xd2, lam2n);
}

// ---------------------------------------------------------------------------
// stage 2 for small orders (M <= kMaxSmallOrder): one workgroup per vortex
// computes its self table, then all k2 and both halves of the contraction at
// once (four barriers per stage), then the drift and the RK4 update.  The same
// stage body drives the persistent kernel k_solo_rk4 below.
// ---------------------------------------------------------------------------
// the first l1 whose rows l2 <= M - l1 no longer fit in half the work of step B
constexpr int small_split(int M)
{
    const int M1 = M + 1, K = M1 * (M1 + 1) / 2;
    int w = 0, L = 0;
    while (L < M1 && 2 * (w + (M1 - L)) <= K) w += M1 - L++;
    return L < 1 ? 1 : L;
}

template <int M>
struct SmallShape {
    static constexpr int K = (M + 1) * (M + 2) / 2;
    static constexpr int GM = M == 0 ? 1 : 2 * M;
    static constexpr int KG = (GM + 1) * (GM + 2) / 2;
    static constexpr int M1 = M + 1;
    static constexpr int G1 = GM + 1;         // rows g1 of the velocity-derivative table
    static constexpr int G2 = GM + 2;         // its columns g2 = 0 .. GM + 1 (zero beyond the triangle)
    static constexpr int NY = 2 * M1 * G1 * M1;  // (pass, k2, g1, l2)
    static constexpr int T0N = ((M == 0 ? 1 : 3 * M) + 1) / 2 + 1;
    static constexpr int NT0 = (T0N + 1) * (T0N + 2) / 2;
    static constexpr int T0W = T0N + 1;       // row length of the rectangular Psi0 table
    // LDS regions (doubles); the rectangular layouts hold zeros outside their triangles
    static constexpr int AL = 0;                     // [K] alpha, shell-major
    static constexpr int AU = AL + K;                // [M1][M1] alpha at (l1, l2)
    static constexpr int AR = AU + M1 * M1;          // [M1][M1] (-1)^{|l|} alpha at (l1, l2)
    static constexpr int SS = AR + M1 * M1;          // [G1][G2] S_self + S_pair
    static constexpr int SY = SS + G1 * G2;          // [NY] step A output
    static constexpr int ST = SY + NY;               // [NY] step B output
    static constexpr int SP = ST + NY;               // [2][K][M1] partials of step C
    static constexpr int F0 = SP + 2 * K * M1;       // [M1^3] factor table f0
    static constexpr int F1 = F0 + M1 * M1 * M1;     // [M1^3] factor table f1
    static constexpr int T0 = F1 + M1 * M1 * M1;     // [T0W][T0W] Psi0 table
    static constexpr int TOTAL = T0 + T0W * T0W;
    // step B: a thread owns l1 < LB or l1 >= LB of one row (about half the work each)
    static constexpr int LB = small_split(M);
};

// The tables of the small-order stage into LDS, and the zeros of the
// rectangular layouts (entries outside the triangles are never written later).
template <int M>
__device__ __forceinline__ void small_load_tables(const DevTables& T, double* smem)
{
    typedef SmallShape<M> Sh;
    const int tid = threadIdx.x, nt = blockDim.x;
    constexpr int M1 = Sh::M1;
    for (int i = tid; i < M1 * M1 * M1; i += nt) {
        smem[Sh::F0 + i] = T.f0_hi[i];
        smem[Sh::F1 + i] = T.f1_hi[i];
    }
    for (int i = tid; i < Sh::T0W * Sh::T0W; i += nt) {
        const int a = i / Sh::T0W, b = i - a * Sh::T0W;
        smem[Sh::T0 + i] = a + b <= Sh::T0N ? T.t0_hi[ctri(a, b)] : 0.0;
    }
    for (int i = tid; i < M1 * M1; i += nt) {
        const int l1 = i / M1, l2 = i - l1 * M1;
        if (l1 + l2 > M) {
            smem[Sh::AU + i] = 0.0;
            smem[Sh::AR + i] = 0.0;
        }
    }
    for (int i = tid; i < Sh::G1 * Sh::G2; i += nt) {
        const int g1 = i / Sh::G2, g2 = i - g1 * Sh::G2;
        if (g1 + g2 > Sh::GM) smem[Sh::SS + i] = 0.0;
    }
}

// the scaled moment alpha_k (k = (k1, k2), shell s) into the three layouts
template <int M>
__device__ __forceinline__ void small_put_alpha(double* smem, int k, int s, int k1, int k2, double a)
{
    typedef SmallShape<M> Sh;
    smem[Sh::AL + k] = a;
    smem[Sh::AU + k1 * Sh::M1 + k2] = a;
    smem[Sh::AR + k1 * Sh::M1 + k2] = (s & 1) ? -a : a;
}

// Self table, steps A, B and C of one stage; alpha is in LDS (a barrier after
// it was written), sp = the pair table or null.  Ends with a barrier; the
// partial sums of step C are in the SP region.
template <int M>
__device__ __forceinline__ void small_stage(double* smem, const double* sp)
{
    typedef SmallShape<M> Sh;
    constexpr int K = Sh::K, GM = Sh::GM, KG = Sh::KG, M1 = Sh::M1, G1 = Sh::G1, G2 = Sh::G2, NY = Sh::NY;
    constexpr int T0W = Sh::T0W, LB = Sh::LB;
    const double* sAU = smem + Sh::AU;
    const double* sAR = smem + Sh::AR;
    double* sS = smem + Sh::SS;
    double* sY = smem + Sh::SY;
    double* sT = smem + Sh::ST;
    double* sP = smem + Sh::SP;
    const double* sF0 = smem + Sh::F0;
    const double* sF1 = smem + Sh::F1;
    const double* sT0 = smem + Sh::T0;
    const int tid = threadIdx.x, nt = blockDim.x;
    // self table S[g1][g2] = sum_m alpha_m Psi0(m + g) (c = 2), plus the pair
    // table; four lanes share one g, each taking every fourth m2 of its parity
    for (int task = tid; task < 4 * KG; task += nt) {
        const int g = task >> 2, q = task & 3;
        const int gs = shell_of(g);
        const int g2 = g - gs * (gs + 1) / 2, g1 = gs - g2;
        double acc = 0.0;
        for (int m2 = (g2 & 1) + 2 * q; m2 <= M; m2 += 8) {
            const double* a = sAU + (g1 & 1) * M1 + m2;
            const double* p = sT0 + ((g1 + (g1 & 1)) >> 1) * T0W + ((m2 + g2) >> 1);
            for (int m1 = g1 & 1; m1 + m2 <= M; m1 += 2, a += 2 * M1, p += T0W) acc = fma(*a, *p, acc);
        }
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        if (q == 0) sS[g1 * G2 + g2] = g == 0 ? 0.0 : (sp ? acc + sp[g] : acc);
    }
    __syncthreads();
    // (A) second axis: Y[pass][k2][g1][l2] = sum_i f[k2][l2][i] S[g1][k2 + l2 - 2i +- 1]
    // (lanes over g1; zeros of S cover g1 + g2 > GM)
    for (int task = tid; task < NY; task += nt) {
        const int c = task / G1, g1 = task - c * G1;  // c = (pass, k2, l2)
        const int pass = c / (M1 * M1);
        const int r = c - pass * (M1 * M1);
        const int k2 = r / M1, l2 = r - k2 * M1;
        const double* f = (pass == 0 ? sF0 : sF1) + (k2 * M1 + l2) * M1;
        const int imax = pass == 0 ? (l2 < k2 ? l2 : k2) : (l2 < k2 - 1 ? l2 : k2 - 1);
        const double* srow = sS + g1 * G2 + k2 + l2 + (pass == 0 ? 1 : -1);
        double acc = 0.0;
        for (int i = 0; i <= imax; ++i) acc = fma(f[i], srow[-2 * i], acc);
        sY[((pass * M1 + k2) * G1 + g1) * M1 + l2] = acc;
    }
    __syncthreads();
    // (B) T[row][l1] = sum_{l2 <= M - l1} (-1)^{|l|} alpha_l Y[row][l2]: the row
    // in registers, a thread per (row, l1 < LB) or (row, l1 >= LB)
    constexpr int NR = 2 * M1 * G1;
    for (int task = tid; task < 2 * NR; task += nt) {
        const int half = task / NR, row = task - half * NR;
        double y[M1];
        const double* yr = sY + row * M1;
#pragma unroll
        for (int l2 = 0; l2 < M1; ++l2) y[l2] = yr[l2];
        double* tr = sT + row * M1;
        if (half == 0) {
#pragma unroll
            for (int l1 = 0; l1 < LB; ++l1) {
                double acc = 0.0;
#pragma unroll
                for (int l2 = 0; l2 <= M - l1; ++l2) acc = fma(sAR[l1 * M1 + l2], y[l2], acc);
                tr[l1] = acc;
            }
        } else {
#pragma unroll
            for (int l1 = LB; l1 < M1; ++l1) {
                double acc = 0.0;
#pragma unroll
                for (int l2 = 0; l2 <= M - l1; ++l2) acc = fma(sAR[l1 * M1 + l2], y[l2], acc);
                tr[l1] = acc;
            }
        }
    }
    __syncthreads();
    // (C) first axis for every (pass, k, l1)
    for (int task = tid; task < 2 * K * M1; task += nt) {
        const int pass = task / (K * M1);
        const int r = task - pass * (K * M1);
        const int k = r / M1, l1 = r - k * M1;
        const int ks = shell_of(k);
        const int k2 = k - ks * (ks + 1) / 2, k1 = ks - k2;
        const double* tcol = sT + (long)(pass * M1 + k2) * G1 * M1 + l1;
        double acc = 0.0;
        if (pass == 0) {
            const double* f = sF1 + (k1 * M1 + l1) * M1;
            const int imax = l1 < k1 - 1 ? l1 : k1 - 1;
            const double* tp = tcol + (k1 + l1 - 1) * M1;
            for (int i = 0; i <= imax; ++i, tp -= 2 * M1) acc = fma(f[i], *tp, acc);
            acc = -acc;
        } else {
            const double* f = sF0 + (k1 * M1 + l1) * M1;
            const int imax = l1 < k1 ? l1 : k1;
            const int i0 = k1 + l1 + 1 > GM ? 1 : 0;  // g1 = k1 + l1 - 2i + 1 <= GM
            const double* tp = tcol + (k1 + l1 + 1 - 2 * i0) * M1;
            for (int i = i0; i <= imax; ++i, tp -= 2 * M1) acc = fma(f[i], *tp, acc);
        }
        sP[task] = acc;
    }
    __syncthreads();
}

// dM_k/dt from the partial sums of step C: lambda^{|k|-2} c1_k G_k, plus the
// drift xdot_1 M_{k-e1} + xdot_2 M_{k-e2} when the vortex moves; dM_00 = 0.
template <int M>
__device__ __forceinline__ double small_value(const DevTables& T, const double* smem, int k, double lam, double lam2,
                                              bool drift, double xd1, double xd2)
{
    typedef SmallShape<M> Sh;
    constexpr int K = Sh::K, M1 = Sh::M1;
    const double* sP = smem + Sh::SP;
    const double* sAl = smem + Sh::AL;
    // the two halves' partial sums over l1 in two chains
    double g = 0.0, h = 0.0;
#pragma unroll
    for (int l1 = 0; l1 < M1; ++l1) {
        g += sP[k * M1 + l1];
        h += sP[(K + k) * M1 + l1];
    }
    g += h;
    const int s = shell_of(k);
    const int k2 = k - s * (s + 1) / 2, k1 = s - k2;
    const double lp = pow_uint(lam, s) / lam2;
    double val = T.c1_hi[k] * g * lp;
    if (drift) {
        const double lq = lp * lam;
        if (k1 >= 1) val += xd1 * sAl[ctri(k1 - 1, k2)] * lq;
        if (k2 >= 1) val += xd2 * sAl[ctri(k1, k2 - 1)] * lq;
    }
    if (k == 0) val = 0.0;
    return val;
}

template <int M>
__global__ __launch_bounds__(1024) void k_stage2_small(DevTables T, StageBufs B, StageArgs S)
{
    typedef SmallShape<M> Sh;
    constexpr int K = Sh::K, KG = Sh::KG;
    extern __shared__ double smem[];
    __shared__ double red[32];
    const double* sAl = smem + Sh::AL;

    const int j = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const double* al = B.alpha[S.cur] + (long)j * K;
    for (int l = tid; l < K; l += nt) {
        const int s = shell_of(l), l2 = l - s * (s + 1) / 2;
        small_put_alpha<M>(smem, l, s, s - l2, l2, al[l]);
    }
    const double lam2 = B.lam2[S.cur][j];
    const double lam = sqrt(lam2);
    double tn = S.t_next;
    if (S.clock)  // graph replay: the stage time from the device clock
        tn = clock_time(S.clock->t0, S.clock->n + S.n_rel, S.c_next, S.dt);
    const double lam2n = B.lam0sq[j] + 4.0 * B.nuv[j] * __dadd_rn(tn, B.toff[j]);
    const double* sp = B.interact ? B.s_pair + (long)j * KG : nullptr;
    __shared__ double spl[KG];
    if (B.interact && B.pair_groups > 1) {
        // the few-vortex pair kernel left one partial table per source group: add them in group order
        const double* part = B.p_part + (long)j * B.pair_groups * KG;
        for (int g = tid; g < KG; g += nt) {
            double v = 0.0;
            for (int q = 0; q < B.pair_groups; ++q) v += part[(long)q * KG + g];
            spl[g] = v;
        }
        sp = spl;
    }
    small_load_tables<M>(T, smem);
    __syncthreads();
    double xd1 = 0.0, xd2 = 0.0;
    if (B.interact) centre_velocity(sAl, sp, K, lam, red, xd1, xd2);
    small_stage<M>(smem, sp);
    for (int k = tid; k < K; k += nt) {
        const double val = small_value<M>(T, smem, k, lam, lam2, B.interact != 0, xd1, xd2);
        emit_moment(B, S, T.M, j, k, shell_of(k), K, val, lam2n);
    }
    if (tid == 0) emit_position(B, S, j, xd1, xd2, lam2n);
}

// ---------------------------------------------------------------------------
// Persistent RK4 for independent single vortices of small order: workgroup j
// advances solve j through all nsteps classic RK4 steps (four stages each)
// without leaving the kernel.  The tables stay in LDS for the whole run; the
// state y_n and the RK4 accumulator of moment k live in the registers of
// thread k.  A single vortex does not move (its pair table and drift are
// zero), so the centre is not touched.  Each stage computes what k_prep and
// k_stage2_small compute at the same stage times (the same stage body and
// power functions).
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(1024) void k_solo_rk4(DevTables T, const double* __restrict__ lam0sq,
                                                   const double* __restrict__ nuv, const double* __restrict__ toff,
                                                   double t0, double dt, int64_t nsteps, double* __restrict__ mom,
                                                   int* __restrict__ flag)
{
    typedef SmallShape<M> Sh;
    constexpr int K = Sh::K;
    static_assert(K <= 1024, "one thread per moment");
    extern __shared__ double smem[];
    const int j = blockIdx.x, tid = threadIdx.x;
    const double l0 = lam0sq[j], nu = nuv[j], tf = toff[j];
    double* my = mom + (long)j * K;
    const bool owner = tid < K;
    const int sk = owner ? shell_of(tid) : 0;
    const int k2 = owner ? tid - sk * (sk + 1) / 2 : 0, k1 = sk - k2;
    double yn = 0.0, acc = 0.0, ys = 0.0;
    if (owner) {
        yn = my[tid];
        ys = yn;
        if (!isfinite(yn)) atomicOr(flag, 2);
    }
    small_load_tables<M>(T, smem);
    const double cst[4] = {0.0, 0.5, 0.5, 1.0};
    const double wts[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    for (int64_t n = 0; n < nsteps; ++n) {
        for (int s = 0; s < 4; ++s) {
            const double ts = t0 + ((double)n + cst[s]) * dt;
            const double lam2 = l0 + 4.0 * nu * __dadd_rn(ts, tf);
            if (owner) small_put_alpha<M>(smem, tid, sk, k1, k2, ys * inv_lambda_pow(lam2, sk));
            __syncthreads();
            small_stage<M>(smem, nullptr);
            if (owner) {
                const double val = small_value<M>(T, smem, tid, sqrt(lam2), lam2, false, 0.0, 0.0);
                // the RK4 bookkeeping of rk4_update, in registers
                if (s == 0) acc = wts[0] * val;
                else if (s < 3) acc += wts[s] * val;
                if (s < 3) {
                    ys = yn + cst[s + 1] * dt * val;
                } else {
                    yn = yn + dt * (acc + wts[3] * val);
                    ys = yn;
                }
            }
            // the next writes of alpha follow the last reads of this stage
            // (steps A-C) across the barrier that ends small_stage
        }
    }
    if (owner) {
        my[tid] = yn;
        if (!isfinite(yn)) atomicOr(flag, 2);
    }
}

bool stage2_fuses_self(int M, bool dd, bool solo) { return !dd && M <= kMaxSmallOrder && !stage2_uses_mfma(M, dd, solo); }

template <int M>
static hipError_t launch_small(const DevTables& T, const StageBufs& B, const StageArgs& A, hipStream_t st)
{
    typedef SmallShape<M> Sh;
    if (T.T0N != Sh::T0N) return hipErrorInvalidValue;
    const size_t shmem = sizeof(double) * (size_t)Sh::TOTAL;
    // few vortices: wide workgroups for latency; many: one to four wavefronts each
    int threads = B.N <= 32 ? 1024 : (Sh::NY >= 1024 ? 256 : (Sh::NY >= 256 ? 128 : 64));
    if (shmem > 64 * 1024) {
        const hipError_t ea =
            lds_limit_once((const void*)k_stage2_small<M>, shmem, "hipFuncSetAttribute(k_stage2_small dynamic LDS)");
        if (ea != hipSuccess) return ea;
    }
    launch_kernel(k_stage2_small<M>, dim3(B.N), dim3(threads), shmem, st, T, B, A);
    return hipGetLastError();
}

template <int M>
static hipError_t launch_solo_M(const DevTables& T, int nb, const double* lam0sq, const double* nuv,
                                const double* toff, double t0, double dt, int64_t nsteps, double* mom, int* flag,
                                hipStream_t st)
{
    typedef SmallShape<M> Sh;
    if (T.T0N != Sh::T0N) return hipErrorInvalidValue;
    const size_t shmem = sizeof(double) * (size_t)Sh::TOTAL;
    if (shmem > 64 * 1024) {
        const hipError_t ea =
            lds_limit_once((const void*)k_solo_rk4<M>, shmem, "hipFuncSetAttribute(k_solo_rk4 dynamic LDS)");
        if (ea != hipSuccess) return ea;
    }
    const int threads = Sh::K > 256 ? 1024 : kSoloThreads;
    launch_kernel(k_solo_rk4<M>, dim3(nb), dim3(threads), shmem, st, T, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag);
    return hipGetLastError();
}

bool solo_persistent(int M, bool dd) { return !dd && M >= 0 && M <= kMaxSoloOrder; }

hipError_t launch_solo_rk4(const DevTables& T, int nb, const double* lam0sq, const double* nuv, const double* toff,
                           double t0, double dt, int64_t nsteps, double* mom, int* flag, hipStream_t st)
{
    switch (T.M) {
    case 0: return launch_solo_M<0>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    case 1: return launch_solo_M<1>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    case 2: return launch_solo_M<2>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    case 3: return launch_solo_M<3>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    case 4: return launch_solo_M<4>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    case 5: return launch_solo_M<5>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    case 6: return launch_solo_M<6>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    case 7: return launch_solo_M<7>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    case 8: return launch_solo_M<8>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    case 9: return launch_solo_M<9>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    case 10: return launch_solo_M<10>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    case 11: return launch_solo_M<11>(T, nb, lam0sq, nuv, toff, t0, dt, nsteps, mom, flag, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stage2(const DevTables& T, const StageBufs& B, const StageArgs& A, bool use_dd, hipStream_t st)
{
    if (stage2_fuses_self(T.M, use_dd, !B.interact)) {
        switch (T.M) {
        case 0: return launch_small<0>(T, B, A, st);
        case 1: return launch_small<1>(T, B, A, st);
        case 2: return launch_small<2>(T, B, A, st);
        case 3: return launch_small<3>(T, B, A, st);
        case 4: return launch_small<4>(T, B, A, st);
        case 5: return launch_small<5>(T, B, A, st);
        case 6: return launch_small<6>(T, B, A, st);
        case 7: return launch_small<7>(T, B, A, st);
        case 8: return launch_small<8>(T, B, A, st);
        case 9: return launch_small<9>(T, B, A, st);
        case 10: return launch_small<10>(T, B, A, st);
        default: break;
        }
    }
    const int M1 = T.M + 1;
    dim3 grid(4 * M1, B.N);
    if (!use_dd) {
        if (!stage2_uses_mfma(T.M, use_dd, !B.interact)) return hipErrorInvalidValue;
        const size_t shmem = sizeof(double) * (size_t)s2m_lds_doubles(T.M);
        // the limit is the largest order's size for every order
        const size_t most = sizeof(double) * (size_t)s2m_lds_doubles(kS2MaxOrder);
        if (shmem > most) return hipErrorInvalidValue;
        const hipError_t ea =
            lds_limit_once((const void*)k_stage2_mfma, most, "hipFuncSetAttribute(k_stage2_mfma dynamic LDS)");
        if (ea != hipSuccess) return ea;
        launch_kernel(k_stage2_mfma, grid, dim3(kS2Threads), shmem, st, T, B, A);
        return hipGetLastError();
    }
    // the fill is sized for kDDThreads threads and orders <= MMVM_MAX_ORDER
    if (!B.s_self_lo || T.M > MMVM_MAX_ORDER) return hipErrorInvalidValue;
    // the workgroups fit one round at one per CU: stage step C's tables in LDS;
    // more: the smaller layout, two workgroups per CU
    const bool ctab = 4 * M1 * B.N <= kDDOneRound;
    const size_t shmem = sizeof(double) * (size_t)DDShape(T.M, 0, ctab).total;
    // each variant's limit is the largest order's size for every order
    const size_t most = sizeof(double) * (size_t)DDShape(MMVM_MAX_ORDER, 0, ctab).total;
    if (shmem > most) return hipErrorInvalidValue;
    const hipError_t ea =
        ctab ? lds_limit_once((const void*)k_stage2_dd<true>, most, "hipFuncSetAttribute(k_stage2_dd dynamic LDS)")
             : lds_limit_once((const void*)k_stage2_dd<false>, most, "hipFuncSetAttribute(k_stage2_dd dynamic LDS)");
    if (ea != hipSuccess) return ea;
    if (ctab) launch_kernel(k_stage2_dd<true>, grid, dim3(kDDThreads), shmem, st, T, B, A);
    else launch_kernel(k_stage2_dd<false>, grid, dim3(kDDThreads), shmem, st, T, B, A);
    return hipGetLastError();
}

bool stage2_needs_emit(int M, bool dd, bool solo) { return !stage2_fuses_self(M, dd, solo); }

hipError_t launch_emit(const DevTables& T, const StageBufs& B, const StageArgs& A, bool use_dd, hipStream_t st)
{
    if (use_dd) launch_kernel(k_emit<ArithDD>, dim3(B.N), dim3(kEmitThreads), 0, st, T, B, A);
    else launch_kernel(k_emit<ArithF64>, dim3(B.N), dim3(kEmitThreads), 0, st, T, B, A);
    return hipGetLastError();
}

}  // namespace mmvm
