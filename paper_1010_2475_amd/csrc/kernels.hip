// HIP kernels (gfx950) of the MMVM hot path.
//
// Per right-hand side (one RK4 stage) the path runs four kernels:
//   k_prep    stage input -> lambda_j(t)^2, scaled moments alpha = M_k / lambda^{|k|}
//             (row-major and source-major copies), circulation/finiteness checks
//   k_self    self velocity-derivative table  S_self[g] = sum_m alpha_m Psi0(m + g)
//   k_pair    pair velocity-derivative table  S_pair[g] = sum_{j'} sum_m ... Psi(m + g; s_jj')
//             (one wavefront per target, lanes over sources, wavefront-shuffle reduction)
//   k_stage2  the factorised contraction of eq:FinalSingleI/II (self + pair share it),
//             the drift term, the centre velocity, and the RK4 bookkeeping
// All quantities are in "lambda units" of the target vortex: with
// alpha_l = M_l lambda^{-|l|} and S in units lambda^{|g|}, eq:moment_evolutionFinish
// becomes dM_k/dt = lambda^{|k|-2} G_k(alpha, S) with lambda-free tables.
#include <type_traits>
#include <utility>

#include "dd.hpp"
#include "kernels.hpp"
#include "util.hpp"

namespace mmvm {

// ---------------------------------------------------------------------------
// prep
// ---------------------------------------------------------------------------
__device__ __forceinline__ double inv_lambda_pow(double l2, int s)
{
    const double il = 1.0 / sqrt(l2);
    double p = 1.0;
    for (int e = 0; e < s; ++e) p *= il;
    return p;
}

__global__ __launch_bounds__(256) void k_prep(int N, int K, const double* __restrict__ xin,
                                              const double* __restrict__ min_, const double* __restrict__ lam0sq,
                                              double t, double nu, double* __restrict__ xs, double* __restrict__ ys,
                                              double* __restrict__ lam2, double* __restrict__ alpha,
                                              double* __restrict__ alphaT, float* __restrict__ alphaT32,
                                              int* __restrict__ flag, unsigned* __restrict__ done, int copy_state)
{
    const long total = (long)N * K;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        int j = (int)(idx / K), k = (int)(idx - (long)j * K);
        double l2 = lam0sq[j] + 4.0 * nu * t;
        double mk = min_[idx];
        double a = mk * inv_lambda_pow(l2, shell_of(k));
        if (copy_state) ys[idx] = mk;
        alpha[idx] = a;
        if (alphaT) alphaT[(long)k * N + j] = a;
        if (alphaT32) alphaT32[(long)k * N + j] = (float)a;
        if (!isfinite(mk)) atomicOr(flag, 2);
        if (k == 0) {
            lam2[j] = l2;
            if (done) done[j] = 0u;
            double x0 = xin[2 * j], x1 = xin[2 * j + 1];
            xs[2 * j] = x0;
            xs[2 * j + 1] = x1;
            if (N > 1 && mk == 0.0) atomicOr(flag, 1);
            if (!isfinite(x0) || !isfinite(x1)) atomicOr(flag, 2);
        }
    }
}

hipError_t launch_prep(const DevTables& T, const StageBufs& B, int cur, const double* xin, const double* min_,
                       double t, double nu, bool need_pair, bool need_f32, hipStream_t st)
{
    long total = (long)B.N * T.K;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    bool copy = (min_ != B.ys);
    hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(256), 0, st, B.N, T.K, xin, min_, B.lam0sq, t, nu, B.xs,
                       B.ys, B.lam2[cur], B.alpha[cur], need_pair && !need_f32 ? B.alphaT[cur] : (double*)nullptr,
                       need_pair && need_f32 ? B.alphaT32[cur] : (float*)nullptr, B.flag, B.done, copy ? 1 : 0);
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
__device__ __forceinline__ void emit_moment(const StageBufs& B, const StageArgs& S, int j, int k, int s, int K,
                                            double val, double lam2_next)
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
    if (S.want_pair) {
        if (S.want_f32) B.alphaT32[nx][(long)k * B.N + j] = (float)a;
        else B.alphaT[nx][(long)k * B.N + j] = a;
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
    B.xs[2 * j] = rk4_update(S.stage, S.dt, S.x + 2 * j, B.accx + 2 * j, xd1);
    B.xs[2 * j + 1] = rk4_update(S.stage, S.dt, S.x + 2 * j + 1, B.accx + 2 * j + 1, xd2);
    B.lam2[1 - S.cur][j] = lam2_next;
}

// ---------------------------------------------------------------------------
// self velocity-derivative table: S_self[j][g] = sum_m alpha_m Psi0(m + g), c = 2
// (the target's own Gaussian convolved with itself: Lambda^2 = 2 lambda^2).
// Psi0 is nonzero only for even-even arguments.
// ---------------------------------------------------------------------------
template <bool DD>
__global__ __launch_bounds__(256) void k_self(int N, int M, int K, int GM, int KG, int T0N,
                                              const double* __restrict__ alpha, const double* __restrict__ t0h,
                                              const double* __restrict__ t0l, double* __restrict__ sself,
                                              double* __restrict__ sself_lo)
{
    // LDS: alpha of the vortex [K] and the Psi0 table [tri(T0N)] (hi, lo).
    // Four lanes share one entry g, each summing every fourth even-step m2.
    extern __shared__ double sm_self[];
    const int nt0 = (T0N + 1) * (T0N + 2) / 2;
    double* sa = sm_self;
    double* th = sa + K;
    double* tl = th + nt0;
    const int j = blockIdx.y;
    const double* a = alpha + (long)j * K;
    for (int i = threadIdx.x; i < K; i += blockDim.x) sa[i] = a[i];
    for (int i = threadIdx.x; i < nt0; i += blockDim.x) {
        th[i] = t0h[i];
        if (DD) tl[i] = t0l[i];
    }
    __syncthreads();
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = gt >> 2, q = gt & 3;
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
        dd acc = dd_make(0.0);
        if (live)
            for (int m2 = (g2 & 1) + 2 * q; m2 <= M; m2 += 8) {
                const int b2 = (m2 + g2) >> 1;
                for (int m1 = g1 & 1; m1 + m2 <= M; m1 += 2) {
                    const int ti = ctri((m1 + g1) >> 1, b2);
                    acc = dd_add(acc, dd_mul(dd_make(th[ti], tl[ti]), dd_make(sa[ctri(m1, m2)])));
                }
            }
        for (int off = 1; off <= 2; off <<= 1) {
            dd o = dd_make(__shfl_xor(acc.hi, off, 64), __shfl_xor(acc.lo, off, 64));
            acc = dd_add(acc, o);
        }
        if (q == 0 && g < KG) {
            sself[(long)j * KG + g] = live ? acc.hi : 0.0;
            sself_lo[(long)j * KG + g] = live ? acc.lo : 0.0;
        }
    }
}

hipError_t launch_self(const DevTables& T, const StageBufs& B, int cur, bool dd, hipStream_t st)
{
    const int threads = 256;
    dim3 grid((4 * T.KG + threads - 1) / threads, B.N);
    const int nt0 = (T.T0N + 1) * (T.T0N + 2) / 2;
    size_t shmem = sizeof(double) * ((size_t)T.K + (dd ? 2 : 1) * (size_t)nt0);
    if (dd)
        hipLaunchKernelGGL(k_self<true>, grid, dim3(threads), shmem, st, B.N, T.M, T.K, T.GM, T.KG, T.T0N,
                           B.alpha[cur], T.t0_hi, T.t0_lo, B.s_self, B.s_self_lo);
    else
        hipLaunchKernelGGL(k_self<false>, grid, dim3(threads), shmem, st, B.N, T.M, T.K, T.GM, T.KG, T.T0N,
                           B.alpha[cur], T.t0_hi, T.t0_lo, B.s_self, (double*)nullptr);
    return hipGetLastError();
}

template <int M>
hipError_t launch_pair_M(const DevTables& T, const StageBufs& B, int cur, bool f32, hipStream_t st);

bool pair_order_supported(int M) { return M >= 0 && M <= kMaxPairOrder; }

hipError_t launch_pair(const DevTables& T, const StageBufs& B, int cur, bool f32, hipStream_t st)
{
    switch (T.M) {
    case 0: return launch_pair_M<0>(T, B, cur, f32, st);
    case 1: return launch_pair_M<1>(T, B, cur, f32, st);
    case 2: return launch_pair_M<2>(T, B, cur, f32, st);
    case 3: return launch_pair_M<3>(T, B, cur, f32, st);
    case 4: return launch_pair_M<4>(T, B, cur, f32, st);
    case 5: return launch_pair_M<5>(T, B, cur, f32, st);
    case 6: return launch_pair_M<6>(T, B, cur, f32, st);
    default: return hipErrorInvalidValue;
    }
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

template <class A, bool FSLICE>
__global__ __launch_bounds__(512) void k_stage2(DevTables T, StageBufs B, StageArgs S)
{
    // blockIdx.x = (k2, pass, par): pass 0 = Y half (f0 on the second axis,
    // f1 on the first, minus sign), pass 1 = X half; par = parity of the rows g1
    // this workgroup owns (step C of (k1, l1) reads rows of parity k1+l1+1 only).
    typedef typename A::T R;
    const int M = T.M, K = T.K, GM = T.GM, KG = T.KG, M1 = M + 1;
    const int N = B.N;
    const int j = blockIdx.y;
    const int k2 = blockIdx.x >> 2, pass = (blockIdx.x >> 1) & 1, par = blockIdx.x & 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int rows = GM + 1;  // rows * M1 == KG
    const int nrp = (rows - par + 1) / 2;  // rows of this parity

    // LDS: sA [K] signed alpha; R1 [KG] S (step A) then T (steps B, C);
    //      R2 [KG] Y (step A -> B); sG [M1*M1] partial per (k1, l1); sF [M1*M1] factor slice
    extern __shared__ double smem[];
    R* sA = reinterpret_cast<R*>(smem);
    R* R1 = sA + K;
    R* R2 = R1 + KG;
    R* sG = R2 + KG;
    R* sF = sG + M1 * M1;
    __shared__ double red[16];
    __shared__ int is_last;

    const double* al = B.alpha[S.cur] + (long)j * K;
    for (int l = tid; l < K; l += nt) {
        int s = shell_of(l);
        sA[l] = A::mk((s & 1) ? -al[l] : al[l]);
    }
    const double* ssh = B.s_self + (long)j * KG;
    const double* ssl = B.s_self_lo ? B.s_self_lo + (long)j * KG : nullptr;
    const double* sp = N > 1 ? B.s_pair + (long)j * KG : nullptr;
    for (int g = tid; g < KG; g += nt) {
        R v = ssl ? A::ld(ssh, ssl, g) : A::mk(ssh[g]);
        if (sp) v = A::add(v, A::mk(sp[g]));
        R1[g] = v;
    }
    const double* fh = pass == 0 ? T.f0_hi : T.f1_hi;
    const double* fl = pass == 0 ? T.f0_lo : T.f1_lo;
    const long fbase = (long)k2 * M1 * M1;
    if (FSLICE)
        for (int i = tid; i < M1 * M1; i += nt) sF[i] = A::ld(fh + fbase, fl + fbase, i);
    __syncthreads();
    // (A) second axis on the rows of parity par
    for (int task = tid; task < nrp * M1; task += nt) {
        const int rr = task / M1, l2 = task - rr * M1;
        const int g1 = par + 2 * rr;
        R acc = A::zero();
        const int imax = pass == 0 ? (l2 < k2 ? l2 : k2) : (l2 < k2 - 1 ? l2 : k2 - 1);
        const int off = pass == 0 ? 1 : -1;
        for (int i = 0; i <= imax; ++i) {
            const int g2 = k2 + l2 - 2 * i + off;
            const int gg = g1 + g2;
            if (gg > GM || gg == 0) continue;
            const R f = FSLICE ? sF[l2 * M1 + i] : A::ld(fh + fbase, fl + fbase, l2 * M1 + i);
            acc = A::madd(acc, f, R1[ctri(g1, g2)]);
        }
        R2[g1 * M1 + l2] = acc;
    }
    __syncthreads();
    // (B) T[g1][l1] = sum_{l2 <= M - l1} sA[l1, l2] Y[g1][l2], register-blocked 4 x 4
    {
        const int nbg = (nrp + 3) / 4, nbl = (M1 + 3) / 4;
        for (int blk = tid; blk < nbg * nbl; blk += nt) {
            const int bg = blk / nbl, bl = blk - bg * nbl;
            const int r0 = bg * 4, l0 = bl * 4;
            R acc[4][4];
            for (int u = 0; u < 4; ++u)
                for (int v = 0; v < 4; ++v) acc[u][v] = A::zero();
            const int l2max = M - l0;
            for (int l2 = 0; l2 <= l2max; ++l2) {
                R y[4], a4[4];
                for (int u = 0; u < 4; ++u)
                    y[u] = (r0 + u < nrp) ? R2[(par + 2 * (r0 + u)) * M1 + l2] : A::zero();
                for (int v = 0; v < 4; ++v) {
                    const int l1 = l0 + v;
                    a4[v] = (l1 <= M && l1 + l2 <= M) ? sA[ctri(l1, l2)] : A::zero();
                }
                for (int u = 0; u < 4; ++u)
                    for (int v = 0; v < 4; ++v) acc[u][v] = A::madd(acc[u][v], a4[v], y[u]);
            }
            for (int u = 0; u < 4; ++u)
                for (int v = 0; v < 4; ++v)
                    if (r0 + u < nrp && l0 + v <= M) R1[(par + 2 * (r0 + u)) * M1 + l0 + v] = acc[u][v];
        }
    }
    __syncthreads();
    // (C) first axis for the (k1, l1) whose rows have parity par
    const int nk1 = M - k2 + 1;
    for (int task = tid; task < nk1 * M1; task += nt) {
        const int k1 = task / M1, l1 = task - k1 * M1;
        R acc = A::zero();
        if (((k1 + l1 + 1) & 1) == par) {
            const long fo = ((long)k1 * M1 + l1) * M1;
            if (pass == 0) {
                // - sum_i f1[k1][l1][i] T[k1+l1-2i-1][l1]
                const int imax = l1 < k1 - 1 ? l1 : k1 - 1;
                for (int i = 0; i <= imax; ++i)
                    acc = A::madd(acc, A::ld(T.f1_hi, T.f1_lo, fo + i), R1[(k1 + l1 - 2 * i - 1) * M1 + l1]);
                acc = A::neg(acc);
            } else {
                // + sum_i f0[k1][l1][i] T[k1+l1-2i+1][l1]
                const int imax = l1 < k1 ? l1 : k1;
                for (int i = 0; i <= imax; ++i) {
                    const int g1 = k1 + l1 - 2 * i + 1;
                    if (g1 > GM) continue;
                    acc = A::madd(acc, A::ld(T.f0_hi, T.f0_lo, fo + i), R1[g1 * M1 + l1]);
                }
            }
        }
        sG[task] = acc;
    }
    __syncthreads();
    // partial over l1 for every k1 of this k2 -> global (hi, lo)
    double* gp = B.gpart + ((long)j * 4 + (pass * 2 + par)) * K * 2;
    for (int k1 = tid; k1 < nk1; k1 += nt) {
        R g = A::zero();
        for (int l1 = 0; l1 <= M; ++l1) g = A::add(g, sG[k1 * M1 + l1]);
        const int k = ctri(k1, k2);
        A::st(gp + 2 * k, g);
    }
    // the last of the 4 (M+1) workgroups of this vortex finishes the stage
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const unsigned total = 4u * (unsigned)M1;
        is_last = atomicAdd(B.done + j, 1u) == total - 1u;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    const double lam2 = B.lam2[S.cur][j];
    const double lam = sqrt(lam2);
    const double lam2n = B.lam0sq[j] + 4.0 * S.nu * S.t_next;
    double xd1 = 0.0, xd2 = 0.0;
    if (N > 1) centre_velocity(al, sp, K, lam, red, xd1, xd2);
    const double* gj = B.gpart + (long)j * 4 * K * 2;
    for (int k = tid; k < K; k += nt) {
        R g = A::zero();
        for (int q = 0; q < 4; ++q) g = A::add(g, A::ldst(gj + ((long)q * K + k) * 2));
        const int s = shell_of(k);
        const int kk2 = k - s * (s + 1) / 2, k1 = s - kk2;
        double lp = 1.0;  // lambda^{s-2}
        for (int e = 0; e < s; ++e) lp *= lam;
        lp /= lam2;
        double val = A::hi(A::madd(A::zero(), A::ld(T.c1_hi, T.c1_lo, k), g)) * lp;
        if (N > 1) {  // drift, eq:last_termsimp: xdot_1 M_{k-e1} + xdot_2 M_{k-e2}
            double lq = lp * lam;  // lambda^{s-1}
            if (k1 >= 1) val += xd1 * al[ctri(k1 - 1, kk2)] * lq;
            if (kk2 >= 1) val += xd2 * al[ctri(k1, kk2 - 1)] * lq;
        }
        if (k == 0) val = 0.0;  // circulation is conserved exactly
        emit_moment(B, S, j, k, s, K, val, lam2n);
    }
    if (tid == 0) {
        emit_position(B, S, j, xd1, xd2, lam2n);
        B.done[j] = 0u;  // ready for the next launch
    }
}

// ---------------------------------------------------------------------------
// stage 2 for small orders (M <= kMaxSmallOrder): one workgroup per vortex
// computes its self table, then all k2 and both halves of the contraction at
// once (four barriers per stage), then the drift and the RK4 update.
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(1024) void k_stage2_small(DevTables T, StageBufs B, StageArgs S)
{
    constexpr int K = (M + 1) * (M + 2) / 2;
    constexpr int GM = M == 0 ? 1 : 2 * M;
    constexpr int KG = (GM + 1) * (GM + 2) / 2;
    constexpr int M1 = M + 1;
    constexpr int NY = 2 * M1 * KG;  // (pass, k2, g1, l2)
    extern __shared__ double smem[];
    double* sAl = smem;        // [K] alpha
    double* sA = sAl + K;      // [K] (-1)^{|l|} alpha
    double* sS = sA + K;       // [KG] S_self + S_pair
    double* sY = sS + KG;      // [NY]
    double* sT = sY + NY;      // [NY]
    double* sP = sT + NY;      // [2][K][M1] partials of step C
    double* sF0 = sP + 2 * K * M1;      // [M1^3] factor table f0
    double* sF1 = sF0 + M1 * M1 * M1;   // [M1^3] factor table f1
    double* sT0 = sF1 + M1 * M1 * M1;   // [tri(T0N)] Psi0 table
    __shared__ double red[32];

    const int N = B.N, j = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const double* al = B.alpha[S.cur] + (long)j * K;
    for (int l = tid; l < K; l += nt) {
        const double a = al[l];
        sAl[l] = a;
        sA[l] = (shell_of(l) & 1) ? -a : a;
    }
    const double lam2 = B.lam2[S.cur][j];
    const double lam = sqrt(lam2);
    const double lam2n = B.lam0sq[j] + 4.0 * S.nu * S.t_next;
    const double* sp = N > 1 ? B.s_pair + (long)j * KG : nullptr;
    for (int i = tid; i < M1 * M1 * M1; i += nt) {
        sF0[i] = T.f0_hi[i];
        sF1[i] = T.f1_hi[i];
    }
    const int nt0 = (T.T0N + 1) * (T.T0N + 2) / 2;
    for (int i = tid; i < nt0; i += nt) sT0[i] = T.t0_hi[i];
    __syncthreads();
    // self table S_self[g] = sum_m alpha_m Psi0(m + g) (c = 2), plus the pair table
    for (int g = tid; g < KG; g += nt) {
        double acc = 0.0;
        if (g > 0) {
            const int gs = shell_of(g);
            const int g2 = g - gs * (gs + 1) / 2, g1 = gs - g2;
            for (int m2 = g2 & 1; m2 <= M; m2 += 2)
                for (int m1 = g1 & 1; m1 + m2 <= M; m1 += 2)
                    acc = fma(sAl[ctri(m1, m2)], sT0[ctri((m1 + g1) >> 1, (m2 + g2) >> 1)], acc);
            if (sp) acc += sp[g];
        }
        sS[g] = acc;
    }
    double xd1 = 0.0, xd2 = 0.0;
    if (N > 1) centre_velocity(sAl, sp, K, lam, red, xd1, xd2);
    __syncthreads();
    // (A) second axis for every (pass, k2, g1, l2)
    for (int task = tid; task < NY; task += nt) {
        const int pass = task / (M1 * KG);
        const int r = task - pass * (M1 * KG);
        const int k2 = r / KG, q = r - k2 * KG;
        const int g1 = q / M1, l2 = q - g1 * M1;
        const double* f = (pass == 0 ? sF0 : sF1) + (k2 * M1 + l2) * M1;
        const int imax = pass == 0 ? (l2 < k2 ? l2 : k2) : (l2 < k2 - 1 ? l2 : k2 - 1);
        const int off = pass == 0 ? 1 : -1;
        double acc = 0.0;
        for (int i = 0; i <= imax; ++i) {
            const int g2 = k2 + l2 - 2 * i + off;
            const int gg = g1 + g2;
            if (gg > GM || gg == 0) continue;
            acc = fma(f[i], sS[ctri(g1, g2)], acc);
        }
        sY[task] = acc;
    }
    __syncthreads();
    // (B) l2 against the moments for every (pass, k2, g1, l1)
    for (int task = tid; task < NY; task += nt) {
        const int base = task - task % M1;  // (pass, k2, g1) row start
        const int l1 = task - base;
        double acc = 0.0;
        for (int l2 = 0; l2 <= M - l1; ++l2) acc = fma(sA[ctri(l1, l2)], sY[base + l2], acc);
        sT[task] = acc;
    }
    __syncthreads();
    // (C) first axis for every (pass, k, l1)
    for (int task = tid; task < 2 * K * M1; task += nt) {
        const int pass = task / (K * M1);
        const int r = task - pass * (K * M1);
        const int k = r / M1, l1 = r - k * M1;
        const int ks = shell_of(k);
        const int k2 = k - ks * (ks + 1) / 2, k1 = ks - k2;
        const double* tcol = sT + (long)(pass * M1 + k2) * KG + l1;
        double acc = 0.0;
        if (pass == 0) {
            const double* f = sF1 + (k1 * M1 + l1) * M1;
            const int imax = l1 < k1 - 1 ? l1 : k1 - 1;
            for (int i = 0; i <= imax; ++i) acc = fma(f[i], tcol[(k1 + l1 - 2 * i - 1) * M1], acc);
            acc = -acc;
        } else {
            const double* f = sF0 + (k1 * M1 + l1) * M1;
            const int imax = l1 < k1 ? l1 : k1;
            for (int i = 0; i <= imax; ++i) {
                const int g1 = k1 + l1 - 2 * i + 1;
                if (g1 <= GM) acc = fma(f[i], tcol[g1 * M1], acc);
            }
        }
        sP[task] = acc;
    }
    __syncthreads();
    for (int k = tid; k < K; k += nt) {
        double g = 0.0;
        for (int l1 = 0; l1 < M1; ++l1) g += sP[k * M1 + l1] + sP[(K + k) * M1 + l1];
        const int s = shell_of(k);
        const int k2 = k - s * (s + 1) / 2, k1 = s - k2;
        double lp = 1.0;
        for (int e = 0; e < s; ++e) lp *= lam;
        lp /= lam2;
        double val = T.c1_hi[k] * g * lp;
        if (N > 1) {
            const double lq = lp * lam;
            if (k1 >= 1) val += xd1 * sAl[ctri(k1 - 1, k2)] * lq;
            if (k2 >= 1) val += xd2 * sAl[ctri(k1, k2 - 1)] * lq;
        }
        if (k == 0) val = 0.0;
        emit_moment(B, S, j, k, s, K, val, lam2n);
    }
    if (tid == 0) emit_position(B, S, j, xd1, xd2, lam2n);
}

bool stage2_fuses_self(int M, bool dd) { return !dd && M <= kMaxSmallOrder; }

template <int M>
static hipError_t launch_small(const DevTables& T, const StageBufs& B, const StageArgs& A, hipStream_t st)
{
    constexpr int K = (M + 1) * (M + 2) / 2;
    constexpr int GM = M == 0 ? 1 : 2 * M;
    constexpr int KG = (GM + 1) * (GM + 2) / 2;
    constexpr int M1 = M + 1;
    const int nt0 = (T.T0N + 1) * (T.T0N + 2) / 2;
    const size_t shmem = sizeof(double) * (2 * K + KG + 4 * (size_t)M1 * KG + 2 * (size_t)K * M1 +
                                           2 * (size_t)M1 * M1 * M1 + (size_t)nt0);
    // few vortices: wide workgroups for latency; many: one to four wavefronts each
    int threads = B.N <= 32 ? 1024 : (2 * M1 * KG >= 1024 ? 256 : (2 * M1 * KG >= 256 ? 128 : 64));
    if (shmem > 64 * 1024) {
        hipError_t ea = hipFuncSetAttribute((const void*)k_stage2_small<M>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (ea != hipSuccess) {
            (void)hipGetLastError();
            report_hip_error(ea, "hipFuncSetAttribute(k_stage2_small dynamic LDS)");
            return ea;
        }
    }
    hipLaunchKernelGGL(k_stage2_small<M>, dim3(B.N), dim3(threads), shmem, st, T, B, A);
    return hipGetLastError();
}

hipError_t launch_stage2(const DevTables& T, const StageBufs& B, const StageArgs& A, bool use_dd, hipStream_t st)
{
    if (stage2_fuses_self(T.M, use_dd)) {
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
    const int threads = 512;
    const size_t elem = use_dd ? sizeof(dd) : sizeof(double);
    // the factor slice goes to LDS when it fits (FP64 always does)
    const size_t base = (size_t)T.K + 2 * (size_t)T.KG + (size_t)M1 * M1;
    const bool fslice = (base + (size_t)M1 * M1) * elem <= 150 * 1024;
    const size_t shmem = elem * (base + (fslice ? (size_t)M1 * M1 : 0));
    const void* fn = use_dd ? (fslice ? (const void*)k_stage2<ArithDD, true> : (const void*)k_stage2<ArithDD, false>)
                            : (fslice ? (const void*)k_stage2<ArithF64, true> : (const void*)k_stage2<ArithF64, false>);
    if (shmem > 64 * 1024) {
        // large orders stage up to ~150 KB of LDS
        hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (ea != hipSuccess) {
            (void)hipGetLastError();
            report_hip_error(ea, "hipFuncSetAttribute(k_stage2 dynamic LDS)");
            return ea;
        }
    }
    dim3 grid(4 * M1, B.N);
    if (use_dd) {
        if (fslice) hipLaunchKernelGGL((k_stage2<ArithDD, true>), grid, dim3(threads), shmem, st, T, B, A);
        else hipLaunchKernelGGL((k_stage2<ArithDD, false>), grid, dim3(threads), shmem, st, T, B, A);
    } else {
        if (fslice) hipLaunchKernelGGL((k_stage2<ArithF64, true>), grid, dim3(threads), shmem, st, T, B, A);
        else hipLaunchKernelGGL((k_stage2<ArithF64, false>), grid, dim3(threads), shmem, st, T, B, A);
    }
    return hipGetLastError();
}

}  // namespace mmvm
