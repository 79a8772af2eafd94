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
__global__ __launch_bounds__(256) void k_prep(int N, int K, const double* __restrict__ xin,
                                              const double* __restrict__ min_, const double* __restrict__ lam0sq,
                                              double t, double nu, double* __restrict__ xs, double* __restrict__ ys,
                                              double* __restrict__ lam2, double* __restrict__ alpha,
                                              double* __restrict__ alphaT, float* __restrict__ alphaT32,
                                              int* __restrict__ flag, int copy_state)
{
    const long total = (long)N * K;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        int j = (int)(idx / K), k = (int)(idx - (long)j * K);
        double l2 = lam0sq[j] + 4.0 * nu * t;
        int s = shell_of(k);
        double il = 1.0 / sqrt(l2), p = 1.0;
        for (int e = 0; e < s; ++e) p *= il;
        double mk = min_[idx];
        double a = mk * p;
        if (copy_state) ys[idx] = mk;
        alpha[idx] = a;
        if (alphaT) alphaT[(long)k * N + j] = a;
        if (alphaT32) alphaT32[(long)k * N + j] = (float)a;
        if (!isfinite(mk)) atomicOr(flag, 2);
        if (k == 0) {
            lam2[j] = l2;
            double x0 = xin[2 * j], x1 = xin[2 * j + 1];
            if (copy_state) {
                xs[2 * j] = x0;
                xs[2 * j + 1] = x1;
            }
            if (N > 1 && mk == 0.0) atomicOr(flag, 1);
            if (!isfinite(x0) || !isfinite(x1)) atomicOr(flag, 2);
        }
    }
}

hipError_t launch_prep(const DevTables& T, const StageBufs& B, const double* xin, const double* min_,
                       double t, double nu, bool need_pair, bool need_f32, hipStream_t st)
{
    long total = (long)B.N * T.K;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    bool copy = (min_ != B.ys);
    hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(256), 0, st, B.N, T.K, xin, min_, B.lam0sq, t, nu, B.xs,
                       B.ys, B.lam2, B.alpha, need_pair && !need_f32 ? B.alphaT : (double*)nullptr,
                       need_pair && need_f32 ? B.alphaT32 : (float*)nullptr, B.flag, copy ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// self velocity-derivative table: S_self[j][g] = sum_m alpha_m Psi0(m + g), c = 2
// (the target's own Gaussian convolved with itself: Lambda^2 = 2 lambda^2).
// Psi0 is nonzero only for even-even arguments.
// ---------------------------------------------------------------------------
template <bool DD>
__global__ __launch_bounds__(256) void k_self(int N, int M, int K, int GM, int KG, const double* __restrict__ alpha,
                                              const double* __restrict__ t0h, const double* __restrict__ t0l,
                                              double* __restrict__ sself, double* __restrict__ sself_lo)
{
    int j = blockIdx.y;
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= KG) return;
    if (g == 0) {
        sself[(long)j * KG] = 0.0;
        if (DD) sself_lo[(long)j * KG] = 0.0;
        return;
    }
    int gs = shell_of(g);
    int g2 = g - gs * (gs + 1) / 2, g1 = gs - g2;
    const double* a = alpha + (long)j * K;
    if constexpr (!DD) {
        double acc = 0.0;
        for (int m2 = g2 & 1; m2 <= M; m2 += 2)
            for (int m1 = g1 & 1; m1 + m2 <= M; m1 += 2)
                acc = fma(a[ctri(m1, m2)], t0h[ctri((m1 + g1) >> 1, (m2 + g2) >> 1)], acc);
        sself[(long)j * KG + g] = acc;
    } else {
        dd acc = dd_make(0.0);
        for (int m2 = g2 & 1; m2 <= M; m2 += 2)
            for (int m1 = g1 & 1; m1 + m2 <= M; m1 += 2) {
                int ti = ctri((m1 + g1) >> 1, (m2 + g2) >> 1);
                acc = dd_add(acc, dd_mul(dd_make(t0h[ti], t0l[ti]), dd_make(a[ctri(m1, m2)])));
            }
        sself[(long)j * KG + g] = acc.hi;
        sself_lo[(long)j * KG + g] = acc.lo;
    }
}

hipError_t launch_self(const DevTables& T, const StageBufs& B, bool dd, hipStream_t st)
{
    dim3 grid((T.KG + 127) / 128, B.N);
    if (dd)
        hipLaunchKernelGGL(k_self<true>, grid, dim3(128), 0, st, B.N, T.M, T.K, T.GM, T.KG, B.alpha, T.t0_hi,
                           T.t0_lo, B.s_self, B.s_self_lo);
    else
        hipLaunchKernelGGL(k_self<false>, grid, dim3(128), 0, st, B.N, T.M, T.K, T.GM, T.KG, B.alpha, T.t0_hi,
                           T.t0_lo, B.s_self, (double*)nullptr);
    return hipGetLastError();
}

template <int M>
hipError_t launch_pair_M(const DevTables& T, const StageBufs& B, bool f32, hipStream_t st);

bool pair_order_supported(int M) { return M >= 0 && M <= kMaxPairOrder; }

hipError_t launch_pair(const DevTables& T, const StageBufs& B, bool f32, int, hipStream_t st)
{
    switch (T.M) {
    case 0: return launch_pair_M<0>(T, B, f32, st);
    case 1: return launch_pair_M<1>(T, B, f32, st);
    case 2: return launch_pair_M<2>(T, B, f32, st);
    case 3: return launch_pair_M<3>(T, B, f32, st);
    case 4: return launch_pair_M<4>(T, B, f32, st);
    case 5: return launch_pair_M<5>(T, B, f32, st);
    case 6: return launch_pair_M<6>(T, B, f32, st);
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
};

template <class A>
__global__ __launch_bounds__(256) void k_stage2(DevTables T, StageBufs B, StageArgs S, int nslab)
{
    typedef typename A::T R;
    const int M = T.M, K = T.K, GM = T.GM, KG = T.KG, M1 = M + 1;
    const int N = B.N;
    const int j = blockIdx.y, slab = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int rows = GM + 1;

    extern __shared__ double smem[];
    R* sA = reinterpret_cast<R*>(smem);  // K: (-1)^{|l|} alpha_l
    R* sY = sA + K;                      // rows x M1
    R* sT = sY + rows * M1;              // rows x M1
    R* sG = sT + rows * M1;              // M1 x M1
    __shared__ double red[8];

    const double* al = B.alpha + (long)j * K;
    for (int l = tid; l < K; l += nt) {
        int s = shell_of(l);
        sA[l] = A::mk((s & 1) ? -al[l] : al[l]);
    }
    const double lam2 = B.lam2[j];
    const double lam = sqrt(lam2);

    // S = S_self + S_pair (global; L2-resident, ~KG values per vortex)
    const double* ssh = B.s_self + (long)j * KG;
    const double* ssl = B.s_self_lo ? B.s_self_lo + (long)j * KG : nullptr;
    const double* sp = N > 1 ? B.s_pair + (long)j * KG : nullptr;
    auto Sget = [&](int g1, int g2) -> R {
        int g = ctri(g1, g2);
        R v = ssl ? A::ld(ssh, ssl, g) : A::mk(ssh[g]);
        if (sp) v = A::add(v, A::mk(sp[g]));
        return v;
    };

    // centre velocity (eq:xjdot_Final):
    //   xdot_1 = -(1/(Gamma lambda)) sum_m (-1)^{|m|} alpha_m S_pair[m + e2]
    //   xdot_2 = +(1/(Gamma lambda)) sum_m (-1)^{|m|} alpha_m S_pair[m + e1]
    double xd1 = 0.0, xd2 = 0.0;
    if (N > 1) {
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
    __syncthreads();

    for (int k2 = slab; k2 <= M; k2 += nslab) {
        const int nk1 = M - k2 + 1;
        for (int pass = 0; pass < 2; ++pass) {
            // (A) second axis: pass 0 -> Y-part (f0), pass 1 -> X-part (f1)
            for (int task = tid; task < rows * M1; task += nt) {
                int g1 = task / M1, l2 = task - g1 * M1;
                R acc = A::zero();
                if (pass == 0) {
                    int imax = l2 < k2 ? l2 : k2;
                    for (int i = 0; i <= imax; ++i) {
                        int g2 = k2 + l2 - 2 * i + 1;
                        if (g1 + g2 > GM) continue;
                        long o = ((long)k2 * M1 + l2) * M1 + i;
                        acc = A::madd(acc, A::ld(T.f0_hi, T.f0_lo, o), Sget(g1, g2));
                    }
                } else {
                    int imax = l2 < k2 - 1 ? l2 : k2 - 1;
                    for (int i = 0; i <= imax; ++i) {
                        int g2 = k2 + l2 - 2 * i - 1;
                        if (g1 + g2 > GM || g1 + g2 == 0) continue;
                        long o = ((long)k2 * M1 + l2) * M1 + i;
                        acc = A::madd(acc, A::ld(T.f1_hi, T.f1_lo, o), Sget(g1, g2));
                    }
                }
                sY[task] = acc;
            }
            __syncthreads();
            // (B) l2 against the moments: T[g1][l1] = sum_{l2 <= M - l1} sA[l1, l2] Y[g1][l2]
            for (int task = tid; task < rows * M1; task += nt) {
                int g1 = task / M1, l1 = task - g1 * M1;
                R acc = A::zero();
                for (int l2 = 0; l2 <= M - l1; ++l2) acc = A::madd(acc, sA[ctri(l1, l2)], sY[g1 * M1 + l2]);
                sT[task] = acc;
            }
            __syncthreads();
            // (C) first axis, partial per (k1, l1)
            for (int task = tid; task < nk1 * M1; task += nt) {
                int k1 = task / M1, l1 = task - k1 * M1;
                R acc = A::zero();
                if (pass == 0) {
                    // - sum_i f1[k1][l1][i] T[k1+l1-2i-1][l1]
                    int imax = l1 < k1 - 1 ? l1 : k1 - 1;
                    for (int i = 0; i <= imax; ++i) {
                        int g1 = k1 + l1 - 2 * i - 1;
                        long o = ((long)k1 * M1 + l1) * M1 + i;
                        acc = A::madd(acc, A::ld(T.f1_hi, T.f1_lo, o), sT[g1 * M1 + l1]);
                    }
                    sG[task] = A::neg(acc);
                } else {
                    // + sum_i f0[k1][l1][i] T[k1+l1-2i+1][l1]
                    int imax = l1 < k1 ? l1 : k1;
                    for (int i = 0; i <= imax; ++i) {
                        int g1 = k1 + l1 - 2 * i + 1;
                        if (g1 > GM) continue;
                        long o = ((long)k1 * M1 + l1) * M1 + i;
                        acc = A::madd(acc, A::ld(T.f0_hi, T.f0_lo, o), sT[g1 * M1 + l1]);
                    }
                    sG[task] = A::add(sG[task], acc);
                }
            }
            __syncthreads();
        }
        // reduce over l1 and emit
        for (int k1 = tid; k1 < nk1; k1 += nt) {
            R g = A::zero();
            for (int l1 = 0; l1 <= M; ++l1) g = A::add(g, sG[k1 * M1 + l1]);
            const int k = ctri(k1, k2), s = k1 + k2;
            double lp = 1.0;  // lambda^{s-2}
            for (int e = 0; e < s; ++e) lp *= lam;
            lp /= lam2;
            double val = A::hi(A::madd(A::zero(), A::ld(T.c1_hi, T.c1_lo, k), g)) * lp;
            if (N > 1) {  // drift, eq:last_termsimp: xdot_1 M_{k-e1} + xdot_2 M_{k-e2}
                double lq = lp * lam;  // lambda^{s-1}
                if (k1 >= 1) val += xd1 * al[ctri(k1 - 1, k2)] * lq;
                if (k2 >= 1) val += xd2 * al[ctri(k1, k2 - 1)] * lq;
            }
            if (k == 0) val = 0.0;  // circulation is conserved exactly
            const long o = (long)j * K + k;
            if (S.mode == MODE_RHS) {
                S.dmom[o] = val;
            } else {
                const double wts[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
                const double cn[4] = {0.5, 0.5, 1.0, 0.0};
                const double yn = S.mom[o];
                if (S.stage == 0) B.accm[o] = wts[0] * val;
                else if (S.stage < 3) B.accm[o] += wts[S.stage] * val;
                if (S.stage < 3) {
                    B.ys[o] = yn + cn[S.stage] * S.dt * val;
                } else {
                    double ynew = yn + S.dt * (B.accm[o] + wts[3] * val);
                    S.mom[o] = ynew;
                    B.ys[o] = ynew;
                }
            }
        }
        __syncthreads();
    }

    if (slab == 0 && tid == 0) {
        if (S.mode == MODE_RHS) {
            S.dx[2 * j] = xd1;
            S.dx[2 * j + 1] = xd2;
        } else {
            const double wts[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
            const double cn[4] = {0.5, 0.5, 1.0, 0.0};
            for (int c = 0; c < 2; ++c) {
                const long o = 2 * j + c;
                const double v = c == 0 ? xd1 : xd2;
                const double yn = S.x[o];
                if (S.stage == 0) B.accx[o] = wts[0] * v;
                else if (S.stage < 3) B.accx[o] += wts[S.stage] * v;
                if (S.stage < 3) {
                    B.xs[o] = yn + cn[S.stage] * S.dt * v;
                } else {
                    double ynew = yn + S.dt * (B.accx[o] + wts[3] * v);
                    S.x[o] = ynew;
                    B.xs[o] = ynew;
                }
            }
        }
    }
}

hipError_t launch_stage2(const DevTables& T, const StageBufs& B, const StageArgs& A, bool use_dd, hipStream_t st)
{
    const int M1 = T.M + 1, rows = T.GM + 1;
    int work = rows * M1;
    int threads = work >= 256 ? 256 : ((work + 63) / 64) * 64;
    if (threads < 64) threads = 64;
    int nslab = T.M >= 10 ? M1 : 1;
    size_t elem = use_dd ? sizeof(dd) : sizeof(double);
    size_t shmem = elem * ((size_t)T.K + 2 * (size_t)rows * M1 + (size_t)M1 * M1);
    dim3 grid(nslab, B.N);
    if (shmem > 64 * 1024) {
        // large orders stage up to ~150 KB of LDS (double-double at order 40)
        const void* fn = use_dd ? (const void*)k_stage2<ArithDD> : (const void*)k_stage2<ArithF64>;
        hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (ea != hipSuccess) {
            (void)hipGetLastError();
            report_hip_error(ea, "hipFuncSetAttribute(k_stage2 dynamic LDS)");
            return ea;
        }
    }
    if (use_dd)
        hipLaunchKernelGGL(k_stage2<ArithDD>, grid, dim3(threads), shmem, st, T, B, A, nslab);
    else
        hipLaunchKernelGGL(k_stage2<ArithF64>, grid, dim3(threads), shmem, st, T, B, A, nslab);
    return hipGetLastError();
}

}  // namespace mmvm
