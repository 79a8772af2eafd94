// Adaptive time stepping with the Dormand-Prince 5(4) pair: the integrator of
// the paper's ode45 runs ("A note on implementation and performance", RelTol =
// AbsTol = 1e-8), on the state y = (x^j, M^j) in physical time.
//
// The right-hand sides run through the library's stage kernels (prep, self,
// pair, stage 2, emit) in RHS mode; the stage combinations
// y + h sum_j a_ij k_j and the weighted RMS error norm are kernels over the
// flat state; the host reads the norm once per step (one small copy into
// pinned memory) and applies the step-size controller:
//   err = RMS_n(e_n / (atol + rtol max(|y_n|, |y_new,n|))),  e = h sum_i (b_i - b*_i) k_i;
//   err < 1: accept, h *= min(10, 0.9 err^(-1/5)) (no growth right after a
//   rejection); else reject, h *= max(0.2, 0.9 err^(-1/5)); the last step ends
//   exactly at t1; the seventh stage f(t + h, y_new) is the next step's first.
// Tableau of Dormand & Prince (1980).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "../../include/mmvm.h"
#include "api_internal.hpp"

namespace mmvm {
namespace {

constexpr double kC[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
constexpr double kA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
// b - b* (fifth minus fourth order weights)
constexpr double kE[7] = {35.0 / 384 - 5179.0 / 57600, 0.0, 500.0 / 1113 - 7571.0 / 16695,
                          125.0 / 192 - 393.0 / 640, -2187.0 / 6784 + 92097.0 / 339200,
                          11.0 / 84 - 187.0 / 2100, -1.0 / 40};

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;

struct Coef {
    double a[7];
};

// out = y + h sum_{j < s} a_j k_j over the flat state of n values
__global__ __launch_bounds__(kThreads) void k_dp_combine(long n, const double* __restrict__ y,
                                                         const double* __restrict__ k, int s, Coef c, double h,
                                                         double* __restrict__ out)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int j = 0; j < s; ++j) v += c.a[j] * k[(long)j * n + i];
        out[i] = y[i] + h * v;
    }
}

// partial sums of (e_n / scale_n)^2 per block (block sums in a fixed order)
__global__ __launch_bounds__(kThreads) void k_dp_error(long n, const double* __restrict__ y,
                                                       const double* __restrict__ yn,
                                                       const double* __restrict__ k, Coef e, double h, double rtol,
                                                       double atol, double* __restrict__ part)
{
    __shared__ double red[kThreads / 64];
    double ss = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int j = 0; j < 7; ++j) v += e.a[j] * k[(long)j * n + i];
        v *= h;
        const double sc = atol + fmax(fabs(y[i]), fabs(yn[i])) * rtol;
        const double q = v / sc;
        ss = fma(q, q, ss);
    }
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += red[w];
        part[blockIdx.x] = t;
    }
}

__global__ void k_dp_sum(int nb, const double* __restrict__ part, double* __restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += part[b];
        *out = t;
    }
}

// per (device, stream): y, y_new, stage input, seven stages, partial sums; a pinned word
struct DPWS {
    char* base = nullptr;
    size_t bytes = 0;
    double* host = nullptr;
};
std::mutex g_dmu;
std::map<std::pair<int, hipStream_t>, DPWS> g_dws;

size_t up256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace
}  // namespace mmvm

using namespace mmvm;

extern "C" mmvm_status mmvm_integrate_adaptive(const mmvm_problem* prob, double t0, double t1, double rtol,
                                               double atol, double h0, double* x, double* mom, mmvm_precision prec,
                                               void* stream, mmvm_adaptive_stats* stats)
{
    mmvm_status s = validate(prob);
    if (s != MMVM_OK) return s;
    if (!x || !mom || !std::isfinite(t0) || !std::isfinite(t1) || !(t1 >= t0) || !(rtol >= 0.0) ||
        !std::isfinite(rtol) || !(atol > 0.0) || !std::isfinite(atol) || !(h0 > 0.0) || !std::isfinite(h0))
        return MMVM_EINVAL;
    if (prec != MMVM_FP64 && prec != MMVM_MIXED) return MMVM_EINVAL;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (t1 == t0) return MMVM_OK;
    const int N = prob->n, M = prob->order, K = (M + 1) * (M + 2) / 2;
    hipStream_t st = (hipStream_t)stream;
    const DevTables* T = nullptr;
    if ((s = device_tables(M, &T)) != MMVM_OK) return s;
    Workspace* W = workspace_for(st);
    if (!W) return MMVM_EDEVICE;
    std::lock_guard<std::mutex> lk(W->mu);
    if ((s = W->ensure(N, M, use_dd(M, prec), N == 1, st)) != MMVM_OK) return s;
    if ((s = W->set_params(prob->lambda0, nullptr, prob->nu, N, st)) != MMVM_OK) return s;

    const long n = 2L * N + (long)N * K;
    const size_t vb = up256(sizeof(double) * (size_t)n);
    const size_t need = 3 * vb + 7 * vb + up256(sizeof(double) * (kMaxBlocks + 1));
    DPWS* D = nullptr;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return MMVM_EDEVICE;
        std::lock_guard<std::mutex> lk2(g_dmu);
        D = &g_dws[std::make_pair(dev, st)];
        if (!D->host && hipHostMalloc((void**)&D->host, sizeof(double), hipHostMallocDefault) != hipSuccess) {
            D->host = nullptr;
            return MMVM_ENOMEM;
        }
        if (need > D->bytes) {
            if (D->base) {
                if (hipStreamSynchronize(st) != hipSuccess) return MMVM_EDEVICE;
                (void)hipFree(D->base);
            }
            D->base = nullptr;
            D->bytes = 0;
            if (hipMalloc((void**)&D->base, need) != hipSuccess) return MMVM_ENOMEM;
            D->bytes = need;
        }
    }
    double* y = (double*)D->base;
    double* yn = (double*)(D->base + vb);
    double* ys = (double*)(D->base + 2 * vb);
    double* k = (double*)(D->base + 3 * vb);  // seven stages of n values (contiguous: k[j * n + i])
    double* part = (double*)(D->base + 10 * vb);
    double* norm = part + kMaxBlocks;
    const int nb = (int)std::min<long>((n + kThreads - 1) / kThreads, kMaxBlocks);

    // right-hand side of the state at ystate, time t, into stage j
    auto rhs = [&](const double* ystate, double t, int j) -> mmvm_status {
        StageArgs A;
        std::memset(&A, 0, sizeof(A));
        A.mode = MODE_RHS;
        A.cur = 0;
        A.t_stage = t;
        A.t_next = t;
        A.dx = k + (long)j * n;
        A.dmom = k + (long)j * n + 2L * N;
        mmvm_status r = run_prep(*T, *W, 0, ystate, ystate + 2L * N, t, prec, st);
        if (r == MMVM_OK) r = run_stage(*T, *W, prec, A, st);
        if (stats) ++stats->rhs_evals;
        return r;
    };
    if (hipMemcpyAsync(y, x, sizeof(double) * 2 * (size_t)N, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(y + 2 * N, mom, sizeof(double) * (size_t)N * K, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return MMVM_EDEVICE;
    if ((s = rhs(y, t0, 0)) != MMVM_OK) return s;
    double t = t0, habs = h0;
    Coef ce;
    for (int j = 0; j < 7; ++j) ce.a[j] = kE[j];
    while (t < t1) {
        bool rejected = false;
        for (;;) {
            double tn = t + habs;
            if (tn > t1) tn = t1;
            const double h = tn - t;
            habs = h;
            if (!(h > 0.0)) return MMVM_EINVAL;  // the step fell below the resolution of t
            for (int st_i = 1; st_i < 7; ++st_i) {
                Coef c{};
                for (int j = 0; j < st_i; ++j) c.a[j] = kA[st_i][j];
                double* out = st_i == 6 ? yn : ys;
                hipLaunchKernelGGL(k_dp_combine, dim3(nb), dim3(kThreads), 0, st, n, (const double*)y,
                                   (const double*)k, st_i, c, h, out);
                if ((s = rhs(out, t + kC[st_i] * h, st_i)) != MMVM_OK) return s;
            }
            hipLaunchKernelGGL(k_dp_error, dim3(nb), dim3(kThreads), 0, st, n, (const double*)y, (const double*)yn,
                               (const double*)k, ce, h, rtol, atol, part);
            hipLaunchKernelGGL(k_dp_sum, dim3(1), dim3(64), 0, st, nb, (const double*)part, norm);
            if (hipMemcpyAsync(D->host, norm, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return MMVM_EDEVICE;
            const double err = std::sqrt(*D->host / (double)n);
            if (!std::isfinite(err)) return MMVM_ENONFINITE;
            if (err < 1.0) {
                double fac = err == 0.0 ? 10.0 : 0.9 * std::pow(err, -0.2);
                if (fac > 10.0) fac = 10.0;
                if (rejected && fac > 1.0) fac = 1.0;
                habs *= fac;
                t = tn;
                // accepted: y <- y_new, the seventh stage becomes the first
                if (hipMemcpyAsync(y, yn, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                    hipMemcpyAsync(k, k + 6 * n, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st) !=
                        hipSuccess)
                    return MMVM_EDEVICE;
                if (stats) ++stats->accepted;
                break;
            }
            double fac = 0.9 * std::pow(err, -0.2);
            if (fac < 0.2) fac = 0.2;
            habs *= fac;
            rejected = true;
            if (stats) ++stats->rejected;
        }
    }
    if (stats) stats->h_next = habs;
    if (hipMemcpyAsync(x, y, sizeof(double) * 2 * (size_t)N, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(mom, y + 2 * N, sizeof(double) * (size_t)N * K, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return MMVM_EDEVICE;
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MMVM_OK : MMVM_EDEVICE;
}
