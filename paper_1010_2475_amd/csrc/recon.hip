// Vorticity reconstruction and non-axisymmetric enstrophy (the diagnostics of
// the section "Shear diffusion / Results"):
//   omega(x) = sum_j sum_{|k| <= M} M^j_k phi_k(x - x^j; lambda_j(t))   (eq:moment_expansion_def_tw0)
// with phi_{k1,k2} = D_1^{k1} D_2^{k2} phi00 (eq:Hermitedef), phi00 = exp(-|x|^2/lambda^2)/(pi lambda^2)
// (eq:phi00).  phi_k is separable: with h_a(u) = d^a/du^a exp(-u^2),
//   phi_k(x) = lambda^{-|k|} h_{k1}(x1/lambda) h_{k2}(x2/lambda) / (pi lambda^2),
// so on a grid omega[iy][ix] = sum_j sum_a X_j[a][ix] Y_j[a][iy], a dense
// product of inner dimension N (M + 1):
//   X_j[a][ix] = lambda_j^{-a} h_a((x_ix - x^j_1)/lambda_j) / (pi lambda_j^2),
//   Y_j[a][iy] = sum_{b <= M - a} M^j_{a,b} lambda_j^{-b} h_b((y_iy - x^j_2)/lambda_j).
// k_recon_tables builds X and Y (one thread per (j, grid line), the Hermite
// recurrence along a), k_recon_grid forms the product on the matrix cores in
// 32 x 64 tiles and writes omega once: with few vortices the kernel is bound
// by those writes.  Vortices are taken in chunks whose tables fit the workspace;
// later chunks add to omega.
//
// Non-axisymmetric enstrophy about a centre c (eq:nonaxi_enstrophy): omega at
// polar nodes (r_i, theta_l), theta_l = 2 pi l / ntheta (trapezoidal rule,
// exact for the angular modes of a vortex at c), r_i^2 = s_i the Gauss-Legendre
// nodes on [0, s_max] (int r dr = int ds / 2); per ring the azimuthal mean and
// the sum of squared deviations, then the rings summed in order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/mmvm.h"
#include "api_internal.hpp"
#include "util.hpp"

namespace mmvm {
namespace {

constexpr double kInvPi = 0.318309886183790671537767526745;
constexpr int kRecRows = 32, kRecCols = 64;  // output tile of one wavefront of the grid product
constexpr int kRecWaves = 4;                 // wavefronts per workgroup
constexpr int kRecDepth = 4;                 // k-steps per operand group in flight
constexpr int kRingThreads = 256;
constexpr size_t kTableBytes = (size_t)64 << 20;  // X and Y tables of one chunk of vortices

// Workspace of the diagnostics, per (device, stream), grown on demand.
struct ReconWS {
    char* base = nullptr;
    size_t bytes = 0;
};
std::mutex g_rmu;
std::map<std::pair<int, hipStream_t>, ReconWS> g_rws;
std::map<std::pair<int, int>, std::vector<double>> g_gl;  // Gauss-Legendre (nodes, weights) on [0, 1] per n

mmvm_status recon_ws(hipStream_t st, size_t need, char** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MMVM_EDEVICE;
    std::lock_guard<std::mutex> lk(g_rmu);
    ReconWS& w = g_rws[std::make_pair(dev, st)];
    if (need > w.bytes) {
        if (w.base) {
            if (hipStreamSynchronize(st) != hipSuccess) return MMVM_EDEVICE;  // queued work may use it
            (void)hipFree(w.base);
        }
        w.base = nullptr;
        w.bytes = 0;
        if (hipMalloc((void**)&w.base, need) != hipSuccess) return MMVM_ENOMEM;
        w.bytes = need;
    }
    *out = w.base;
    return MMVM_OK;
}

// Gauss-Legendre rule of n points on [0, 1] (Newton iteration on P_n from the
// Chebyshev-like first guesses cos(pi (i + 3/4) / (n + 1/2))), cached for the
// process: the device copy of a call reads it after the call returns.
const std::vector<double>& gauss_legendre01(int n)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_rmu);
    std::vector<double>& v = g_gl[std::make_pair(dev, n)];
    if (!v.empty()) return v;
    v.assign(2 * (size_t)n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;  // P_0, P_1
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double pn = n == 1 ? z : p1, pm = n == 1 ? 1.0 : p0;
            dp = n * (z * pn - pm) / (z * z - 1.0);
            const double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        v[i] = 0.5 * (1.0 - z);                       // node on [0, 1]
        v[n + i] = 1.0 / ((1.0 - z * z) * dp * dp);   // weight on [0, 1] (half of [-1, 1]'s)
    }
    return v;
}

// X[j][a][ix] (thread per (j, ix)) and Y[j][a][iy] (thread per (j, iy, group of
// kYGroup values of a: the moment sums are the bulk of the work) of vortices
// j0 .. j0 + nj - 1
constexpr int kYGroup = 8;

__global__ __launch_bounds__(256) void k_recon_tables(int M, int K, int j0, int nj, int nx, int ny, double gx0,
                                                      double gy0, double h, const double* __restrict__ x,
                                                      const double* __restrict__ mom,
                                                      const double* __restrict__ lam2, double* __restrict__ X,
                                                      double* __restrict__ Y)
{
    const int M1 = M + 1, ng = (M1 + kYGroup - 1) / kYGroup;
    const long tx = (long)nj * nx, total = tx + (long)nj * ny * ng;
    for (long id = blockIdx.x * (long)blockDim.x + threadIdx.x; id < total; id += (long)gridDim.x * blockDim.x) {
        const bool isx = id < tx;
        const long e = isx ? id : (id - tx) / ng;
        const int grp = isx ? 0 : (int)((id - tx) - e * ng);
        const int n = isx ? nx : ny;
        const int jj = (int)(e / n), i = (int)(e - (long)jj * n), j = j0 + jj;
        const double l2 = lam2[j], il = 1.0 / sqrt(l2);
        const double u = ((isx ? gx0 : gy0) + h * i - x[2 * j + (isx ? 0 : 1)]) * il;
        // h_a(u) lambda^{-a}, a = 0..M, by h_{a+1} = -2u h_a - 2a h_{a-1}
        double hv[MMVM_MAX_ORDER + 1];
        double hm = 0.0, hc = exp(-u * u), p = 1.0;
        for (int a = 0; a <= M; ++a) {
            hv[a] = hc * p;
            const double hn = -2.0 * u * hc - 2.0 * (double)a * hm;
            hm = hc;
            hc = hn;
            p *= il;
        }
        if (isx) {
            const double c = kInvPi / l2;
            double* o = X + (long)jj * M1 * nx + i;
            for (int a = 0; a <= M; ++a) o[(long)a * nx] = c * hv[a];
        } else {
            const double* mj = mom + (long)j * K;
            double* o = Y + (long)jj * M1 * ny + i;
            const int a1 = min(M1, (grp + 1) * kYGroup);
            for (int a = grp * kYGroup; a < a1; ++a) {
                double s = 0.0;
                for (int b = 0; a + b <= M; ++b) s = fma(mj[ctri(a, b)], hv[b], s);
                o[(long)a * ny] = s;
            }
        }
    }
}

// omega[iy][ix] (+)= sum_l Y[l][iy] X[l][ix], l over the chunk's nl = nj (M + 1)
// rows, on the FP64 matrix cores (v_mfma_f64_16x16x4f64: lane l supplies
// A[r0 + l%16][4s + l/16] = Y[4s + l/16][iy], B[4s + l/16][c0 + l%16] = X[..][ix]
// and receives D[r0 + l/16 + 4q][c0 + l%16] in component q).  One wavefront
// per 32 x 64 tile (2 x 4 blocks of 16 x 16); the operands come straight from
// the L2-resident tables as runs of 16 consecutive grid points (128-byte
// loads), and each store writes four whole 128-byte rows of omega, once
// (non-temporal: the grid is not read back).
typedef double dbl4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(64 * kRecWaves) void k_recon_grid(int nl, int nx, int ny, const double* __restrict__ X,
                                                              const double* __restrict__ Y, double* __restrict__ om,
                                                              int accumulate)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles_x = (nx + kRecCols - 1) / kRecCols;
    const int tile = blockIdx.x * kRecWaves + wave;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    if (ty * kRecRows >= ny) return;  // uniform per wavefront; no barrier in this kernel
    const int iy0 = ty * kRecRows, ix0 = tx * kRecCols;
    const int li = lane & 15, lk = lane >> 4;
    int iyA[2], ixB[4];
    bool okA[2], okB[4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        iyA[rb] = iy0 + 16 * rb + li;
        okA[rb] = iyA[rb] < ny;
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        ixB[cb] = ix0 + 16 * cb + li;
        okB[cb] = ixB[cb] < nx;
    }
    dbl4 acc[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = dbl4{0.0, 0.0, 0.0, 0.0};
    // operands of kRecDepth k-steps in flight: the next group is loaded while
    // the current one multiplies (one L2 round trip per group, not per k-step)
    const int ks = (nl + 3) >> 2;
    double a[kRecDepth][2], b[kRecDepth][4];
    auto load_group = [&](int s0, double (&ga)[kRecDepth][2], double (&gb)[kRecDepth][4]) {
#pragma unroll
        for (int d = 0; d < kRecDepth; ++d) {
            const int l = 4 * (s0 + d) + lk;
            const bool okl = l < nl;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) ga[d][rb] = (okl && okA[rb]) ? Y[(long)l * ny + iyA[rb]] : 0.0;
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) gb[d][cb] = (okl && okB[cb]) ? X[(long)l * nx + ixB[cb]] : 0.0;
        }
    };
    load_group(0, a, b);
    for (int s0 = 0; s0 < ks; s0 += kRecDepth) {
        double an[kRecDepth][2], bn[kRecDepth][4];
        if (s0 + kRecDepth < ks) load_group(s0 + kRecDepth, an, bn);
#pragma unroll
        for (int d = 0; d < kRecDepth; ++d)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[d][rb], b[d][cb], acc[rb][cb], 0, 0, 0);
        if (s0 + kRecDepth < ks) {
#pragma unroll
            for (int d = 0; d < kRecDepth; ++d) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) a[d][rb] = an[d][rb];
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) b[d][cb] = bn[d][cb];
            }
        }
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int iy = iy0 + 16 * rb + lk + 4 * q;
            if (iy >= ny) continue;
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                if (!okB[cb]) continue;
                double* o = om + (long)iy * nx + ixB[cb];
                const double v = acc[rb][cb][q];
                if (accumulate) *o += v;
                else __builtin_nontemporal_store(v, o);
            }
        }
}

// lambda_j(t)^2 = lambda_{j,0}^2 + 4 nu t (eq:phi00) of vortices j0 .. j0 + cnt - 1; the
// core scales travel as kernel arguments, so nothing waits for a host copy
constexpr int kParamChunk = 128;
struct ParamChunk {
    double lam0[kParamChunk];
};
__global__ __launch_bounds__(kParamChunk) void k_recon_lam2(int j0, int cnt, double nu, double t, ParamChunk c,
                                                            double* __restrict__ lam2)
{
    const int i = threadIdx.x;
    if (i < cnt) lam2[j0 + i] = c.lam0[i] * c.lam0[i] + 4.0 * nu * t;
}

void launch_lam2(const mmvm_problem* prob, double t, double* lam2, hipStream_t st)
{
    for (int j0 = 0; j0 < prob->n; j0 += kParamChunk) {
        ParamChunk c;
        std::memset(&c, 0, sizeof(c));
        const int cnt = prob->n - j0 < kParamChunk ? prob->n - j0 : kParamChunk;
        for (int i = 0; i < cnt; ++i) c.lam0[i] = prob->lambda0[j0 + i];
        hipLaunchKernelGGL(k_recon_lam2, dim3(1), dim3(kParamChunk), 0, st, j0, cnt, prob->nu, t, c, lam2);
    }
}

// omega at one point from every vortex (direct sum)
__device__ double omega_point(int N, int M, int K, const double* __restrict__ x, const double* __restrict__ mom,
                              const double* __restrict__ lam2, double p1, double p2)
{
    double om = 0.0;
    for (int j = 0; j < N; ++j) {
        const double l2 = lam2[j], il = 1.0 / sqrt(l2);
        const double u1 = (p1 - x[2 * j]) * il, u2 = (p2 - x[2 * j + 1]) * il;
        double h1[MMVM_MAX_ORDER + 1], h2[MMVM_MAX_ORDER + 1];
        double a1 = 0.0, c1 = exp(-u1 * u1), a2 = 0.0, c2 = exp(-u2 * u2), p = 1.0;
        for (int a = 0; a <= M; ++a) {
            h1[a] = c1 * p;
            h2[a] = c2 * p;
            const double n1 = -2.0 * u1 * c1 - 2.0 * (double)a * a1;
            const double n2 = -2.0 * u2 * c2 - 2.0 * (double)a * a2;
            a1 = c1;
            c1 = n1;
            a2 = c2;
            c2 = n2;
            p *= il;
        }
        const double* mj = mom + (long)j * K;
        double s = 0.0;
        for (int a = 0; a <= M; ++a) {
            double ya = 0.0;
            for (int b = 0; a + b <= M; ++b) ya = fma(mj[ctri(a, b)], h2[b], ya);
            s = fma(h1[a], ya, s);
        }
        om = fma(kInvPi / l2, s, om);
    }
    return om;
}

// ring i: r^2 = s_i; writes w_i/2 * (2 pi / ntheta) sum_l (omega_il - mean_i)^2
__global__ __launch_bounds__(kRingThreads) void k_enstrophy_rings(int N, int M, int K, int ntheta, double cx,
                                                                 double cy, double smax,
                                                                 const double* __restrict__ gl, int nr,
                                                                 const double* __restrict__ x,
                                                                 const double* __restrict__ mom,
                                                                 const double* __restrict__ lam2,
                                                                 double* __restrict__ ring)
{
    extern __shared__ double sw[];  // [ntheta] omega on the ring, then [waves] partial sums
    __shared__ double red[kRingThreads / 64];
    const int i = blockIdx.x, tid = threadIdx.x;
    const double s = smax * gl[i], wgt = smax * gl[nr + i];
    const double r = sqrt(s);
    double sum = 0.0;
    for (int l = tid; l < ntheta; l += blockDim.x) {
        const double th = 2.0 * M_PI * (double)l / (double)ntheta;
        const double v = omega_point(N, M, K, x, mom, lam2, cx + r * cos(th), cy + r * sin(th));
        sw[l] = v;
        sum += v;
    }
    // block sums in a fixed order: wavefront shuffle, then the wavefronts in order
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = sum;
    __syncthreads();
    double mean = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) mean += red[q];
    mean /= (double)ntheta;
    __syncthreads();
    double sq = 0.0;
    for (int l = tid; l < ntheta; l += blockDim.x) {
        const double d = sw[l] - mean;
        sq = fma(d, d, sq);
    }
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = sq;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
        ring[i] = 0.5 * wgt * (2.0 * M_PI / (double)ntheta) * t;
    }
}

// E = the sum of the ring values: lane l adds rings l, l + 64, ... in order,
// then a fixed shuffle tree (the same bits on every run)
__global__ __launch_bounds__(64) void k_enstrophy_sum(int nr, const double* __restrict__ ring, double* __restrict__ E)
{
    const int lane = threadIdx.x;
    double e = 0.0;
    for (int i = lane; i < nr; i += 64) e += ring[i];
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if (lane == 0) *E = e;
}

size_t up256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace
}  // namespace mmvm

using namespace mmvm;

extern "C" {

mmvm_status mmvm_vorticity_grid(const mmvm_problem* prob, double t, const double* x, const double* mom, double x0,
                                double y0, double h, int32_t nx, int32_t ny, double* omega, void* stream)
{
    if (!prob) return MMVM_EINVAL;
    if (prob->n < 1 || prob->order < 0 || prob->order > MMVM_MAX_ORDER) return MMVM_EORDER;
    if (!prob->lambda0 || !(prob->nu >= 0.0) || !std::isfinite(prob->nu)) return MMVM_EINVAL;
    for (int j = 0; j < prob->n; ++j)
        if (!(prob->lambda0[j] > 0.0) || !std::isfinite(prob->lambda0[j])) return MMVM_EINVAL;
    if (!x || !mom || !omega || nx < 1 || ny < 1 || !(h > 0.0) || !std::isfinite(x0) || !std::isfinite(y0) ||
        !std::isfinite(t))
        return MMVM_EINVAL;
    const int N = prob->n, M = prob->order, M1 = M + 1, K = (M + 1) * (M + 2) / 2;
    hipStream_t st = (hipStream_t)stream;
    // vortices per chunk: the X and Y tables of a chunk fit kTableBytes
    const size_t per = sizeof(double) * (size_t)M1 * ((size_t)nx + ny);
    if (per > kTableBytes) return MMVM_EINVAL;  // grid too large for one vortex's tables
    const int chunk = (int)std::min<size_t>((size_t)N, kTableBytes / per);
    const size_t off_lam = 0, off_x = up256(sizeof(double) * N);
    const size_t off_y = off_x + up256(sizeof(double) * (size_t)chunk * M1 * nx);
    const size_t need = off_y + up256(sizeof(double) * (size_t)chunk * M1 * ny);
    char* base = nullptr;
    mmvm_status s = recon_ws(st, need, &base);
    if (s != MMVM_OK) return s;
    double* lam2 = (double*)(base + off_lam);
    double* X = (double*)(base + off_x);
    double* Y = (double*)(base + off_y);
    launch_lam2(prob, t, lam2, st);
    for (int j0 = 0; j0 < N; j0 += chunk) {
        const int nj = std::min(chunk, N - j0);
        const long tot = (long)nj * (nx + (long)ny * ((M1 + kYGroup - 1) / kYGroup));
        const int tb = (int)std::min<long>((tot + 255) / 256, 8192);
        hipLaunchKernelGGL(k_recon_tables, dim3(tb), dim3(256), 0, st, M, K, j0, nj, (int)nx, (int)ny, x0, y0, h, x,
                           mom, (const double*)lam2, X, Y);
        const long tiles = (long)((nx + kRecCols - 1) / kRecCols) * ((ny + kRecRows - 1) / kRecRows);
        void* tk = timing_begin(st);
        launch_kernel(k_recon_grid, dim3((unsigned)((tiles + kRecWaves - 1) / kRecWaves)), dim3(64 * kRecWaves), 0, st,
                      nj * M1, (int)nx, (int)ny, (const double*)X, (const double*)Y, omega, j0 > 0 ? 1 : 0);
        timing_end(tk, "recon", st);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        report_hip_error(e, "mmvm_vorticity_grid launch");
        return MMVM_EDEVICE;
    }
    return MMVM_OK;
}

mmvm_status mmvm_enstrophy_nonaxi(const mmvm_problem* prob, double t, const double* x, const double* mom, double cx,
                                  double cy, double rmax, int32_t nr, int32_t ntheta, double* E, void* stream)
{
    if (!prob) return MMVM_EINVAL;
    if (prob->n < 1 || prob->order < 0 || prob->order > MMVM_MAX_ORDER) return MMVM_EORDER;
    if (!prob->lambda0 || !(prob->nu >= 0.0) || !std::isfinite(prob->nu)) return MMVM_EINVAL;
    for (int j = 0; j < prob->n; ++j)
        if (!(prob->lambda0[j] > 0.0) || !std::isfinite(prob->lambda0[j])) return MMVM_EINVAL;
    if (!x || !mom || !E || nr < 1 || nr > 4096 || ntheta < 1 || ntheta > 8192 || !(rmax > 0.0) ||
        !std::isfinite(cx) || !std::isfinite(cy) || !std::isfinite(t))
        return MMVM_EINVAL;
    const int N = prob->n, M = prob->order, K = (M + 1) * (M + 2) / 2;
    hipStream_t st = (hipStream_t)stream;
    const size_t off_gl = up256(sizeof(double) * N);
    const size_t off_ring = off_gl + up256(sizeof(double) * 2 * nr);
    const size_t need = off_ring + up256(sizeof(double) * nr);
    char* base = nullptr;
    mmvm_status s = recon_ws(st, need, &base);
    if (s != MMVM_OK) return s;
    double* lam2 = (double*)base;
    double* gl = (double*)(base + off_gl);
    double* ring = (double*)(base + off_ring);
    // the rule is cached for the process, so the copy's source outlives the call
    const std::vector<double>& g = gauss_legendre01(nr);
    if (hipMemcpyAsync(gl, g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        return MMVM_EDEVICE;
    launch_lam2(prob, t, lam2, st);
    const size_t shmem = sizeof(double) * (size_t)ntheta;
    if (shmem > 64 * 1024) return MMVM_EINVAL;
    void* tk = timing_begin(st);
    launch_kernel(k_enstrophy_rings, dim3(nr), dim3(kRingThreads), (std::uint32_t)shmem, st, N, M, K, (int)ntheta,
                  cx, cy, rmax * rmax, (const double*)gl, (int)nr, x, mom, (const double*)lam2, ring);
    timing_end(tk, "enstrophy", st);
    hipLaunchKernelGGL(k_enstrophy_sum, dim3(1), dim3(64), 0, st, (int)nr, (const double*)ring, E);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        report_hip_error(e, "mmvm_enstrophy_nonaxi launch");
        return MMVM_EDEVICE;
    }
    return MMVM_OK;
}

}  // extern "C"
