// Pair-interaction kernel for any order (the order is a runtime argument): the
// path of multi-vortex problems above the orders of the unrolled kernel
// (pair.hpp).  Same quantity as k_pair:
//   S_pair[j][g] = sum_{j' != j} sum_{|m| <= M} alpha'_m Psi'(m + g; s_jj'),
// the derivatives of the source's velocity smoothed by the target Gaussian
// (eq:FinalCrossI/II, H^B = D^a V00 through the stream function), in the
// target's lambda units.  FP64 throughout, in both precisions.
//
// One workgroup per target; the sources are visited in order.  Per source the
// stream-function derivatives Psi(a), |a| <= P = 3M, are generated into LDS:
//   * seeds on four lanes: the incomplete-gamma sequence, the complex powers,
//     and the 1-D Gaussian derivatives h_c(s1), h_c(s2);
//   * one lane per shell n: the edges a = (0, n), (1, n - 1) from the complex
//     derivative plus the kappa-weighted Gaussian products, then the rest of
//     the shell by the Laplacian relation Psi(a1 + 2, a2) = h_a1 h_a2 / pi -
//     Psi(a1, a2 + 2);
// then every lane accumulates its entries g of the contraction from LDS.
//
// The complex derivative of the shell is (-1)^{n-1} (n-1)! P(n, w) / (4 pi z^n)
// (P the regularised lower incomplete gamma function, w = |s|^2), evaluated in
// two forms that keep every intermediate in range up to shell 120:
//   w <= 1:  q_n = (n-1)! P(n, w) / w^n  times  zbar^n   (q_n <= 1/n, |zbar^n| <= 1),
//   w >  1:  q_n = (n-1)! P(n, w)        times  z^{-n}   (q_n <= (n-1)!, |z^{-n}| <= 1),
// both by the stable downward recurrences q_n = (w q_{n+1} + e^{-w}) / n and
// q_n = (q_{n+1} + e^{-w} w^n) / n from a seed at n = P (a series for w <= P,
// the complement of the upper incomplete gamma function above).
#include <hip/hip_runtime.h>

#include "../../include/mmvm.h"
#include "kernels.hpp"
#include "util.hpp"

namespace mmvm {
namespace {

constexpr int kGenThreads = 256;
constexpr int kGenSlots = ((2 * MMVM_MAX_ORDER + 1) * (2 * MMVM_MAX_ORDER + 2) / 2 + kGenThreads - 1) / kGenThreads;
static_assert(3 * MMVM_MAX_ORDER <= kGenThreads, "one lane per shell");

// LDS regions (doubles)
struct GenShape {
    int P, K, KG, psi, am, q, zr, zi, h1, h2, total;
    __host__ __device__ explicit GenShape(int M)
    {
        const int GM = M == 0 ? 1 : 2 * M;
        P = M == 0 ? 1 : 3 * M;
        K = (M + 1) * (M + 2) / 2;
        KG = (GM + 1) * (GM + 2) / 2;
        psi = 0;                            // Psi'(a), shell-major [tri(P)]
        am = psi + (P + 1) * (P + 2) / 2;   // source moments in the target's units [K]
        q = am + K;                         // q_n [P + 1]
        zr = q + P + 1;                     // the complex powers [P + 1] x 2
        zi = zr + P + 1;
        h1 = zi + P + 1;                    // h_c(s1), h_c(s2) [P]
        h2 = h1 + P;
        total = h2 + P;
    }
};

__global__ __launch_bounds__(kGenThreads) void k_pair_gen(int M, int N, const double* __restrict__ xs,
                                                         const double* __restrict__ lam2,
                                                         const double* __restrict__ alpha,
                                                         const double* __restrict__ kap0,
                                                         const double* __restrict__ kap1,
                                                         double* __restrict__ spair)
{
    constexpr double kInvPi = 0.318309886183790671537767526745;
    constexpr double kInv4Pi = 0.0795774715459476678844418816863;
    const GenShape L(M);
    const int P = L.P, K = L.K, KG = L.KG;
    extern __shared__ double sm_gen[];
    double* sPsi = sm_gen + L.psi;
    double* sAm = sm_gen + L.am;
    double* sQ = sm_gen + L.q;
    double* sZr = sm_gen + L.zr;
    double* sZi = sm_gen + L.zi;
    double* sH1 = sm_gen + L.h1;
    double* sH2 = sm_gen + L.h2;
    const int j = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;

    const double xj1 = xs[2 * j], xj2 = xs[2 * j + 1], lj2 = lam2[j];
    const double ilj = 1.0 / sqrt(lj2);
    const double lj = lj2 * ilj;

    // this lane's entries g = tid + u nt of the table
    double acc[kGenSlots];
    int gsh[kGenSlots], gcol[kGenSlots];
#pragma unroll
    for (int u = 0; u < kGenSlots; ++u) {
        acc[u] = 0.0;
        const int g = tid + u * nt;
        const int s = g < KG ? shell_of(g) : 0;
        gsh[u] = s;
        gcol[u] = g - s * (s + 1) / 2;  // g2
    }

    for (int jp = 0; jp < N; ++jp) {
        if (jp == j) continue;
        const double lp2 = lam2[jp];
        const double c = lj2 + lp2;
        const double isc = 1.0 / sqrt(c);
        const double s1 = (xj1 - xs[2 * jp]) * isc, s2 = (xj2 - xs[2 * jp + 1]) * isc;
        const double w = s1 * s1 + s2 * s2;
        const bool far = w > 1.0;
        const double tau = lj * isc;

        if (tid == 0) {
            // q_P: the series sum_k prod_{i <= k} w / (P + i) (terms decrease for w <= P)
            double q;
            if (w <= (double)P) {
                double term = 1.0, sum = 0.0;
                for (int k = 1; k < 4096 && term > 1e-18 * sum; ++k) {
                    sum += term;
                    term *= w / (double)(P + k);
                }
                // q_P = e^{-w} (w^P if far) sum / P
                q = (far ? exp((double)P * log(w) - w) : exp(-w)) * sum / (double)P;
            } else {
                // (P - 1)! (1 - Q(P, w)) / w^P (w^P dropped when far; always far here)
                double t = exp(-w), Q = 0.0, f = 1.0;
                for (int k = 0; k < P; ++k) {
                    Q += t;
                    t *= w / (double)(k + 1);
                }
                for (int k = 1; k < P; ++k) f *= (double)k;  // (P - 1)!
                q = f * (1.0 - Q);
            }
            sQ[P] = q;
            // downward: near q_n = (w q_{n+1} + e^{-w}) / n; far q_n = (q_{n+1} + e^{-w} w^n) / n
            const double E = exp(-w);
            double d = far ? exp((double)(P - 1) * log(w) - w) : 0.0;  // e^{-w} w^n at n = P - 1
            for (int n = P - 1; n >= 1; --n) {
                q = far ? (q + d) / (double)n : fma(w, q, E) / (double)n;
                sQ[n] = q;
                if (far) d /= w;
            }
        } else if (tid == 1) {
            // zbar^n (near) or z^{-n} = (zbar / w)^n (far)
            const double br = far ? s1 / w : s1, bi = far ? -s2 / w : -s2;
            double zr = 1.0, zi = 0.0;
            sZr[0] = 1.0;
            sZi[0] = 0.0;
            for (int n = 1; n <= P; ++n) {
                const double nr = zr * br - zi * bi, ni = zr * bi + zi * br;
                zr = nr;
                zi = ni;
                sZr[n] = zr;
                sZi[n] = zi;
            }
        } else if (tid == 2 || tid == 3) {
            // h_c(x) = d^c/dx^c exp(-x^2), c = 0 .. P - 2
            const double x = tid == 2 ? s1 : s2;
            double* h = tid == 2 ? sH1 : sH2;
            double hm = 0.0, hc = exp(-x * x);
            h[0] = hc;
            for (int a = 0; a + 1 <= P - 2; ++a) {
                const double hn = -2.0 * x * hc - 2.0 * (double)a * hm;
                hm = hc;
                hc = hn;
                h[a + 1] = hc;
            }
        }
        // the source's moments in the target's lambda units: alpha_m (lambda_j' / lambda_j)^{|m|}
        {
            const double ratio = sqrt(lp2) * ilj;
            const double* al = alpha + (long)jp * K;
            for (int m = tid; m < K; m += nt) {
                const int s = shell_of(m);
                double r = 1.0;
                for (int i = 0; i < s; ++i) r *= ratio;
                sAm[m] = al[m] * r;
            }
        }
        __syncthreads();
        // shell n = tid + 1: Psi'(a, n - a) at tri index n(n+1)/2 + n - a
        for (int n = tid + 1; n <= P; n += nt) {
            // h = (-1)^{n-1} q_n {zbar^n or z^{-n}} / (4 pi): the holomorphic edge part
            const double sg = (n & 1) ? kInv4Pi : -kInv4Pi;
            const double hr = sg * sQ[n] * sZr[n], hi = sg * sQ[n] * sZi[n];
            double e0, e1;  // 2 Re(i^n h), 2 Re(i^{n-1} h)
            switch (n & 3) {
            case 0: e0 = hr; e1 = hi; break;
            case 1: e0 = -hi; e1 = hr; break;
            case 2: e0 = -hr; e1 = -hi; break;
            default: e0 = hi; e1 = -hr; break;
            }
            double p0 = 2.0 * e0, p1 = 2.0 * e1;
            const double* k0 = kap0 + (long)n * (P + 1);
            const double* k1 = kap1 + (long)n * (P + 1);
            for (int cc = 0; cc <= n - 2; ++cc) {
                const double pr = sH1[cc] * sH2[n - 2 - cc];
                p0 = fma(k0[cc], pr, p0);
                p1 = fma(k1[cc], pr, p1);
            }
            double tn = 1.0;
            for (int i = 0; i < n; ++i) tn *= tau;
            double* row = sPsi + n * (n + 1) / 2 + n;  // row[-a] = Psi'(a, n - a)
            row[0] = p0 * tn;
            if (n >= 1) row[-1] = p1 * tn;
            double pa = p0, pb = p1;  // Psi(a, n - a) for the even and odd chains
            for (int a = 0; a + 2 <= n; ++a) {
                const double prev = (a & 1) ? pb : pa;
                const double v = sH1[a] * sH2[n - 2 - a] * kInvPi - prev;
                row[-(a + 2)] = v * tn;
                if (a & 1) pb = v;
                else pa = v;
            }
        }
        __syncthreads();
        // contraction: S[g] += sum_m alpha'_m Psi'(m + g), m by shells (contiguous in m2)
#pragma unroll
        for (int u = 0; u < kGenSlots; ++u) {
            const int g = tid + u * nt;
            if (g > 0 && g < KG) {
                double a = acc[u];
                for (int s = 0; s <= M; ++s) {
                    const int n = s + gsh[u];
                    const double* pr = sPsi + n * (n + 1) / 2 + gcol[u];
                    const double* ar = sAm + s * (s + 1) / 2;
                    for (int m2 = 0; m2 <= s; ++m2) a = fma(ar[m2], pr[m2], a);
                }
                acc[u] = a;
            }
        }
        __syncthreads();  // the next source overwrites LDS
    }
#pragma unroll
    for (int u = 0; u < kGenSlots; ++u) {
        const int g = tid + u * nt;
        if (g < KG) spair[(long)j * KG + g] = g == 0 ? 0.0 : acc[u];
    }
}

}  // namespace

size_t pair_gen_lds_bytes(int M) { return sizeof(double) * (size_t)GenShape(M).total; }

hipError_t launch_pair_gen(const DevTables& T, const StageBufs& B, int cur, hipStream_t st)
{
    if (T.M < 0 || T.M > MMVM_MAX_ORDER) return hipErrorInvalidValue;
    const size_t shmem = pair_gen_lds_bytes(T.M);
    const hipError_t ea = lds_limit_once((const void*)k_pair_gen, pair_gen_lds_bytes(MMVM_MAX_ORDER),
                                         "hipFuncSetAttribute(k_pair_gen dynamic LDS)");
    if (ea != hipSuccess) return ea;
    launch_kernel(k_pair_gen, dim3(B.N), dim3(kGenThreads), (std::uint32_t)shmem, st, T.M, B.N, B.xs, B.lam2[cur],
                  B.alpha[cur], T.kap0, T.kap1, B.s_pair);
    return hipGetLastError();
}

}  // namespace mmvm
