// Pair-interaction kernel for few vortices: one pair per slot of 16 lanes.
//
// With few vortices there are too few pairs to occupy the chip one pair per
// lane (64 vortices: 4032 pairs, 63 wavefronts), and a lane that carries a
// whole pair runs thousands of dependent instructions.  Here a workgroup of
// 256 lanes holds 16 pairs of one target at a time and splits each pair's work
// across lanes:
//   1. the per-pair sequences, each on its own wavefront (no divergence inside
//      a wavefront): the incomplete-gamma sequence g_n (wave 0), the complex
//      powers zbar^n (wave 1), the 1-D Gaussian derivatives h_c(s1), h_c(s2)
//      (wave 2), the source moments in the target's units (wave 3);
//   2. the shells n = 1..P of Psi' (two per lane, n and P + 1 - n, so every
//      lane does about the same work): edges from the complex derivative and
//      the kappa-weighted Gaussian products, the rest by the Laplacian relation;
//   3. the contraction S[g] += sum_m alpha'_m Psi'(m + g), sixteen lanes per
//      pair, each owning every sixteenth entry g.
// Then the 16 pair slots are summed in slot order (deterministic).  The same
// formulas as the unrolled kernel (pair.hpp), in FP64 for both precisions.
// A target's sources can be split over G workgroups (grid N x G); their partial
// tables are added in group order by the stage-2 kernel that reads them.
#pragma once
#include "kernels.hpp"
#include "util.hpp"

namespace mmvm {

constexpr int kSplitSlots = 16;  // pairs per workgroup
constexpr int kSplitLanes = 16;  // lanes per pair
constexpr int kSplitThreads = kSplitSlots * kSplitLanes;
static_assert(kSplitThreads == 256, "four wavefronts");

template <int M>
struct SplitShape {
    static constexpr int K = (M + 1) * (M + 2) / 2;
    static constexpr int P = M == 0 ? 1 : 3 * M;
    static constexpr int GM = M == 0 ? 1 : 2 * M;
    static constexpr int KG = (GM + 1) * (GM + 2) / 2;
    static constexpr int HN = P >= 2 ? P - 1 : 1;
    static constexpr int NPSI = (P + 1) * (P + 2) / 2;
    static constexpr int NG = (KG + kSplitLanes - 1) / kSplitLanes;  // entries g per lane
    static constexpr int NSH = (P + 1) / 2;                          // shell tasks per pair
    static_assert(NSH <= kSplitLanes, "two shells per lane");
    static_assert(kSplitSlots * KG <= kSplitSlots * NPSI, "the reduction reuses the Psi region");
};

template <int M>
__global__ __launch_bounds__(kSplitThreads) void k_pair_split(int N, int G, const double* __restrict__ xs,
                                                              const double* __restrict__ lam2,
                                                              const double* __restrict__ alpha,
                                                              const double* __restrict__ kap0,
                                                              const double* __restrict__ kap1,
                                                              const double* __restrict__ hol,
                                                              double* __restrict__ out)
{
    typedef SplitShape<M> Sh;
    constexpr int K = Sh::K, P = Sh::P, KG = Sh::KG, HN = Sh::HN, NPSI = Sh::NPSI, NG = Sh::NG;
    constexpr double kInvPi = 0.318309886183790671537767526745;
    __shared__ double sPsi[kSplitSlots][NPSI];
    __shared__ double sAm[kSplitSlots][K];
    __shared__ double sG[kSplitSlots][P + 1];
    __shared__ double sZr[kSplitSlots][P + 1], sZi[kSplitSlots][P + 1];
    __shared__ double sH[2][kSplitSlots][HN];
    __shared__ double sKap[2][P + 1][P + 1];  // the edge coefficients of every shell

    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
    for (int e = tid; e < (P + 1) * (P + 1); e += kSplitThreads) {
        sKap[0][e / (P + 1)][e % (P + 1)] = kap0[e];
        sKap[1][e / (P + 1)][e % (P + 1)] = kap1[e];
    }
    const int j = blockIdx.x / G, grp = blockIdx.x - (blockIdx.x / G) * G;
    const double xj1 = xs[2 * j], xj2 = xs[2 * j + 1], lj2 = lam2[j];
    const double ilj = 1.0 / sqrt(lj2);
    const double lj = lj2 * ilj;
    // phase 3 role: pair slot tid % 16, entries g = q + 16 u
    const int cslot = tid & (kSplitSlots - 1), q = tid >> 4;
    double acc[NG];
#pragma unroll
    for (int u = 0; u < NG; ++u) acc[u] = 0.0;

    // sources grp, grp + G, ... (skipping the target), 16 per round
    const int nsrc = (N - grp + G - 1) / G;
    for (int r0 = 0; r0 < nsrc; r0 += kSplitSlots) {
        // ---- 1. per-pair sequences
        if (wave == 0 && l < kSplitSlots) {
            const int jp = grp + G * (r0 + l);
            if (jp < N && jp != j) {
                const double c = lj2 + lam2[jp];
                const double isc = 1.0 / sqrt(c);
                const double s1 = (xj1 - xs[2 * jp]) * isc, s2 = (xj2 - xs[2 * jp + 1]) * isc;
                const double w = s1 * s1 + s2 * s2;
                const double E = exp(-w);
                // g_P (series below P, complement above), then g_n = w g_{n+1} + e^{-w}/n!
                double ifP = 1.0;
                for (int f = 2; f <= P; ++f) ifP *= 1.0 / (double)f;
                double gP;
                if (w <= (double)P) {  // 56 terms reach double precision for P <= 18
                    double term = ifP, sum = 0.0;
#pragma unroll
                    for (int k = 0; k < kSeriesTerms; ++k) {
                        sum += term;
                        term *= w * (1.0 / (double)(P + k + 1));
                    }
                    gP = E * sum;
                } else {
                    double sm = 0.0, term = 1.0, wp = 1.0;
                    for (int k = 0; k < P; ++k) {
                        sm += term;
                        term *= w * (1.0 / (double)(k + 1));
                        wp *= w;
                    }
                    gP = (1.0 - E * sm) / wp;
                }
                sG[l][P] = gP;
                double g = gP, ifn = ifP;
                for (int n = P - 1; n >= 1; --n) {
                    ifn *= (double)(n + 1);  // 1/n!
                    g = fma(w, g, E * ifn);
                    sG[l][n] = g;
                }
            }
        } else if (wave == 1 && l < kSplitSlots) {
            const int jp = grp + G * (r0 + l);
            if (jp < N && jp != j) {
                const double isc = 1.0 / sqrt(lj2 + lam2[jp]);
                const double s1 = (xj1 - xs[2 * jp]) * isc, s2 = (xj2 - xs[2 * jp + 1]) * isc;
                double zr = 1.0, zi = 0.0;
                for (int n = 1; n <= P; ++n) {  // zbar^n
                    const double nr = zr * s1 + zi * s2, ni = zi * s1 - zr * s2;
                    zr = nr;
                    zi = ni;
                    sZr[l][n] = zr;
                    sZi[l][n] = zi;
                }
            }
        } else if (wave == 2 && l < 2 * kSplitSlots) {
            const int slot = l & (kSplitSlots - 1), axis = l >> 4;
            const int jp = grp + G * (r0 + slot);
            if (jp < N && jp != j) {
                const double isc = 1.0 / sqrt(lj2 + lam2[jp]);
                const double x = axis == 0 ? (xj1 - xs[2 * jp]) * isc : (xj2 - xs[2 * jp + 1]) * isc;
                double hm = 0.0, hc = exp(-x * x);
                sH[axis][slot][0] = hc;
                for (int a = 0; a + 1 < HN; ++a) {  // h_{a+1} = -2x h_a - 2a h_{a-1}
                    const double hn = -2.0 * x * hc - 2.0 * (double)a * hm;
                    hm = hc;
                    hc = hn;
                    sH[axis][slot][a + 1] = hc;
                }
            }
        } else if (wave == 3) {
            // source moments alpha_m (lambda_j' / lambda_j)^{|m|}, 16 rows of K
            for (int e = l; e < kSplitSlots * K; e += 64) {
                const int slot = e / K, m = e - slot * K;
                const int jp = grp + G * (r0 + slot);
                if (jp < N && jp != j) {
                    const double ratio = sqrt(lam2[jp]) * ilj;
                    const int s = shell_of(m);
                    double rp = 1.0;
                    for (int i = 0; i < s; ++i) rp *= ratio;
                    sAm[slot][m] = alpha[(long)jp * K + m] * rp;
                }
            }
        }
        __syncthreads();
        // ---- 2. shells: slot tid % 16, task tid / 16 -> shells task + 1 and P - task
        {
            const int slot = tid & (kSplitSlots - 1), task = tid >> 4;
            const int jp = grp + G * (r0 + slot);
            if (task < Sh::NSH && jp < N && jp != j) {
                const double tau = lj / sqrt(lj2 + lam2[jp]);
                for (int h2 = 0; h2 < 2; ++h2) {
                    const int n = h2 == 0 ? task + 1 : P - task;
                    if (h2 == 1 && n == task + 1) break;
                    const double hc = hol[n] * sG[slot][n];
                    const double hr = hc * sZr[slot][n], hi = hc * sZi[slot][n];
                    double e0, e1;  // 2 Re(i^n h), 2 Re(i^{n-1} h)
                    switch (n & 3) {
                    case 0: e0 = hr; e1 = hi; break;
                    case 1: e0 = -hi; e1 = hr; break;
                    case 2: e0 = -hr; e1 = -hi; break;
                    default: e0 = hi; e1 = -hr; break;
                    }
                    double p0 = 2.0 * e0, p1 = 2.0 * e1;
                    const double* k0 = sKap[0][n];
                    const double* k1 = sKap[1][n];
                    for (int cc = 0; cc <= n - 2; ++cc) {
                        const double pr = sH[0][slot][cc] * sH[1][slot][n - 2 - cc];
                        p0 = fma(k0[cc], pr, p0);
                        p1 = fma(k1[cc], pr, p1);
                    }
                    double tn = 1.0;
                    for (int i = 0; i < n; ++i) tn *= tau;
                    double* row = &sPsi[slot][n * (n + 1) / 2 + n];  // row[-a] = Psi'(a, n - a)
                    row[0] = p0 * tn;
                    row[-1] = p1 * tn;
                    double pa = p0, pb = p1;
                    for (int a = 0; a + 2 <= n; ++a) {
                        const double v = sH[0][slot][a] * sH[1][slot][n - 2 - a] * kInvPi - ((a & 1) ? pb : pa);
                        row[-(a + 2)] = v * tn;
                        if (a & 1) pb = v;
                        else pa = v;
                    }
                }
            }
        }
        __syncthreads();
        // ---- 3. contraction over this pair's moments
        {
            const int jp = grp + G * (r0 + cslot);
            if (jp < N && jp != j) {
                double am[K];
#pragma unroll
                for (int m = 0; m < K; ++m) am[m] = sAm[cslot][m];
                const double* ps = sPsi[cslot];
#pragma unroll
                for (int u = 0; u < NG; ++u) {
                    const int g = q + kSplitLanes * u;
                    if (g >= 1 && g < KG) {
                        const int gs = shell_of(g), g2 = g - gs * (gs + 1) / 2;
                        double a = acc[u];
#pragma unroll
                        for (int s = 0; s <= M; ++s) {
                            const double* pr = ps + (s + gs) * (s + gs + 1) / 2 + g2;  // Psi'(m + g), m2 = 0..s
#pragma unroll
                            for (int m2 = 0; m2 <= s; ++m2) a = fma(am[s * (s + 1) / 2 + m2], pr[m2], a);
                        }
                        acc[u] = a;
                    }
                }
            }
        }
        __syncthreads();
    }
    // ---- sum of the 16 slots, in slot order
    double* red = &sPsi[0][0];  // [slot][KG]
#pragma unroll
    for (int u = 0; u < NG; ++u) {
        const int g = q + kSplitLanes * u;
        if (g < KG) red[cslot * KG + g] = acc[u];
    }
    __syncthreads();
    for (int g = tid; g < KG; g += kSplitThreads) {
        double v = 0.0;
        if (g > 0)
            for (int sl = 0; sl < kSplitSlots; ++sl) v += red[sl * KG + g];
        out[((long)j * G + grp) * KG + g] = v;
    }
}


// the source groups are those of pair_split_groups(N) (the shape is tuned per N
// bucket; the group count follows the exact N)
template <int M>
hipError_t launch_pair_split_M(const DevTables& T, const StageBufs& B, int cur, hipStream_t st)
{
    typedef SplitShape<M> Sh;
    const int G = pair_split_groups(B.N);
    if (!T.kap0 || T.P != Sh::P) return hipErrorInvalidValue;
    double* dst = G == 1 ? B.s_pair : B.p_part;  // G > 1: partial tables [N][G][KG]
    if (!dst) return hipErrorInvalidValue;
    launch_kernel((k_pair_split<M>), dim3(B.N * G), dim3(kSplitThreads), 0, st, B.N, G, B.xs, B.lam2[cur],
                  B.alpha[cur], T.kap0, T.kap1, T.hol, dst);
    return hipGetLastError();
}

}  // namespace mmvm
