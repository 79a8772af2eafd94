// Pair-interaction kernel, templated on the order M (included by one
// translation unit per order, so that the fully unrolled variants compile in
// parallel).
#pragma once
#include <cstdlib>
#include <type_traits>
#include <utility>

#include "kernels.hpp"
#include "util.hpp"

namespace mmvm {

// terms of the series e^{-w} sum_k w^k/(P+k)! for w <= P: the tail ratio is at
// most w/(P+k+1) <= P/(P+k+1), so 56 terms reach double precision for P <= 18
constexpr int kSeriesTerms = 56;

// the edge coefficients kappa_e[n][c] and hol[n] of every shell n <= 18 as
// constants (written by gen_pair_consts.py; the same values as the host tables)
#include "pair_consts.inc"

}  // namespace mmvm

#include "pair_split.hpp"  // the few-vortex variant (uses kSeriesTerms)

namespace mmvm {

// 1/P! as the product 1/2 * 1/3 * ... * 1/P, each factor and product rounded
constexpr double pair_inv_factorial(int P)
{
    double r = 1.0;
    for (int f = 2; f <= P; ++f) r *= 1.0 / (double)f;
    return r;
}

// ---------------------------------------------------------------------------
// pair velocity-derivative table.
//
// For target j and source j' with c = lambda_j^2 + lambda_{j'}^2 and
// s = (x^j - x^{j'}) / sqrt(c), the derivatives D^a psi of the stream
// function psi(s) = (ln|s|^2 + E1(|s|^2)) / (4 pi) (velocity V00 = (-d2 psi, d1 psi)
// of a unit Gaussian) are generated shell by shell n = |a| = 1..P:
//   * the two edges a = (0, n), (1, n-1) from the complex derivative
//     psi_{n0} = (-1)^{n-1} (n-1)! P(n, w) / (4 pi z^n),   w = |s|^2,
//     written (-1)^{n-1}(n-1)!/(4pi) g_n zbar^n with g_n = P(n,w)/w^n obtained
//     by the stable downward recurrence g_n = w g_{n+1} + e^{-w}/n!, plus the
//     kappa-weighted products of 1-D Gaussian derivatives h_c(s1) h_d(s2);
//   * the rest of the shell by the Laplacian relation
//     Psi(a1+2, a2) = h_{a1}(s1) h_{a2}(s2) / pi - Psi(a1, a2+2).
// Each shell is consumed at once by the Hankel contraction
//   S[g] += sum_m alpha'_m Psi'(m + g),
// alpha'_m = alpha^{j'}_m (lambda_{j'}/lambda_j)^{|m|}, Psi' = (lambda_j/sqrt(c))^{|a|} Psi,
// which is D^g of the source's velocity smoothed by the target Gaussian, in
// the target's lambda units.
// ---------------------------------------------------------------------------
// Launch shape (PairShape): split wavefronts share the sources of one target
// (wave q of a target takes the sources q*64 + lane, stepping by 64 split);
// their wavefront sums meet in LDS and are added in wave order, so a shape
// always gives the same bits.  A workgroup holds tpb targets.
// Far-field threshold of shell count P: beyond w = |s|^2 = 50 + 2.5 P every
// Gaussian part of Psi (the deficit of the incomplete gamma factor and the 1-D
// Gaussian products) is below FP64 rounding of its shell (measured against the
// quad-precision H^B at P = 3..18), and Psi'(a) = 2 Re(i^{a2} H_{|a|}),
// H_n = hol[n] (tau / z)^n, the harmonic part alone.
constexpr double pair_far_w(int P) { return 50.0 + 2.5 * P; }
// relative margin of the record-based far test against rounding at the threshold
constexpr double kFarBoundMargin = 1.0 + 1e-9;

// FAR: a wavefront whose pairs of one 64-source chunk are all beyond the
// threshold skips them and marks the chunk in farmask[j][chunk] (0 otherwise);
// k_pair_far adds those pairs afterwards.
// Targets j come from (xt, lam2t) in the caller's order; sources from (xs,
// lam2, aT) in the sources' order, where target j is source rank[j] (rank null:
// the same order).
template <int M, typename R, bool FAR>
__global__ __launch_bounds__(kPairMaxThreads) void k_pair(int N, int split, const double* __restrict__ xt,
                                                          const double* __restrict__ lam2t,
                                                          const double* __restrict__ xs,
                                                          const double* __restrict__ lam2, const R* __restrict__ aT,
                                                          double* __restrict__ spair,
                                                          unsigned char* __restrict__ farmask,
                                                          const int* __restrict__ rank,
                                                          const double* __restrict__ crec)
{
    constexpr int K = (M + 1) * (M + 2) / 2;
    constexpr int P = M == 0 ? 1 : 3 * M;
    constexpr int GM = M == 0 ? 1 : 2 * M;
    constexpr int KG = (GM + 1) * (GM + 2) / 2;
    constexpr int HN = P >= 2 ? P - 1 : 1;
    constexpr bool F32 = std::is_same<R, float>::value;
    // shells n <= NF are generated and contracted in FP64: every entry g with
    // |g| <= M + 1 (what the centre velocity and the first-moment rates read)
    // takes terms from those shells only; the mixed kernel keeps the shells
    // above in FP32
    constexpr int NF = F32 ? 2 * M + 1 : P;
    constexpr double kInvPi = 0.318309886183790671537767526745;
    static_assert(P <= kPairConstShells, "edge coefficients of every shell");

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tpb = (blockDim.x >> 6) / split;
    const int jt = wave / split, sp = wave - jt * split;
    const int j = blockIdx.x * tpb + jt;
    const bool live = j < N;  // uniform per wavefront; every wave reaches the barrier below
    const int jc = live ? j : 0;

    const double xj1 = xt[2 * jc], xj2 = xt[2 * jc + 1], lj2 = lam2t[jc];
    const double ilj = 1.0 / sqrt(lj2);
    const double lj = lj2 * ilj;
    const int self = rank ? rank[jc] : jc;

    double acc[KG];
    R acc32[F32 ? KG : 1];
    sfor<0, KG>([&](auto g) { acc[g] = 0.0; });
    if constexpr (F32) sfor<0, KG>([&](auto g) { acc32[g] = 0.0f; });
    int pending = 0;

    // one source per lane: the pair (target j, source jp) added into acc
    auto visit = [&](int jp, bool own) {
        const double lp2 = lam2[jp];
        const double c = lj2 + lp2;
        const double isc = 1.0 / sqrt(c);
        const double s1 = (xj1 - xs[2 * jp]) * isc, s2 = (xj2 - xs[2 * jp + 1]) * isc;
        const double w = s1 * s1 + s2 * s2;
        if constexpr (FAR) {
            // every lane of the chunk takes part (the mask byte of each visited
            // chunk is rewritten each stage); the target's own source does not
            // count, and a chunk holding nothing else is near
            const bool all_far = __all(own || w > pair_far_w(P)) && __any(!own);  // uniform over the wavefront
            farmask[(long)j * pair_mask_stride(N) + (jp >> 6)] = all_far ? 1 : 0;
            if (all_far || own) return;
        }
        const double e1 = exp(-s1 * s1), e2 = exp(-s2 * s2);
        const double E = e1 * e2;

        // g_n = P(n, w) / w^n, n = 1..P (P the regularised lower incomplete
        // gamma function), by the downward recurrence g_n = w g_{n+1} + e^{-w}/n!
        // from g_P:  w <= P: g_P = e^{-w} sum_k w^k/(P+k)!  (fixed-length Horner);
        //            w >  P: g_P = (1 - e^{-w} sum_{k<P} w^k/k!) / w^P.
        // (the reciprocals 1/n are compile-time constants: no table loads in
        // these dependent chains)
        double gsr[P + 1];
        {
            constexpr double ifP = pair_inv_factorial(P);  // 1/P!
            double gP;
            if (w <= (double)P) {
                double term = ifP, sum = 0.0;
                sfor<0, kSeriesTerms>([&](auto k) {
                    sum += term;
                    term *= w * (1.0 / (double)(P + k + 1));
                });
                gP = E * sum;
            } else {
                double sm = 0.0, term = 1.0, wp = 1.0;
                sfor<0, P>([&](auto k) {
                    sm += term;
                    term *= w * (1.0 / (double)(k + 1));
                    wp *= w;
                });
                gP = (1.0 - E * sm) / wp;
            }
            gsr[P] = gP;
            double ifn = ifP;
            sfor<1, P>([&](auto q) {
                constexpr int n = P - q;  // P-1 .. 1
                ifn *= (double)(n + 1);   // 1/n!
                gsr[n] = fma(w, gsr[n + 1], E * ifn);
            });
        }

        // 1-D Gaussian derivatives h_a(x) = d^a/dx^a exp(-x^2) (FP64: the FP64 shells use them)
        double h1[HN], h2[HN];
        h1[0] = e1;
        h2[0] = e2;
        if constexpr (HN > 1) {
            h1[1] = (-2.0 * s1) * h1[0];
            h2[1] = (-2.0 * s2) * h2[0];
        }
        sfor<1, HN - 1>([&](auto a) {
            h1[a + 1] = (-2.0 * s1) * h1[a] - (double)(2 * a) * h1[a - 1];
            h2[a + 1] = (-2.0 * s2) * h2[a] - (double)(2 * a) * h2[a - 1];
        });

        // scaled source moments (FP64 for the FP64 shells, R for the others)
        double am[K];
        R am32[F32 ? K : 1];
        {
            const double ratio = sqrt(lp2) * ilj;
            double rp = 1.0;
            sfor<0, M + 1>([&](auto s) {
                sfor<0, s + 1>([&](auto m2) {
                    constexpr int idx = ctri(s - m2, m2);
                    am[idx] = (double)aT[(long)idx * N + jp] * rp;
                    if constexpr (F32) am32[idx] = (R)am[idx];
                });
                rp *= ratio;
            });
        }

        const double tau = lj * isc;
        double tn = 1.0;
        double zr = 1.0, zi = 0.0;
        sfor<1, P + 1>([&](auto nc) {
            constexpr int n = nc;
            // zbar^n
            {
                double nr = zr * s1 + zi * s2;  // (zr + i zi)(s1 - i s2)
                double ni = zi * s1 - zr * s2;
                zr = nr;
                zi = ni;
            }
            const double hr = kPairHol[n] * gsr[n] * zr, hi = kPairHol[n] * gsr[n] * zi;
            // 2 Re(i^n h), 2 Re(i^{n-1} h)
            double e0, e1v;
            if constexpr (n % 4 == 0) { e0 = hr; e1v = hi; }
            else if constexpr (n % 4 == 1) { e0 = -hi; e1v = hr; }
            else if constexpr (n % 4 == 2) { e0 = -hr; e1v = -hi; }
            else { e0 = hi; e1v = -hr; }
            typedef typename std::conditional<(n <= NF), double, R>::type T;
            T psi[n + 1];
            T p0 = (T)(2.0 * e0), p1 = (T)(2.0 * e1v);
            T prod[n >= 2 ? n - 1 : 1];
            if constexpr (n >= 2) {
                sfor<0, n - 1>([&](auto cc) {
                    prod[cc] = (T)h1[cc] * (T)h2[n - 2 - cc];
                    p0 += (T)kPairKappa0[n][cc] * prod[cc];
                    p1 += (T)kPairKappa1[n][cc] * prod[cc];
                });
            }
            psi[0] = p0;
            psi[1] = p1;
            if constexpr (n >= 2) {
                sfor<0, n - 1>([&](auto a) { psi[a + 2] = prod[a] * (T)kInvPi - psi[a]; });
            }
            tn *= tau;
            sfor<0, n + 1>([&](auto a) { psi[a] *= (T)tn; });
            // Hankel contraction of this shell
            sfor<0, n + 1>([&](auto a) {
                constexpr int m1max = a < M ? (int)a : M;
                sfor<0, m1max + 1>([&](auto m1) {
                    constexpr int rem = M - m1;
                    constexpr int m2max = (n - a) < rem ? (n - a) : rem;
                    sfor<0, m2max + 1>([&](auto m2) {
                        constexpr int g1 = a - m1, g2 = n - a - m2;
                        if constexpr (g1 + g2 >= 1 && g1 + g2 <= GM) {
                            if constexpr (n > NF)
                                acc32[ctri(g1, g2)] += am32[ctri(m1, m2)] * psi[a];
                            else
                                acc[ctri(g1, g2)] = fma(am[ctri(m1, m2)], psi[a], acc[ctri(g1, g2)]);
                        }
                    });
                });
            });
        });
        if constexpr (F32) {
            if (++pending == 8) {
                sfor<0, KG>([&](auto g) { acc[g] += (double)acc32[g]; acc32[g] = 0.0f; });
                pending = 0;
            }
        }
    };
    const int nch = (N + 63) >> 6;
    if constexpr (FAR) {
        if (crec) {
            // A chunk whose record (centre, radius r_c, largest lambda^2) puts
            // every source beyond the threshold is far without reading its
            // sources: |x_j - x_q| >= rho - r_c, so w_q >= (rho - r_c)^2 /
            // (lambda_j^2 + max lambda^2).  The records of 64 chunks at a time,
            // one per lane: the provably far ones are flagged with one store, and
            // the wavefront visits only the others of its share (chunk
            // c = sp mod split, in increasing order as below), which take the
            // exact test (the same flags either way, up to a margin of rounding).
            const unsigned long long mine = split == 1   ? ~0ull
                                            : split == 2 ? 0x5555555555555555ull << sp
                                                         : 0x1111111111111111ull << sp;
            for (int g0 = 0; live && g0 < nch; g0 += 64) {
                const int cc = g0 + lane;
                bool bf = false;
                if (cc < nch) {
                    const double* r = crec + (long)cc * kChunkRec;
                    const double e1 = xj1 - r[0], e2 = xj2 - r[1];
                    const double gap = sqrt(e1 * e1 + e2 * e2) - r[2];
                    bf = gap > 0.0 && gap * gap > kFarBoundMargin * pair_far_w(P) * (lj2 + r[3]);
                }
                if (bf && (cc & (split - 1)) == sp) farmask[(long)j * pair_mask_stride(N) + cc] = 1;
                const unsigned long long valid = nch - g0 >= 64 ? ~0ull : (1ull << (nch - g0)) - 1;
                unsigned long long todo = ~__ballot(bf) & valid & mine;  // uniform per wavefront
                while (todo) {
                    const int c = g0 + __builtin_ctzll(todo);
                    todo &= todo - 1;
                    const int jp = c * 64 + lane;
                    if (jp < N) visit(jp, jp == self);
                }
            }
        } else {
            for (int jp = sp * 64 + lane; live && jp < N; jp += 64 * split) visit(jp, jp == self);
        }
    } else {
        for (int jp = sp * 64 + lane; live && jp < N; jp += 64 * split)
            if (jp != self) visit(jp, false);
    }
    if constexpr (F32) sfor<0, KG>([&](auto g) { acc[g] += (double)acc32[g]; });

    // wavefront reduction over the sources held by the 64 lanes
    extern __shared__ double red_pair[];  // [waves][KG] when split > 1
    double* out = split == 1 ? spair + (long)jc * KG : red_pair + wave * KG;
    sfor<1, KG>([&](auto g) {
        double v = acc[g];
        v += __shfl_xor(v, 32, 64);
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 8, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 1, 64);
        if (lane == (g & 63) && (live || split > 1)) out[g] = v;
    });
    if (split == 1) {
        if (live && lane == 0) spair[(long)j * KG] = 0.0;
        return;
    }
    __syncthreads();
    if (!live || sp != 0) return;
    for (int g = lane; g < KG; g += 64) {
        double v = 0.0;
        if (g > 0)
            for (int q = 0; q < split; ++q) v += red_pair[(wave + q) * KG + g];
        spair[(long)j * KG + g] = v;
    }
}

// Orders LDS writes of some lanes of a wavefront before later reads by other
// lanes of the same wavefront (its LDS operations complete in order).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The pairs of the chunks marked far, added to the pair table after the near
// kernel (FP64 in both precisions; the same multipole form for every shape):
//   Q_s = sum_{|m| = s} alpha'_m i^{m2},  T_p = sum_s Q_s H_{s+p},
//   S[g] += 2 Re(i^{g2} T_{|g|}),  H_n = hol[n] (lambda_j / Delta z)^n,
// Delta z = (x^j - x^{j'})_1 + i (x^j - x^{j'})_2, generated shell by shell
// (lanes over the 64 sources of a chunk), or for a whole chunk or cell through
// its expansion where that converges (queued, several per wavefront pass).
// A workgroup of kFarWaves wavefronts takes one target.  For each group of 64
// chunks every wavefront reads the flags, the chunk and the cell decisions
// lane-parallel (one record load per lane), then takes its share: the
// accepted cells k = q mod kFarWaves and the other far chunks
// c = q mod kFarWaves (the far chunks of a target tend to be runs of
// consecutive sorted chunks: the targets at the edge of a dense region carry
// many, the others none).  A target with no far chunk costs one load per
// group; the wavefront sums meet in LDS in wavefront order.
constexpr int kFarWaves = 4;
constexpr int kFarThreads = 64 * kFarWaves;

template <int M>
__global__ __launch_bounds__(kFarThreads) void k_pair_far(int N, const double* __restrict__ xt,
                                                          const double* __restrict__ lam2t,
                                                          const double* __restrict__ xs,
                                                          const double* __restrict__ lam2,
                                                          const double* __restrict__ aT,
                                                          const unsigned char* __restrict__ farmask,
                                                          const int* __restrict__ rank,
                                                          const double* __restrict__ cmp,
                                                          const double* __restrict__ cells, double* __restrict__ spair)
{
    constexpr int P = M == 0 ? 1 : 3 * M;
    constexpr int GM = M == 0 ? 1 : 2 * M;
    constexpr int KG = (GM + 1) * (GM + 2) / 2;
    // a far chunk of radius r_c at distance |zeta| from the target takes its
    // multipole expansion when r_c <= theta |zeta|: the truncation after
    // kFarPM terms is then below ~3e-14 of the chunk's own contribution for
    // every derivative order p <= 2M (the tail ratio of term n is about
    // theta^n C(n + p - 1, n))
    constexpr double kTheta2 = M >= 5 ? 0.0625 : 0.09;
    static_assert(kFarPM + GM <= kPairHolFarMax, "hol[n] of every expansion term");
    __shared__ double red[kFarWaves][2 * GM + 2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, j = blockIdx.x;
    // chunk c0 + b of a group of 64 belongs to this wavefront when b = wave mod
    // kFarWaves, cell k (chunks k kFarCellChunks ...) when k = wave mod kFarWaves
    static_assert(64 % kFarCellChunks == 0, "cells tile a group of 64 chunks");
    unsigned long long mine = 0;
    for (int b = wave; b < 64; b += kFarWaves) mine |= 1ull << b;
    const int stride = pair_mask_stride(N), nch = (N + 63) >> 6;
    const unsigned char* row = farmask + (long)j * stride;
    const int self = rank ? rank[j] : j;
    const double xj1 = xt[2 * j], xj2 = xt[2 * j + 1], lj2 = lam2t[j];
    const double ilj = 1.0 / sqrt(lj2), lj = lj2 * ilj;
    // T_p summed over the lane's pairs (S is linear in T: expanded to the
    // entries g once, after the wavefront sum)
    double Tr[GM + 1], Ti[GM + 1];
    sfor<1, GM + 1>([&](auto p) { Tr[p] = 0.0; Ti[p] = 0.0; });
    // Expansions (chunk or cell records) are queued per wavefront and evaluated
    // kRB at a time: lane (g, p - 1) takes queued record g and derivative order
    // p, S_p = sum_n hol[n + p] B_n u^n by Horner's rule in u = 1 / zeta
    // (zeta = z_j - z_c), then T_p += (lambda_j u)^p S_p.  The coefficients of
    // a batch are staged in LDS (one lane-parallel copy), the factors hol[m]
    // once per wavefront.
    constexpr int kPL = GM <= 8 ? 8 : 16;  // lanes per queued record
    constexpr int kRB = 64 / kPL;          // records per batch
    constexpr int kBT = 2 * (kFarPM + 1);  // doubles of B in a record
    static_assert(kFarPM + GM < 64, "a lane per factor hol[m]");
    __shared__ double hol_s[kFarWaves][kFarPM + GM + 1];  // a copy per wavefront: no workgroup barrier
    __shared__ double bq[kFarWaves][kRB][kBT];
    __shared__ int qid[kFarWaves][kRB];
    if (lane <= kFarPM + GM) hol_s[wave][lane] = kPairHolFar[lane];
    int qn = 0;  // queued records of this wavefront (uniform)
    // the expansions' T_p of this lane's fixed p = lane mod kPL + 1, added into
    // the sum over lanes of T_p at the end (a separate register: no indexing of
    // T by a lane-dependent p)
    const int ep = lane % kPL + 1;
    double er = 0.0, ei = 0.0;
    auto flush = [&]() __attribute__((always_inline)) {
        wave_lds_sync();
        for (int e = lane; e < qn * kBT; e += 64) {
            const int r = e / kBT, t = e - r * kBT;
            bq[wave][r][t] = cmp[(long)qid[wave][r] * kChunkRec + 4 + t];
        }
        wave_lds_sync();
        const int g = lane / kPL, p = ep;
        if (g < qn && p <= GM) {
            const double* rec = cmp + (long)qid[wave][g] * kChunkRec;
            const double zr = xj1 - rec[0], zi = xj2 - rec[1];
            const double id = 1.0 / (zr * zr + zi * zi);
            const double ur = zr * id, ui = -zi * id;  // 1 / zeta
            const double* b = bq[wave][g];
            double sr = 0.0, si = 0.0;
#pragma unroll 2
            for (int n = kFarPM; n >= 0; --n) {
                const double h = hol_s[wave][n + p];
                const double tr = sr * ur - si * ui + h * b[2 * n];
                si = sr * ui + si * ur + h * b[2 * n + 1];
                sr = tr;
            }
            double wr = 1.0, wi = 0.0, qr = lj * ur, qi = lj * ui;
            for (int e = p; e; e >>= 1) {  // (lambda_j u)^p
                if (e & 1) {
                    const double t = wr * qr - wi * qi;
                    wi = wr * qi + wi * qr;
                    wr = t;
                }
                const double t = qr * qr - qi * qi;
                qi = 2.0 * qr * qi;
                qr = t;
            }
            er += sr * wr - si * wi;
            ei += sr * wi + si * wr;
        }
        wave_lds_sync();  // the queue and the staged coefficients are reused
        qn = 0;
    };
    auto push = [&](const double* rec) __attribute__((always_inline)) {
        if (lane == 0) qid[wave][qn] = (int)((rec - cmp) / kChunkRec);
        if (++qn == kRB) flush();
    };
    int any = 0;  // this wavefront had far chunks
    for (int c0 = 0; c0 < nch; c0 += 64) {
        // the decisions of a group of 64 chunks, lane-parallel (one record load
        // each): flag, chunk expansion converging here, cell expansion
        // converging here for cells whose chunks are all far
        const bool flag = c0 + lane < nch && row[c0 + lane] != 0;
        unsigned long long far = __ballot(flag);  // uniform per wavefront
        bool cexp = false;
        if (cmp && flag) {
            const double* rec = cmp + (long)(c0 + lane) * kChunkRec;
            const double zr = xj1 - rec[0], zi = xj2 - rec[1], rc = rec[2];
            const double rho2 = zr * zr + zi * zi;
            cexp = rho2 > 0.0 && rc * rc <= kTheta2 * rho2;
        }
        const unsigned long long chunk_exp = __ballot(cexp);
        if (cells) {
            // a cell whose chunks are all far takes its own expansion where that
            // converges (one record for kFarCellChunks chunks): every wavefront
            // has the same decisions, takes its share of these cells, and drops
            // their chunks from the per-chunk work
            bool kexp = false;
            const int b = kFarCellChunks * lane, c = c0 + b;
            if (lane < 64 / kFarCellChunks && c < nch) {
                const int nc = nch - c < kFarCellChunks ? nch - c : kFarCellChunks;
                const unsigned long long need = ((1ull << nc) - 1) << b;
                if ((far & need) == need) {
                    const double* rec = cells + (long)(c / kFarCellChunks) * kChunkRec;
                    const double zr = xj1 - rec[0], zi = xj2 - rec[1], rc = rec[2];
                    const double rho2 = zr * zr + zi * zi;
                    kexp = rho2 > 0.0 && rc * rc <= kTheta2 * rho2;
                }
            }
            unsigned long long kq = __ballot(kexp), taken = 0;
            while (kq) {
                const int k = __builtin_ctzll(kq);
                kq &= kq - 1;
                taken |= ((1ull << kFarCellChunks) - 1) << (kFarCellChunks * k);
                if (k % kFarWaves == wave) {
                    any = 1;
                    push(cells + (long)((c0 >> 6) * (64 / kFarCellChunks) + k) * kChunkRec);
                }
            }
            far &= ~taken;
        }
        far &= mine;
        any |= far != 0;
        while (far) {
            const int c = c0 + __builtin_ctzll(far);
            if ((chunk_exp >> (c - c0)) & 1ull) {
                far &= far - 1;
                push(cmp + (long)c * kChunkRec);
                continue;
            }
            far &= far - 1;
            const int jp = c * 64 + lane;
            if (jp >= N || jp == self) continue;
            const double lp2 = lam2[jp];
            const double isc = 1.0 / sqrt(lj2 + lp2);
            const double s1 = (xj1 - xs[2 * jp]) * isc, s2 = (xj2 - xs[2 * jp + 1]) * isc;
            const double w = s1 * s1 + s2 * s2;
            const double ratio = sqrt(lp2) * ilj, tz = lj * isc / w;
            const double ur = tz * s1, ui = -tz * s2;  // lambda_j / Delta z
            double Qr[M + 1], Qi[M + 1];
            {
                double rp = 1.0;
                sfor<0, M + 1>([&](auto s) {
                    double qr = 0.0, qi = 0.0;
                    sfor<0, s + 1>([&](auto m2) {
                        const double a = aT[(long)ctri(s - m2, m2) * N + jp] * rp;
                        if constexpr (m2 % 4 == 0) qr += a;
                        else if constexpr (m2 % 4 == 1) qi += a;
                        else if constexpr (m2 % 4 == 2) qr -= a;
                        else qi -= a;
                    });
                    Qr[s] = qr;
                    Qi[s] = qi;
                    rp *= ratio;
                });
            }
            double pr = 1.0, pim = 0.0;
            sfor<1, P + 1>([&](auto nc) {
                constexpr int n = nc;
                const double nr = pr * ur - pim * ui, ni = pr * ui + pim * ur;
                pr = nr;
                pim = ni;
                const double hr = kPairHol[n] * pr, hi = kPairHol[n] * pim;
                sfor<0, M + 1>([&](auto s) {
                    constexpr int p = n - s;
                    if constexpr (p >= 1 && p <= GM) {
                        Tr[p] += Qr[s] * hr - Qi[s] * hi;
                        Ti[p] += Qr[s] * hi + Qi[s] * hr;
                    }
                });
            });
        }
    }
    if (qn) flush();
    // a target without far chunks (most of a dense field) leaves here
    if (!__syncthreads_or(any)) return;
    sfor<1, GM + 1>([&](auto p) {
        double vr = Tr[p] + (ep == p ? er : 0.0), vi = Ti[p] + (ep == p ? ei : 0.0);
        for (int off = 32; off > 0; off >>= 1) {
            vr += __shfl_xor(vr, off, 64);
            vi += __shfl_xor(vi, off, 64);
        }
        if (lane == 0) {
            red[wave][2 * p] = vr;
            red[wave][2 * p + 1] = vi;
        }
    });
    __syncthreads();
    if (wave != 0) return;
    sfor<1, GM + 1>([&](auto p) {
        double vr = red[0][2 * p], vi = red[0][2 * p + 1];
        for (int q = 1; q < kFarWaves; ++q) {
            vr += red[q][2 * p];
            vi += red[q][2 * p + 1];
        }
        sfor<0, p + 1>([&](auto g2) {
            constexpr int g1 = p - g2;
            constexpr int g = ctri(g1, g2);
            const double v = (g2 % 4 == 0) ? vr : (g2 % 4 == 1) ? -vi : (g2 % 4 == 2) ? -vr : vi;
            if (lane == (g & 63)) spair[(long)j * KG + g] += 2.0 * v;
        });
    });
}

// Multipole expansion of each chunk of 64 sorted sources about its centre z_c
// (the mean of its positions).  Beyond the cores the field of source q is
// sum_s Qu_s L^(s)(z - z_q), L^(s) the s-th complex derivative of the
// harmonic potential (L^(n)(z) = hol[n] / z^n), Qu_s = sum_{|m| = s} M_m i^{m2}
// its unscaled multipoles; the Taylor series of L^(s) about z - z_c gives the
// chunk's field as sum_n B_n L^(n)(z - z_c),
//   B_n = sum_q sum_{s <= min(n, M)} Qu_{q,s} (-d_q)^{n-s} / (n-s)!,  d_q = z_q - z_c,
// convergent for |z - z_c| > max |d_q| (the chunk radius), kept to n = kFarPM.
// The record: centre, radius, the largest lambda^2 of the chunk, then B_n.
// One workgroup per chunk, lane = source.  Every wavefront forms the centre
// (the same shuffle trees, so the same bits), its sources' multipoles and the
// factors (-d)^m / m! by their recurrence; wavefront w keeps the per-source
// terms of B_n for its quarter of the n range, in LDS.  Thread t then adds
// column t (a real or imaginary part of one B_n) over the 64 sources: four
// interleaved partial sums in source order, combined pairwise.
constexpr int kMpTerms = kFarPM + 1;
constexpr int kMpPerWave = (kMpTerms + 3) / 4;
static_assert(2 * kMpTerms <= 256, "a thread per column of the chunk sums");

template <int M>
__global__ __launch_bounds__(256) void k_chunk_multipoles(int N, const double* __restrict__ xs,
                                                          const double* __restrict__ lam2,
                                                          const double* __restrict__ aT, double* __restrict__ cmp)
{
    __shared__ double part[2 * kMpTerms][65];  // [column][source]; odd row length spreads the banks
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, c = blockIdx.x;
    const int q = c * 64 + lane;
    const bool live = q < N;
    const double x1 = live ? xs[2 * q] : 0.0, x2 = live ? xs[2 * q + 1] : 0.0;
    double s1 = x1, s2 = x2, cnt = live ? 1.0 : 0.0;
    for (int off = 32; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off, 64);
        s2 += __shfl_xor(s2, off, 64);
        cnt += __shfl_xor(cnt, off, 64);
    }
    const double c1 = s1 / cnt, c2 = s2 / cnt;
    const double d1 = live ? x1 - c1 : 0.0, d2 = live ? x2 - c2 : 0.0;
    double r2 = d1 * d1 + d2 * d2;
    const double l2q = live ? lam2[q] : 0.0;
    double l2m = l2q;
    for (int off = 32; off > 0; off >>= 1) {
        r2 = fmax(r2, __shfl_xor(r2, off, 64));
        l2m = fmax(l2m, __shfl_xor(l2m, off, 64));
    }
    double qr[M + 1], qi[M + 1];
    sfor<0, M + 1>([&](auto s) { qr[s] = 0.0; qi[s] = 0.0; });
    if (live) {
        const double lq = sqrt(l2q);
        double lp = 1.0;  // lambda_q^s: the unscaled moments M = alpha lambda^{|m|}
        sfor<0, M + 1>([&](auto s) {
            sfor<0, s + 1>([&](auto m2) {
                const double a = aT[(long)ctri(s - m2, m2) * N + q] * lp;
                if constexpr (m2 % 4 == 0) qr[s] += a;
                else if constexpr (m2 % 4 == 1) qi[s] += a;
                else if constexpr (m2 % 4 == 2) qr[s] -= a;
                else qi[s] -= a;
            });
            lp *= lq;
        });
    }
    double* rec = cmp + (long)c * kChunkRec;
    if (threadIdx.x == 0) {
        rec[0] = c1;
        rec[1] = c2;
        rec[2] = sqrt(r2);
        rec[3] = l2m;  // the largest lambda^2 of the chunk (for the near kernel's far test)
    }
    // e_k = (-d)^k / k!: er[s], ei[s] hold e_{n - s} (zero for n - s < 0)
    const int n0 = wave * kMpPerWave, n1 = n0 + kMpPerWave < kMpTerms ? n0 + kMpPerWave : kMpTerms;
    double er[M + 1], ei[M + 1];
    sfor<0, M + 1>([&](auto s) { er[s] = 0.0; ei[s] = 0.0; });
    double pr = 1.0, pim = 0.0;  // e_n
    for (int n = 0; n < n1; ++n) {  // uniform per wavefront
        if (n > 0) {
            const double f = 1.0 / (double)n;
            const double nr = -(pr * d1 - pim * d2) * f, ni = -(pr * d2 + pim * d1) * f;
            pr = nr;
            pim = ni;
        }
        sfor<0, M>([&](auto t) {
            constexpr int s = M - t;  // M .. 1
            er[s] = er[s - 1];
            ei[s] = ei[s - 1];
        });
        er[0] = pr;
        ei[0] = pim;
        if (n >= n0) {
            double br = 0.0, bi = 0.0;
            sfor<0, M + 1>([&](auto s) {
                br += qr[s] * er[s] - qi[s] * ei[s];
                bi += qr[s] * ei[s] + qi[s] * er[s];
            });
            part[2 * n][lane] = br;
            part[2 * n + 1][lane] = bi;
        }
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < 2 * kMpTerms) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 64; k += 4) {
            a[0] += part[t][k];
            a[1] += part[t][k + 1];
            a[2] += part[t][k + 2];
            a[3] += part[t][k + 3];
        }
        rec[4 + t] = (a[0] + a[1]) + (a[2] + a[3]);
    }
}

// Expansion of each cell of kFarCellChunks consecutive chunks about its centre
// z_K (the mean of its sources' positions, from the chunks' centres and source
// counts), translated from the chunks' expansions: with delta_c = z_c - z_K,
//   B^K_n = sum_c sum_{k <= n} B^c_k (-delta_c)^{n-k} / (n-k)!
// (term n needs the chunks' terms up to n only, so the truncation is theirs);
// radius max_c (|delta_c| + r_c).  A workgroup per cell, wavefront w = chunk w
// of the cell, lane n = term; the chunks' terms meet in LDS and are added in
// chunk order.  (Instantiated per order only to live in the unit of that order.)
template <int M>
__global__ __launch_bounds__(256) void k_cell_multipoles(int N, const double* __restrict__ cmp,
                                                         double* __restrict__ cells)
{
    static_assert(kFarCellChunks * 64 == 256, "a wavefront per chunk of the cell");
    __shared__ double sb[kFarCellChunks][2 * kMpTerms];
    __shared__ double sa[kFarCellChunks][2 * kMpTerms];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, k = blockIdx.x;
    const int nch = (N + 63) >> 6, cfirst = k * kFarCellChunks;
    for (int e = threadIdx.x; e < kFarCellChunks * 2 * kMpTerms; e += 256) {
        const int w = e / (2 * kMpTerms), t = e - w * (2 * kMpTerms);
        sb[w][t] = cfirst + w < nch ? cmp[(long)(cfirst + w) * kChunkRec + 4 + t] : 0.0;
    }
    // centre and radius (every thread the same values, chunks in order)
    double s1 = 0.0, s2 = 0.0, cnt = 0.0;
    for (int w = 0; w < kFarCellChunks && cfirst + w < nch; ++w) {
        const double* r = cmp + (long)(cfirst + w) * kChunkRec;
        const int left = N - (cfirst + w) * 64;
        const double n = (double)(left < 64 ? left : 64);
        s1 += n * r[0];
        s2 += n * r[1];
        cnt += n;
    }
    const double z1 = s1 / cnt, z2 = s2 / cnt;
    double rad = 0.0, l2m = 0.0;
    for (int w = 0; w < kFarCellChunks && cfirst + w < nch; ++w) {
        const double* r = cmp + (long)(cfirst + w) * kChunkRec;
        const double e1 = r[0] - z1, e2 = r[1] - z2;
        rad = fmax(rad, sqrt(e1 * e1 + e2 * e2) + r[2]);
        l2m = fmax(l2m, r[3]);
    }
    __syncthreads();
    if (lane < kMpTerms) {
        double ar = 0.0, ai = 0.0;
        if (cfirst + wave < nch) {
            const double* r = cmp + (long)(cfirst + wave) * kChunkRec;
            const double d1 = z1 - r[0], d2 = z2 - r[1];  // -delta_c
            double er = 1.0, ei = 0.0;                    // (-delta_c)^m / m!
            for (int m = 0; m <= lane; ++m) {
                const double br = sb[wave][2 * (lane - m)], bi = sb[wave][2 * (lane - m) + 1];
                ar += br * er - bi * ei;
                ai += br * ei + bi * er;
                const double f = 1.0 / (double)(m + 1);
                const double nr = (er * d1 - ei * d2) * f, ni = (er * d2 + ei * d1) * f;
                er = nr;
                ei = ni;
            }
        }
        sa[wave][2 * lane] = ar;
        sa[wave][2 * lane + 1] = ai;
    }
    __syncthreads();
    double* rec = cells + (long)k * kChunkRec;
    const int t = threadIdx.x;
    if (t < 2 * kMpTerms) {
        double v = sa[0][t];
        for (int w = 1; w < kFarCellChunks; ++w) v += sa[w][t];
        rec[4 + t] = v;
    }
    if (t == 0) {
        rec[0] = z1;
        rec[1] = z2;
        rec[2] = rad;
        rec[3] = l2m;
    }
}

template <int M>
hipError_t launch_pair_M(const DevTables& T, const StageBufs& B, int cur, bool f32, PairShape sh, hipStream_t st)
{
    constexpr int GM = M == 0 ? 1 : 2 * M;
    constexpr int KG = (GM + 1) * (GM + 2) / 2;
    if (!pair_shape_valid(sh)) return hipErrorInvalidValue;
    if (sh.kind == 1) return B.rank ? hipErrorInvalidValue : launch_pair_split_M<M>(T, B, cur, st);
    if (sh.far && !B.far_mask) return hipErrorInvalidValue;
    const int waves = sh.split * sh.tpb;
    dim3 grid((B.N + sh.tpb - 1) / sh.tpb);
    const size_t shmem = sh.split > 1 ? sizeof(double) * (size_t)waves * KG : 0;
    const bool use32 = f32 && !sh.f64 && M <= kPairF32MaxOrder;
    const double* xt = B.xs;
    const double* lt = B.lam2[cur];
    const double* xsrc = B.xsS;
    const double* lsrc = B.lam2S[cur];
    // With the far split and sorted sources the chunk records come first: the
    // near kernel reads them to skip provably far chunks, the far kernel takes
    // distant chunks (and cells of kFarCellChunks chunks) through their
    // expansions.  MMVM_FAR_M2P=0 keeps every far pair on the pairwise form,
    // MMVM_FAR_CELLS=0 the chunk expansions but not the cells'.
    const bool recs = sh.far && B.rank && B.chunk_mp;
    const char* env = std::getenv("MMVM_FAR_M2P");
    const bool m2p = !(env && env[0] == '0');
    const double* cmp = (recs && m2p) ? B.chunk_mp : nullptr;
    const int nch = (B.N + 63) >> 6, ncell = (nch + kFarCellChunks - 1) / kFarCellChunks;
    const char* cenv = std::getenv("MMVM_FAR_CELLS");
    // one cell holds every source (the target's own among them): never used
    double* cells = (cmp && ncell > 1 && !(cenv && cenv[0] == '0')) ? B.chunk_mp + (long)nch * kChunkRec : nullptr;
    if (recs) {
        TimingSlot* outer = timing_slot();  // the caller's slot times the near kernel
        timing_slot() = nullptr;
        void* tk = timing_begin(st);
        launch_kernel((k_chunk_multipoles<M>), dim3(nch), dim3(256), 0, st, B.N, xsrc, lsrc,
                      (const double*)B.alphaT[cur], B.chunk_mp);
        if (cells)
            launch_kernel((k_cell_multipoles<M>), dim3(ncell), dim3(256), 0, st, B.N, (const double*)B.chunk_mp,
                          cells);
        timing_end(tk, "pair_mp", st);
        timing_slot() = outer;
    }
    const double* crec = recs ? B.chunk_mp : nullptr;
    if (use32 && sh.far)
        launch_kernel((k_pair<M, float, true>), grid, dim3(64 * waves), shmem, st, B.N, sh.split, xt, lt, xsrc, lsrc,
                      (const float*)B.alphaT32[cur], B.s_pair, B.far_mask, B.rank, crec);
    else if (use32)
        launch_kernel((k_pair<M, float, false>), grid, dim3(64 * waves), shmem, st, B.N, sh.split, xt, lt, xsrc, lsrc,
                      (const float*)B.alphaT32[cur], B.s_pair, B.far_mask, B.rank, (const double*)nullptr);
    else if (sh.far)
        launch_kernel((k_pair<M, double, true>), grid, dim3(64 * waves), shmem, st, B.N, sh.split, xt, lt, xsrc,
                      lsrc, (const double*)B.alphaT[cur], B.s_pair, B.far_mask, B.rank, crec);
    else
        launch_kernel((k_pair<M, double, false>), grid, dim3(64 * waves), shmem, st, B.N, sh.split, xt, lt, xsrc,
                      lsrc, (const double*)B.alphaT[cur], B.s_pair, B.far_mask, B.rank, (const double*)nullptr);
    if (sh.far) {
        // timed on its own (the caller's slot took the near kernel)
        void* tk = timing_begin(st);
        launch_kernel((k_pair_far<M>), dim3(B.N), dim3(kFarThreads), 0, st, B.N, xt, lt, xsrc, lsrc,
                      (const double*)B.alphaT[cur], (const unsigned char*)B.far_mask, B.rank, cmp,
                      (const double*)cells, B.s_pair);
        timing_end(tk, "pair_far", st);
    }
    return hipGetLastError();
}

}  // namespace mmvm
