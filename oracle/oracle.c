/*
 * oracle.c -- plain, slow CPU evaluation of the multi-moment vortex method
 * (MMVM) moment equations of Uminsky, Wayne & Barbaro, "A multi-moment
 * vortex method for 2D viscous fluids" (arXiv:1010.2475).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the CPU-baseline leg of the benchmark load this library.  It shares no code
 * with the HIP library: every formula below is written out from the paper's
 * appendix ("Combinatorial formulae"), term by term, in the paper's order.
 *
 * Arithmetic is quad precision (__float128).  The paper generated its ODE
 * coefficients symbolically (Maple, section "A note on implementation and
 * performance"), i.e. exactly.  The combinatorial sums eq:FinalSingleI/II are
 * alternating sums whose largest terms exceed the coefficient by up to ~1e18
 * at order 24 and ~1e27 at order 40, so evaluating them in FP64 would not
 * reproduce the paper's coefficients; 113-bit arithmetic does at the orders
 * the tests use.  Inputs and outputs are FP64.
 *
 * Readings of the paper that this file fixes (each is pinned by a test):
 *  R1  dM/dt = + c_k sum Gamma~ M M   (eq:moment_evolutionFinish), Gamma~ = Gamma^I + Gamma^II.
 *  R2  in the pair term B the binomial index l belongs to the target vortex j
 *      and the velocity index m to the source j'  (the derivation of Gamma^I
 *      puts l on the vorticity and m on the velocity).
 *  R3  s_{j,j'} = x^j - x^{j'}  (the argument of u^{j'} in eq:xjdot).
 *  R4  the centre velocity sums over j' != j (eq:xjdot).
 *  R5  every sum over l, m, k is truncated at total order <= M.
 *  R6  per-vortex core scales: lambda_j^2 = lambda_{j,0}^2 + 4 nu t; the
 *      pair kernel H^B uses Lambda^2 = lambda_j^2 + lambda_{j'}^2 in place of
 *      the paper's 2 lambda^2 (Gaussian convolution adds squared widths, as in
 *      eq:Fullint); all other lambda factors are the target's lambda_j.
 *  R7  Gamma^II uses the second velocity component (H_2).
 *  R11 time stepping is classic RK4 in physical time on (x^j, M^j).
 *
 * Moment layout: shell-major, ord k = k1+k2 = 0..M, then k2 ascending;
 * index(k1,k2) = s(s+1)/2 + k2 with s = k1+k2; K = (M+1)(M+2)/2 per vortex.
 */
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef __float128 R;

#define NFACT 400
#define NB 200
static R g_fact[NFACT];
static R g_binom[NB][NB];
/* g_f0[k][i] = 2^i k!/(k-i)!,  g_f1[k][i] = 2^{i+1} k!/(k-i-1)!  (factors of
 * eq:FinalSingleI/II without their lambda powers) */
static R g_f0[NB][NB], g_f1[NB][NB];
static int g_fact_ready = 0;

static void init_fact(void)
{
    if (g_fact_ready) return;
    g_fact[0] = 1;
    for (int i = 1; i < NFACT; ++i) g_fact[i] = g_fact[i - 1] * (R)i;
    for (int n = 0; n < NB; ++n)
        for (int k = 0; k < NB; ++k) {
            g_binom[n][k] = (k <= n) ? g_fact[n] / (g_fact[k] * g_fact[n - k]) : 0;
            R p2 = 1;
            for (int e = 0; e < k; ++e) p2 *= 2;
            g_f0[n][k] = (k <= n) ? p2 * g_fact[n] / g_fact[n - k] : 0;
            g_f1[n][k] = (k + 1 <= n) ? 2 * p2 * g_fact[n] / g_fact[n - k - 1] : 0;
        }
    g_fact_ready = 1;
}

static R fact(int n) { return g_fact[n]; }
static R binom(int n, int k)
{
    if (k < 0 || k > n) return 0;
    return g_binom[n][k];
}
static R ipow(R x, int n)
{
    R r = 1;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}
static R sgn(int n) { return (n & 1) ? (R)-1 : (R)1; }

static int K_of(int M) { return (M + 1) * (M + 2) / 2; }
static int idx(int k1, int k2)
{
    int s = k1 + k2;
    return s * (s + 1) / 2 + k2;
}

int oracle_K(int M) { return K_of(M); }

/* threads of the parallel loops (the CPU-baseline timing runs 1 and all) */
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------
 * H_1, H_2: derivatives at b = 0 of the two components of the velocity of a
 * Gaussian of squared width Lam2 (the paper writes 2 lambda^2), appendix
 * "The Single Vortex Case", the closed forms for H_1 and H_2.
 * ---------------------------------------------------------------------- */
static R H1_origin(int a1, int a2, R Lam2)
{
    if ((a1 % 2) != 0 || (a2 % 2) != 1) return 0;
    int n = (a1 + a2 - 1) / 2;
    return -1 / (2 * M_PIq) * ipow(1 / Lam2, n + 1) * sgn(n) / fact(n + 1) *
           binom(n, a1 / 2) * fact(a1) * fact(a2);
}
static R H2_origin(int a1, int a2, R Lam2)
{
    if ((a1 % 2) != 1 || (a2 % 2) != 0) return 0;
    int n = (a1 + a2 - 1) / 2;
    return 1 / (2 * M_PIq) * ipow(1 / Lam2, n + 1) * sgn(n) / fact(n + 1) *
           binom(n, (a1 - 1) / 2) * fact(a1) * fact(a2);
}

/* ------------------------------------------------------------------------
 * H^B: D^alpha of V00(b; Lambda) at a point b = s (appendix, multi-vortex
 * expansion: the definition of H^B).  V00 = (1/2pi)(-b2, b1)/|b|^2
 * (1 - exp(-|b|^2/Lam2)).  Evaluated exactly through the complex form
 *   F = u1 - i u2 = (1 - exp(-z zbar/Lam2)) / (2 pi i z),  z = b1 + i b2,
 * D_{b1} = d + dbar, D_{b2} = i (d - dbar):
 *   d^p F         = (-1)^p p! P(p+1, w) / (2 pi i z^{p+1}),  w = z zbar / Lam2,
 *   d^p dbar^q F  = d^p dbar^{q-1} exp(-z zbar/Lam2) / (2 pi i Lam2),  q >= 1,
 *   d^p dbar^r E  = E sum_t C(p,t) (-1/Lam2)^r r!/(r-t)! z^{r-t} (-zbar/Lam2)^{p-t},
 * with P the regularised lower incomplete gamma function.  H^B_1 = Re D^a F,
 * H^B_2 = -Im D^a F.  P(p+1,w)/z^{p+1} is written (zbar/Lam2)^{p+1} P/w^{p+1},
 * which stays finite as z -> 0.
 * ---------------------------------------------------------------------- */
typedef struct { R re, im; } C;
static C cmk(R re, R im) { C c; c.re = re; c.im = im; return c; }
static C cadd(C a, C b) { return cmk(a.re + b.re, a.im + b.im); }
static C cmul(C a, C b) { return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static C cscale(C a, R s) { return cmk(a.re * s, a.im * s); }
static C cpowi(C a, int n)
{
    C r = cmk(1, 0);
    for (int i = 0; i < n; ++i) r = cmul(r, a);
    return r;
}

/* P(a, w) / w^a for integer a >= 1 */
static R Pinc_over_wa(int a, R w)
{
    R E = expq(-w);
    if (w < (R)a) {
        /* P(a,w) = e^{-w} sum_{k>=a} w^k/k!  =>  P/w^a = e^{-w} sum_{n>=0} w^n/(a+n)! */
        R term = 1 / fact(a), sum = 0;
        for (int n = 0; n < 2000; ++n) {
            sum += term;
            term *= w / (R)(a + n + 1);
            if (term < sum * 1e-40Q) break;
        }
        return E * sum;
    }
    /* P(a,w) = 1 - e^{-w} sum_{k<a} w^k/k! */
    R s = 0, term = 1;
    for (int k = 0; k < a; ++k) {
        s += term;
        term *= w / (R)(k + 1);
    }
    return (1 - E * s) / ipow(w, a);
}

/* Table of d^p dbar^q F at z for p + q <= n (row-major [p][q], stride n+1). */
static void dF_table(int n, C z, R Lam2, C* out)
{
    C zb = cmk(z.re, -z.im);
    R w = (z.re * z.re + z.im * z.im) / Lam2;
    R E = expq(-w);
    C inv2pii = cmk(0, -1 / (2 * M_PIq)); /* 1/(2 pi i) */
    C* zp = (C*)malloc(sizeof(C) * (size_t)(n + 2));  /* z^r */
    C* bp = (C*)malloc(sizeof(C) * (size_t)(n + 2));  /* (-zbar/Lam2)^r */
    C* ap = (C*)malloc(sizeof(C) * (size_t)(n + 2));  /* (zbar/Lam2)^r */
    zp[0] = bp[0] = ap[0] = cmk(1, 0);
    for (int r = 1; r <= n + 1; ++r) {
        zp[r] = cmul(zp[r - 1], z);
        bp[r] = cmul(bp[r - 1], cscale(zb, -1 / Lam2));
        ap[r] = cmul(ap[r - 1], cscale(zb, 1 / Lam2));
    }
    for (int p = 0; p <= n; ++p)
        for (int q = 0; p + q <= n; ++q) {
            C v;
            if (q == 0) {
                v = cscale(ap[p + 1], sgn(p) * fact(p) * Pinc_over_wa(p + 1, w));
                v = cmul(inv2pii, v);
            } else {
                int r = q - 1;
                C sum = cmk(0, 0);
                for (int t = 0; t <= (p < r ? p : r); ++t) {
                    R coef = binom(p, t) * ipow(-1 / Lam2, r) * fact(r) / fact(r - t);
                    sum = cadd(sum, cscale(cmul(zp[r - t], bp[p - t]), coef));
                }
                v = cscale(cmul(inv2pii, sum), E / Lam2);
            }
            out[p * (n + 1) + q] = v;
        }
    free(zp); free(bp); free(ap);
}

/* D^alpha F from the table: the real operator (d + dbar)^a1 (i(d - dbar))^a2
 * expanded in powers of d and dbar */
static C DalphaF(int a1, int a2, const C* tab, int n)
{
    int na = a1 + a2;
    C tot = cmk(0, 0);
    for (int p = 0; p <= na; ++p) {
        /* coefficient of x^p y^{na-p} in (x+y)^a1 (x-y)^a2 */
        R co = 0;
        for (int a = 0; a <= a1; ++a) {
            int b = p - a;
            if (b < 0 || b > a2) continue;
            co += binom(a1, a) * binom(a2, b) * sgn(a2 - b);
        }
        if (co == 0) continue;
        tot = cadd(tot, cscale(tab[p * (n + 1) + (na - p)], co));
    }
    return cmul(cpowi(cmk(0, 1), a2), tot);
}

static void HB_point(int a1, int a2, R s1, R s2, R Lam2, R* h1, R* h2)
{
    int n = a1 + a2;
    C* tab = (C*)malloc(sizeof(C) * (size_t)(n + 1) * (n + 1));
    dF_table(n, cmk(s1, s2), Lam2, tab);
    C d = DalphaF(a1, a2, tab, n);
    free(tab);
    *h1 = d.re;
    *h2 = -d.im;
}

/* ------------------------------------------------------------------------
 * Gamma^I + Gamma^II for one triple (k, l, m): eq:FinalSingleI/II, and with
 * H replaced by H^B, eq:FinalCrossI/II.  `Ht` holds H_1 (comp 0) and H_2
 * (comp 1) on the triangle |alpha| <= nH, indexed idx(a1, a2).
 * ---------------------------------------------------------------------- */
typedef struct {
    int nH;
    R* h[2];
} Htab;

static R Htab_get(const Htab* t, int c, int a1, int a2) { return t->h[c][idx(a1, a2)]; }

static R gamma_tilde(int k1, int k2, int l1, int l2, int m1, int m2, const R* il2p, const Htab* Ht)
{
    /* il2p[i] = lambda^{-2i} */
    R g = 0;
    /* Gamma^I: sum_{i<=min(l1,k1-1)} sum_{j<=min(l2,k2)} C(l1,i)C(l2,j)(-1)^{l1+l2}
       [2^{i+1}k1!/(lambda^{2(i+1)}(k1-i-1)!)] [2^j k2!/(lambda^{2j}(k2-j)!)]
       H_1(m1+k1-i-1+l1-i, m2+k2-j+l2-j) */
    for (int i = 0; i <= (l1 < k1 - 1 ? l1 : k1 - 1); ++i)
        for (int j = 0; j <= (l2 < k2 ? l2 : k2); ++j) {
            R f = binom(l1, i) * binom(l2, j) * sgn(l1 + l2) * (g_f1[k1][i] * il2p[i + 1]) *
                  (g_f0[k2][j] * il2p[j]);
            g += f * Htab_get(Ht, 0, m1 + k1 - i - 1 + l1 - i, m2 + k2 - j + l2 - j);
        }
    /* Gamma^II: sum_{i<=min(l1,k1)} sum_{j<=min(l2,k2-1)} C(l1,i)C(l2,j)(-1)^{l1+l2}
       [2^i k1!/(lambda^{2i}(k1-i)!)] [2^{j+1}k2!/(lambda^{2(j+1)}(k2-j-1)!)]
       H_2(m1+k1-i+l1-i, m2+k2-j-1+l2-j) */
    for (int i = 0; i <= (l1 < k1 ? l1 : k1); ++i)
        for (int j = 0; j <= (l2 < k2 - 1 ? l2 : k2 - 1); ++j) {
            R f = binom(l1, i) * binom(l2, j) * sgn(l1 + l2) * (g_f0[k1][i] * il2p[i]) *
                  (g_f1[k2][j] * il2p[j + 1]);
            g += f * Htab_get(Ht, 1, m1 + k1 - i + l1 - i, m2 + k2 - j - 1 + l2 - j);
        }
    return g;
}

/* c_k = (-1)^{|k|} lambda^{2|k|} / (2^{|k|} k1! k2!)  (eq:coefficient) */
static R ck(int k1, int k2, R lam)
{
    int n = k1 + k2;
    return sgn(n) * ipow(lam * lam, n) / (ipow(2, n) * fact(k1) * fact(k2));
}

static Htab htab_alloc(int nH)
{
    Htab t;
    t.nH = nH;
    int n = K_of(nH);
    t.h[0] = (R*)calloc((size_t)n, sizeof(R));
    t.h[1] = (R*)calloc((size_t)n, sizeof(R));
    return t;
}
static void htab_free(Htab* t)
{
    free(t->h[0]);
    free(t->h[1]);
}
static void htab_origin(Htab* t, R Lam2)
{
    for (int s = 0; s <= t->nH; ++s)
        for (int a2 = 0; a2 <= s; ++a2) {
            int a1 = s - a2;
            t->h[0][idx(a1, a2)] = H1_origin(a1, a2, Lam2);
            t->h[1][idx(a1, a2)] = H2_origin(a1, a2, Lam2);
        }
}
static void htab_point(Htab* t, R s1, R s2, R Lam2)
{
    int n = t->nH;
    C* tab = (C*)malloc(sizeof(C) * (size_t)(n + 1) * (n + 1));
    dF_table(n, cmk(s1, s2), Lam2, tab);
    for (int s = 0; s <= n; ++s)
        for (int a2 = 0; a2 <= s; ++a2) {
            int a1 = s - a2;
            C d = DalphaF(a1, a2, tab, n);
            t->h[0][idx(a1, a2)] = d.re;
            t->h[1][idx(a1, a2)] = -d.im;
        }
    free(tab);
}

/* ------------------------------------------------------------------------
 * Right-hand side.  State in quad precision.
 * ---------------------------------------------------------------------- */
typedef struct {
    int N, M, K;
    R nu;
    const double* lambda0;
} Prob;

/* parity of H_1/H_2 at the origin: nonzero only for (even, odd) / (odd, even)
 * arguments, which for every (i, j) term of the triple means k1+l1+m1 odd and
 * k2+l2+m2 odd. */
static int origin_parity_ok(int k1, int k2, int l1, int l2, int m1, int m2)
{
    return ((k1 + l1 + m1) & 1) && ((k2 + l2 + m2) & 1);
}

static int nH_of(int M) { return 3 * M + 1; }

/* dM^j_k (A + B + C) and xdot^j for vortex j.  rows: list of k indices to
 * evaluate (or NULL for all).  dmom_row receives K entries (only rows set). */
static void rhs_vortex(const Prob* P, R t, const R* X, const R* Mo, int j,
                       const int* rows, int nrows, R* dmom_row, R* xdot)
{
    int N = P->N, M = P->M, K = P->K;
    int nH = nH_of(M);
    int nrow = rows ? nrows : K;
    R lam0 = (R)P->lambda0[j];
    R lam2 = lam0 * lam0 + 4 * P->nu * t; /* eq:phi00 */
    R lam = sqrtq(lam2);
    const R* Mj = Mo + (size_t)j * K;

    /* decode shell-major indices once */
    int* d1 = (int*)malloc(sizeof(int) * (size_t)K);
    int* d2 = (int*)malloc(sizeof(int) * (size_t)K);
    for (int s = 0; s <= M; ++s)
        for (int k2 = 0; k2 <= s; ++k2) {
            d1[idx(s - k2, k2)] = s - k2;
            d2[idx(s - k2, k2)] = k2;
        }
    R* il2p = (R*)malloc(sizeof(R) * (size_t)(M + 2)); /* lambda^{-2i} */
    il2p[0] = 1;
    for (int i = 1; i <= M + 1; ++i) il2p[i] = il2p[i - 1] / lam2;

    /* ---- A: self interaction, eq:moment_evolutionFinish ---- */
    Htab Hs = htab_alloc(nH);
    htab_origin(&Hs, 2 * lam2);
    for (int r = 0; r < nrow; ++r) {
        int kk = rows ? rows[r] : r;
        int k1 = d1[kk], k2 = d2[kk];
        R acc = 0;
        for (int l = 0; l < K; ++l) {
            if (Mj[l] == 0) continue;
            for (int m = 0; m < K; ++m) {
                if (Mj[m] == 0) continue;
                if (!origin_parity_ok(k1, k2, d1[l], d2[l], d1[m], d2[m])) continue;
                acc += Mj[l] * Mj[m] * gamma_tilde(k1, k2, d1[l], d2[l], d1[m], d2[m], il2p, &Hs);
            }
        }
        dmom_row[kk] = ck(k1, k2, lam) * acc;
    }
    htab_free(&Hs);

    xdot[0] = xdot[1] = 0;
    if (N > 1) {
        /* ---- B and xdot: pair terms, eq:Final_CrossCoef, eq:xjdot_Final ---- */
        R* Bk = (R*)calloc((size_t)K, sizeof(R));
        Htab Hb = htab_alloc(nH);
        for (int jp = 0; jp < N; ++jp) {
            if (jp == j) continue; /* R4 */
            const R* Mp = Mo + (size_t)jp * K;
            R lamp0 = (R)P->lambda0[jp];
            R lamp2 = lamp0 * lamp0 + 4 * P->nu * t;
            R s1 = X[2 * j] - X[2 * jp], s2 = X[2 * j + 1] - X[2 * jp + 1]; /* R3 */
            htab_point(&Hb, s1, s2, lam2 + lamp2);                        /* R6 */
            for (int r = 0; r < nrow; ++r) {
                int kk = rows ? rows[r] : r;
                int k1 = d1[kk], k2 = d2[kk];
                R acc = 0;
                for (int l = 0; l < K; ++l) {
                    if (Mj[l] == 0) continue;
                    for (int m = 0; m < K; ++m) {
                        if (Mp[m] == 0) continue;
                        /* R2: l on the target j, m on the source j' */
                        acc += Mj[l] * Mp[m] * gamma_tilde(k1, k2, d1[l], d2[l], d1[m], d2[m], il2p, &Hb);
                    }
                }
                Bk[kk] += ck(k1, k2, lam) * acc;
            }
            /* xdot: (1/M^j_00) sum_l sum_m M^{j'}_l M^j_m (-1)^{|m|} H^B(l+m) */
            for (int l = 0; l < K; ++l)
                for (int m = 0; m < K; ++m) {
                    R f = Mp[l] * Mj[m] * sgn(d1[m] + d2[m]);
                    xdot[0] += f * Htab_get(&Hb, 0, d1[l] + d1[m], d2[l] + d2[m]);
                    xdot[1] += f * Htab_get(&Hb, 1, d1[l] + d1[m], d2[l] + d2[m]);
                }
        }
        htab_free(&Hb);
        xdot[0] /= Mj[0];
        xdot[1] /= Mj[0];

        /* ---- C: drift term, eq:last_termsimp ---- */
        for (int r = 0; r < nrow; ++r) {
            int kk = rows ? rows[r] : r;
            int k1 = d1[kk], k2 = d2[kk];
            R c = 0;
            if (k1 >= 1) c += xdot[0] * Mj[idx(k1 - 1, k2)];
            if (k2 >= 1) c += xdot[1] * Mj[idx(k1, k2 - 1)];
            dmom_row[kk] += Bk[kk] + c;
        }
        free(Bk);
    }
    free(d1); free(d2); free(il2p);
}

static void rhs_all(const Prob* P, R t, const R* X, const R* Mo, R* dX, R* dM)
{
    int N = P->N, K = P->K;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < N; ++j) rhs_vortex(P, t, X, Mo, j, NULL, 0, dM + (size_t)j * K, dX + 2 * j);
}

static int check_args(int N, int M, double nu, const double* lambda0)
{
    if (N < 1 || M < 0 || M > 60) return -1;
    if (!(nu >= 0)) return -1;
    for (int j = 0; j < N; ++j)
        if (!(lambda0[j] > 0)) return -1;
    return 0;
}

int oracle_rhs(int N, int M, double nu, const double* lambda0, double t, const double* x,
               const double* mom, double* dx, double* dmom)
{
    init_fact();
    if (check_args(N, M, nu, lambda0)) return -1;
    Prob P = {N, M, K_of(M), (R)nu, lambda0};
    int K = P.K;
    R* X = (R*)malloc(sizeof(R) * 2 * N);
    R* Mo = (R*)malloc(sizeof(R) * (size_t)N * K);
    R* dX = (R*)calloc((size_t)2 * N, sizeof(R));
    R* dM = (R*)calloc((size_t)N * K, sizeof(R));
    for (int i = 0; i < 2 * N; ++i) X[i] = x[i];
    for (size_t i = 0; i < (size_t)N * K; ++i) Mo[i] = mom[i];
    rhs_all(&P, (R)t, X, Mo, dX, dM);
    for (int i = 0; i < 2 * N; ++i) dx[i] = (double)dX[i];
    for (size_t i = 0; i < (size_t)N * K; ++i) dmom[i] = (double)dM[i];
    free(X); free(Mo); free(dX); free(dM);
    return 0;
}

int oracle_rhs_rows(int N, int M, double nu, const double* lambda0, double t, const double* x,
                    const double* mom, int nrows, const int* row_j, const int* row_k,
                    double* out_dmom, double* out_dx)
{
    init_fact();
    if (check_args(N, M, nu, lambda0)) return -1;
    Prob P = {N, M, K_of(M), (R)nu, lambda0};
    int K = P.K;
    for (int r = 0; r < nrows; ++r)
        if (row_j[r] < 0 || row_j[r] >= N || row_k[r] < 0 || row_k[r] >= K) return -1;
    R* X = (R*)malloc(sizeof(R) * 2 * N);
    R* Mo = (R*)malloc(sizeof(R) * (size_t)N * K);
    for (int i = 0; i < 2 * N; ++i) X[i] = x[i];
    for (size_t i = 0; i < (size_t)N * K; ++i) Mo[i] = mom[i];
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < nrows; ++r) {
        R* row = (R*)calloc((size_t)K, sizeof(R));
        R xd[2];
        rhs_vortex(&P, (R)t, X, Mo, row_j[r], &row_k[r], 1, row, xd);
        out_dmom[r] = (double)row[row_k[r]];
        out_dx[2 * r] = (double)xd[0];
        out_dx[2 * r + 1] = (double)xd[1];
        free(row);
    }
    free(X); free(Mo);
    return 0;
}

/* classic RK4 (c = 0, 1/2, 1/2, 1; weights 1/6, 1/3, 1/3, 1/6) in t on (x, M) */
int oracle_rk4(int N, int M, double nu, const double* lambda0, double t0, double dt, long nsteps,
               double* x, double* mom)
{
    init_fact();
    if (check_args(N, M, nu, lambda0) || nsteps < 0) return -1;
    Prob P = {N, M, K_of(M), (R)nu, lambda0};
    int K = P.K;
    size_t nx = (size_t)2 * N, nm = (size_t)N * K;
    R* X = (R*)malloc(sizeof(R) * nx);
    R* Mo = (R*)malloc(sizeof(R) * nm);
    R* Xs = (R*)malloc(sizeof(R) * nx);
    R* Ms = (R*)malloc(sizeof(R) * nm);
    R* kx[4];
    R* km[4];
    for (int s = 0; s < 4; ++s) {
        kx[s] = (R*)calloc(nx, sizeof(R));
        km[s] = (R*)calloc(nm, sizeof(R));
    }
    for (size_t i = 0; i < nx; ++i) X[i] = x[i];
    for (size_t i = 0; i < nm; ++i) Mo[i] = mom[i];
    const R cs[4] = {0, 0.5Q, 0.5Q, 1};
    const R w[4] = {1 / 6.0Q, 1 / 3.0Q, 1 / 3.0Q, 1 / 6.0Q};
    R h = (R)dt;
    for (long n = 0; n < nsteps; ++n) {
        R t = (R)t0 + (R)n * h;
        for (int s = 0; s < 4; ++s) {
            if (s == 0) {
                memcpy(Xs, X, sizeof(R) * nx);
                memcpy(Ms, Mo, sizeof(R) * nm);
            } else {
                for (size_t i = 0; i < nx; ++i) Xs[i] = X[i] + cs[s] * h * kx[s - 1][i];
                for (size_t i = 0; i < nm; ++i) Ms[i] = Mo[i] + cs[s] * h * km[s - 1][i];
            }
            rhs_all(&P, t + cs[s] * h, Xs, Ms, kx[s], km[s]);
        }
        for (size_t i = 0; i < nx; ++i)
            X[i] += h * (w[0] * kx[0][i] + w[1] * kx[1][i] + w[2] * kx[2][i] + w[3] * kx[3][i]);
        for (size_t i = 0; i < nm; ++i)
            Mo[i] += h * (w[0] * km[0][i] + w[1] * km[1][i] + w[2] * km[2][i] + w[3] * km[3][i]);
    }
    for (size_t i = 0; i < nx; ++i) x[i] = (double)X[i];
    for (size_t i = 0; i < nm; ++i) mom[i] = (double)Mo[i];
    for (int s = 0; s < 4; ++s) {
        free(kx[s]);
        free(km[s]);
    }
    free(X); free(Mo); free(Xs); free(Ms);
    return 0;
}

/* ---- single-coefficient accessors for the pins ---- */
double oracle_H_origin(int comp, int a1, int a2, double Lam2)
{
    init_fact();
    if (a1 < 0 || a2 < 0) return 0;
    return (double)(comp == 1 ? H1_origin(a1, a2, (R)Lam2) : H2_origin(a1, a2, (R)Lam2));
}

double oracle_HB(int comp, int a1, int a2, double s1, double s2, double Lam2)
{
    init_fact();
    R h1, h2;
    HB_point(a1, a2, (R)s1, (R)s2, (R)Lam2, &h1, &h2);
    return (double)(comp == 1 ? h1 : h2);
}

double oracle_gamma_tilde(int k1, int k2, int l1, int l2, int m1, int m2, double lam)
{
    init_fact();
    if (k1 < 0 || k2 < 0 || l1 < 0 || l2 < 0 || m1 < 0 || m2 < 0) return 0;
    int nH = k1 + k2 + l1 + l2 + m1 + m2 + 1;
    int np = (k1 > k2 ? k1 : k2) + 2;
    R lam2 = (R)lam * (R)lam;
    R* il2p = (R*)malloc(sizeof(R) * (size_t)(np + 1));
    il2p[0] = 1;
    for (int i = 1; i <= np; ++i) il2p[i] = il2p[i - 1] / lam2;
    Htab Hs = htab_alloc(nH);
    htab_origin(&Hs, 2 * lam2);
    R g = gamma_tilde(k1, k2, l1, l2, m1, m2, il2p, &Hs);
    htab_free(&Hs);
    free(il2p);
    return (double)g;
}

double oracle_ck(int k1, int k2, double lam)
{
    init_fact();
    return (double)ck(k1, k2, (R)lam);
}

/* ------------------------------------------------------------------------
 * Vorticity reconstruction from the moments (eq:moment_expansion_def_tw0,
 * with the Hermite functions eq:Hermitedef and eq:phi00):
 *   omega(x) = sum_j sum_{|k| <= M} M^j_k phi_k(x - x^j; lambda_j(t)),
 *   phi_{k1,k2} = D_{x1}^{k1} D_{x2}^{k2} phi00,  phi00 = exp(-|x|^2/lambda^2) / (pi lambda^2).
 * The 1-D derivatives come from the explicit Hermite-polynomial sum
 *   d^a/du^a exp(-u^2/l^2) = exp(-u^2/l^2) a! sum_{i <= a/2} (-1)^{a-i} (2u/l^2)^{a-2i} (1/l^2)^i / (i! (a-2i)!),
 * term by term.
 * ---------------------------------------------------------------------- */
static R gauss_deriv(int a, R u, R l2)
{
    R s = 0;
    for (int i = 0; 2 * i <= a; ++i)
        s += sgn(a - i) * ipow(2 * u / l2, a - 2 * i) * ipow(1 / l2, i) / (fact(i) * fact(a - 2 * i));
    return fact(a) * s * expq(-u * u / l2);
}

static R omega_at(int N, int M, const double* lambda0, double nu, double t, const double* x, const double* mom,
                  R p1, R p2)
{
    const int K = K_of(M);
    R om = 0;
    for (int j = 0; j < N; ++j) {
        const R l2 = (R)lambda0[j] * (R)lambda0[j] + 4 * (R)nu * (R)t;
        const R u1 = p1 - (R)x[2 * j], u2 = p2 - (R)x[2 * j + 1];
        for (int s = 0; s <= M; ++s)
            for (int k2 = 0; k2 <= s; ++k2) {
                const int k1 = s - k2;
                const R phik = gauss_deriv(k1, u1, l2) * gauss_deriv(k2, u2, l2) / (M_PIq * l2);
                om += (R)mom[(size_t)j * K + idx(k1, k2)] * phik;
            }
    }
    return om;
}

int oracle_vorticity(int N, int M, double nu, const double* lambda0, double t, const double* x, const double* mom,
                     int npts, const double* px, const double* py, double* out)
{
    if (N < 1 || M < 0 || M > 60 || nu < 0 || npts < 0) return -1;
    for (int j = 0; j < N; ++j)
        if (!(lambda0[j] > 0)) return -1;
    init_fact();
#pragma omp parallel for schedule(dynamic, 16)
    for (int p = 0; p < npts; ++p) out[p] = (double)omega_at(N, M, lambda0, nu, t, x, mom, (R)px[p], (R)py[p]);
    return 0;
}

/* ------------------------------------------------------------------------
 * Non-axisymmetric enstrophy about the centre c (eq:nonaxi_enstrophy):
 *   E = int (omega(x) - <omega>(|x - c|))^2 dx,  <omega>(r) = (1/2pi) int_0^{2pi} omega dtheta,
 * written out in polar coordinates about c: the azimuthal mean and integral by
 * the trapezoidal rule on ntheta angles, the radial integral int_0^rmax r (.) dr
 * by composite Simpson on nr (even) intervals.
 * ---------------------------------------------------------------------- */
int oracle_enstrophy_nonaxi(int N, int M, double nu, const double* lambda0, double t, const double* x,
                            const double* mom, double cx, double cy, double rmax, int nr, int ntheta, double* out_E)
{
    if (N < 1 || M < 0 || M > 60 || nu < 0 || nr < 2 || (nr & 1) || ntheta < 1 || !(rmax > 0)) return -1;
    for (int j = 0; j < N; ++j)
        if (!(lambda0[j] > 0)) return -1;
    init_fact();
    R* ring = (R*)calloc((size_t)nr + 1, sizeof(R));  /* 2pi-normalised ring integrals of (omega - mean)^2 */
    if (!ring) return -1;
    const R h = (R)rmax / nr;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i <= nr; ++i) {
        const R r = h * i;
        R* w = (R*)malloc(sizeof(R) * (size_t)ntheta);
        R mean = 0;
        for (int l = 0; l < ntheta; ++l) {
            const R th = 2 * M_PIq * l / ntheta;
            w[l] = omega_at(N, M, lambda0, nu, t, x, mom, (R)cx + r * cosq(th), (R)cy + r * sinq(th));
            mean += w[l];
        }
        mean /= ntheta;
        R sq = 0;
        for (int l = 0; l < ntheta; ++l) sq += (w[l] - mean) * (w[l] - mean);
        ring[i] = r * (2 * M_PIq / ntheta) * sq;
        free(w);
    }
    R E = 0;
    for (int i = 0; i <= nr; ++i) E += ring[i] * ((i == 0 || i == nr) ? 1 : ((i & 1) ? 4 : 2));
    E *= h / 3;
    free(ring);
    *out_E = (double)E;
    return 0;
}

/* ------------------------------------------------------------------------
 * Adaptive integration with the Dormand-Prince 5(4) pair (the method of the
 * ode45 runs in "A note on implementation and performance", RelTol = AbsTol
 * = 1e-8 there), on the state y = (x^j, M^j) in physical time, FP64:
 *   stages k_i = f(t + c_i h, y + h sum_j a_ij k_j), i = 1..6, y_new = y + h sum b_i k_i,
 *   k_7 = f(t + h, y_new), error e = h sum_i (b_i - b*_i) k_i (b* the 4th-order weights);
 *   err = RMS_n( e_n / (atol + rtol max(|y_n|, |y_new,n|)) );
 *   accepted when err < 1: h *= min(10, 0.9 err^(-1/5)) (no growth right after a
 *   rejection; 10 when err = 0); rejected: h *= max(0.2, 0.9 err^(-1/5)).
 *   The last step is clipped to end exactly at t1.
 * Tableau of Dormand & Prince (1980).
 * ---------------------------------------------------------------------- */
static const double kDPc[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
static const double kDPa[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
static const double kDPb[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0};
static const double kDPbs[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200, 187.0 / 2100,
                                1.0 / 40};

static int dp_rhs(int N, int M, double nu, const double* lambda0, double t, const double* y, double* f)
{
    return oracle_rhs(N, M, nu, lambda0, t, y, y + 2 * N, f, f + 2 * N);
}

int oracle_dopri5(int N, int M, double nu, const double* lambda0, double t0, double t1, double rtol, double atol,
                  double h0, double* x, double* mom, long* out_accepted, long* out_rejected)
{
    if (N < 1 || M < 0 || M > 60 || !(t1 >= t0) || !(rtol >= 0) || !(atol > 0) || !(h0 > 0)) return -1;
    const int K = K_of(M);
    const size_t n = 2 * (size_t)N + (size_t)N * K;
    double* y = (double*)malloc(sizeof(double) * n);
    double* yn = (double*)malloc(sizeof(double) * n);
    double* ys = (double*)malloc(sizeof(double) * n);
    double* k = (double*)malloc(sizeof(double) * n * 7);
    if (!y || !yn || !ys || !k) return -1;
    memcpy(y, x, sizeof(double) * 2 * N);
    memcpy(y + 2 * N, mom, sizeof(double) * N * K);
    long acc = 0, rej = 0;
    double t = t0, habs = h0;
    int rc = dp_rhs(N, M, nu, lambda0, t, y, k);
    while (rc == 0 && t < t1) {
        int accepted = 0, rejected = 0;
        while (!accepted) {
            double tn = t + habs;
            if (tn > t1) tn = t1;
            const double h = tn - t;
            habs = h;
            for (int s = 1; s < 7 && rc == 0; ++s) {
                for (size_t i = 0; i < n; ++i) {
                    double v = 0;
                    for (int j = 0; j < s; ++j) v += kDPa[s][j] * k[j * n + i];
                    ys[i] = y[i] + h * v;
                }
                if (s == 6) memcpy(yn, ys, sizeof(double) * n);  /* the fifth-order solution */
                rc = dp_rhs(N, M, nu, lambda0, t + kDPc[s] * h, ys, k + s * n);
            }
            if (rc) break;
            double ss = 0;
            for (size_t i = 0; i < n; ++i) {
                double e = 0;
                for (int j = 0; j < 7; ++j) e += (kDPb[j] - kDPbs[j]) * k[j * n + i];
                e *= h;
                const double ay = y[i] < 0 ? -y[i] : y[i], an = yn[i] < 0 ? -yn[i] : yn[i];
                const double sc = atol + (ay > an ? ay : an) * rtol;
                ss += (e / sc) * (e / sc);
            }
            const double err = sqrt(ss / (double)n);
            if (err < 1) {
                double fac = err == 0 ? 10.0 : 0.9 * pow(err, -0.2);
                if (fac > 10.0) fac = 10.0;
                if (rejected && fac > 1.0) fac = 1.0;
                habs *= fac;
                accepted = 1;
                t = tn;
                memcpy(y, yn, sizeof(double) * n);
                memcpy(k, k + 6 * n, sizeof(double) * n);  /* f(t + h, y_new): the next first stage */
                ++acc;
            } else {
                double fac = 0.9 * pow(err, -0.2);
                if (fac < 0.2) fac = 0.2;
                habs *= fac;
                rejected = 1;
                ++rej;
            }
        }
    }
    if (rc == 0) {
        memcpy(x, y, sizeof(double) * 2 * N);
        memcpy(mom, y + 2 * N, sizeof(double) * N * K);
    }
    if (out_accepted) *out_accepted = acc;
    if (out_rejected) *out_rejected = rej;
    free(y);
    free(yn);
    free(ys);
    free(k);
    return rc;
}
