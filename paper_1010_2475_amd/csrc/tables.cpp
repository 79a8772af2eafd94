// Host generator of the coefficient tables (see tables.hpp for the formulas).
#include "tables.hpp"

#include <complex>
#include <map>
#include <memory>
#include <mutex>

#include "dd.hpp"

namespace mmvm {

namespace {

// pi to double-double accuracy
const dd kPi = {3.141592653589793116e+00, 1.224646799147353207e-16};

dd dd_from_int(long long v) { return dd_make((double)v, (double)(v - (long long)(double)v)); }

dd dd_fact(int n)
{
    dd r = dd_make(1.0);
    for (int i = 2; i <= n; ++i) r = dd_mul_d(r, (double)i);
    return r;
}

dd dd_binom(int n, int k)
{
    if (k < 0 || k > n) return dd_make(0.0);
    // exact in double-double up to the sizes used (C(120, 60) ~ 1e35 needs care:
    // build it multiplicatively, each step exact to ~1e-32 relative)
    dd r = dd_make(1.0);
    for (int i = 1; i <= k; ++i) r = dd_div(dd_mul_d(r, (double)(n - k + i)), dd_make((double)i));
    return r;
}

dd dd_pow2(int e) { return dd_make(std::ldexp(1.0, e)); }

void build(Tables& T, int M)
{
    T.M = M;
    T.K = (M + 1) * (M + 2) / 2;
    T.P = M == 0 ? 1 : 3 * M;
    T.GM = M == 0 ? 1 : 2 * M;
    T.KG = (T.GM + 1) * (T.GM + 2) / 2;
    T.T0N = (T.P + 1) / 2 + 1;

    // --- Psi0 at the origin, c = 2:  Psi0(2a, 2b) = f_n C(n, a) (2a)! (2b)!,
    //     f_n = -(-1)^n / (4 pi n n! 2^n), n = a + b >= 1
    int nt = (T.T0N + 1) * (T.T0N + 2) / 2;
    T.t0_hi.assign(nt, 0.0);
    T.t0_lo.assign(nt, 0.0);
    dd inv4pi = dd_div(dd_make(1.0), dd_mul_d(kPi, 4.0));
    for (int a = 0; a <= T.T0N; ++a)
        for (int b = 0; a + b <= T.T0N; ++b) {
            int n = a + b;
            if (n == 0) continue;
            dd num = dd_mul(dd_mul(dd_binom(n, a), dd_fact(2 * a)), dd_fact(2 * b));
            dd den = dd_mul(dd_mul_d(dd_fact(n), (double)n), dd_pow2(n));
            dd v = dd_mul(dd_div(num, den), inv4pi);
            if ((n & 1) == 0) v = dd_neg(v);  // -(-1)^n
            T.t0_hi[tri(a, b)] = v.hi;
            T.t0_lo[tri(a, b)] = v.lo;
        }

    // --- factor tables
    int M1 = M + 1;
    size_t nf = (size_t)M1 * M1 * M1;
    T.f0_hi.assign(nf, 0.0); T.f0_lo.assign(nf, 0.0);
    T.f1_hi.assign(nf, 0.0); T.f1_lo.assign(nf, 0.0);
    for (int k = 0; k <= M; ++k)
        for (int l = 0; l <= M; ++l)
            for (int i = 0; i <= M; ++i) {
                size_t o = ((size_t)k * M1 + l) * M1 + i;
                if (i <= l && i <= k) {
                    // C(l,i) 2^i k!/(k-i)!
                    dd v = dd_mul(dd_binom(l, i), dd_pow2(i));
                    for (int f = k - i + 1; f <= k; ++f) v = dd_mul_d(v, (double)f);
                    T.f0_hi[o] = v.hi; T.f0_lo[o] = v.lo;
                }
                if (i <= l && i <= k - 1) {
                    // C(l,i) 2^{i+1} k!/(k-i-1)!
                    dd v = dd_mul(dd_binom(l, i), dd_pow2(i + 1));
                    for (int f = k - i; f <= k; ++f) v = dd_mul_d(v, (double)f);
                    T.f1_hi[o] = v.hi; T.f1_lo[o] = v.lo;
                }
            }

    T.binom.assign((size_t)M1 * M1, 0.0);
    for (int l = 0; l <= M; ++l) {
        T.binom[(size_t)l * M1] = 1.0;
        for (int i = 1; i <= l; ++i)
            T.binom[(size_t)l * M1 + i] = T.binom[(size_t)(l - 1) * M1 + i - 1] + (i <= l - 1 ? T.binom[(size_t)(l - 1) * M1 + i] : 0.0);
    }

    T.fd0.assign((size_t)M1 * M1, 0.0);
    T.fd1.assign((size_t)M1 * M1, 0.0);
    T.fd0_lo.assign((size_t)M1 * M1, 0.0);
    T.fd1_lo.assign((size_t)M1 * M1, 0.0);
    for (int k = 0; k <= M; ++k)
        for (int i = 0; i <= M; ++i) {
            const size_t o = ((size_t)k * M1 + i) * M1 + i;
            T.fd0[(size_t)k * M1 + i] = T.f0_hi[o];
            T.fd1[(size_t)k * M1 + i] = T.f1_hi[o];
            T.fd0_lo[(size_t)k * M1 + i] = T.f0_lo[o];
            T.fd1_lo[(size_t)k * M1 + i] = T.f1_lo[o];
        }

    // --- projection constants at lambda = 1
    T.c1_hi.assign(T.K, 0.0); T.c1_lo.assign(T.K, 0.0);
    for (int s = 0; s <= M; ++s)
        for (int k2 = 0; k2 <= s; ++k2) {
            int k1 = s - k2;
            dd den = dd_mul(dd_mul(dd_pow2(s), dd_fact(k1)), dd_fact(k2));
            dd v = dd_div(dd_make(1.0), den);
            if (s & 1) v = dd_neg(v);
            T.c1_hi[tri(k1, k2)] = v.hi;
            T.c1_lo[tri(k1, k2)] = v.lo;
        }

    // --- pair-kernel edge coefficients.  With x = d, y = dbar (complex
    // derivatives), the real derivative D^a = (x + y)^{a1} (i (x - y))^{a2}.
    // Its pure terms give 2 Re(i^{a2} psi_{n0}); the mixed terms are x y Q(x, y)
    // and x y psi = Laplacian(psi)/4 = exp(-|s|^2)/(4 pi) at c = 1, so with
    // x = (u - i v)/2, y = (u + i v)/2 (u = d/ds1, v = d/ds2) the mixed part is
    // (1/(4 pi)) sum_{c+d=n-2} kappa_{cd} h_c(s1) h_d(s2).
    typedef std::complex<long double> cld;
    int P = T.P;
    T.kap0.assign((size_t)(P + 1) * (P + 1), 0.0);
    T.kap1.assign((size_t)(P + 1) * (P + 1), 0.0);
    T.hol.assign(P + 1, 0.0);
    {
        long double fct = 1.0L;  // (n-1)!
        for (int n = 1; n <= P; ++n) {
            if (n > 1) fct *= (long double)(n - 1);
            long double v = ((n - 1) & 1 ? -1.0L : 1.0L) * fct / (4.0L * 3.14159265358979323846264338327950288L);
            T.hol[n] = (double)v;
        }
    }
    for (int n = 2; n <= P; ++n)
        for (int e = 0; e < 2; ++e) {
            int a1 = e, a2 = n - e;
            // coefficients of x^p y^q in (x + y)^{a1} (i(x - y))^{a2}
            std::vector<cld> A(n + 1, cld(0, 0));  // index p (q = n - p)
            {
                std::vector<cld> poly(1, cld(1, 0));
                for (int r = 0; r < a1; ++r) {
                    std::vector<cld> nx(poly.size() + 1, cld(0, 0));
                    for (size_t p = 0; p < poly.size(); ++p) { nx[p + 1] += poly[p]; nx[p] += poly[p]; }
                    poly.swap(nx);
                }
                for (int r = 0; r < a2; ++r) {
                    std::vector<cld> nx(poly.size() + 1, cld(0, 0));
                    for (size_t p = 0; p < poly.size(); ++p) {
                        nx[p + 1] += cld(0, 1) * poly[p];  // i x
                        nx[p] += cld(0, -1) * poly[p];     // -i y
                    }
                    poly.swap(nx);
                }
                for (int p = 0; p <= n; ++p) A[p] = poly[p];
            }
            // mixed part / (xy):  sum_{p=1}^{n-1} A[p] x^{p-1} y^{n-p-1}, then x, y -> u, v
            std::vector<cld> uv(n - 1, cld(0, 0));  // coefficient of u^c v^{n-2-c}
            for (int p = 1; p <= n - 1; ++p) {
                if (A[p] == cld(0, 0)) continue;
                std::vector<cld> poly(1, A[p]);  // in powers of u (v completes the degree)
                for (int r = 0; r < p - 1; ++r) {  // times (u - i v)/2
                    std::vector<cld> nx(poly.size() + 1, cld(0, 0));
                    for (size_t c = 0; c < poly.size(); ++c) {
                        nx[c + 1] += 0.5L * poly[c];
                        nx[c] += cld(0, -0.5L) * poly[c];
                    }
                    poly.swap(nx);
                }
                for (int r = 0; r < n - p - 1; ++r) {  // times (u + i v)/2
                    std::vector<cld> nx(poly.size() + 1, cld(0, 0));
                    for (size_t c = 0; c < poly.size(); ++c) {
                        nx[c + 1] += 0.5L * poly[c];
                        nx[c] += cld(0, 0.5L) * poly[c];
                    }
                    poly.swap(nx);
                }
                for (int c = 0; c <= n - 2; ++c) uv[c] += poly[c];
            }
            std::vector<double>& kap = e == 0 ? T.kap0 : T.kap1;
            for (int c = 0; c <= n - 2; ++c)
                kap[(size_t)n * (P + 1) + c] =
                    (double)(uv[c].real() / (4.0L * 3.14159265358979323846264338327950288L));
        }
}

std::mutex g_mu;
std::map<int, std::unique_ptr<Tables>> g_cache;

}  // namespace

const Tables& get_tables(int M)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(M);
    if (it != g_cache.end()) return *it->second;
    std::unique_ptr<Tables> t(new Tables());
    build(*t, M);
    const Tables& ref = *t;
    g_cache[M] = std::move(t);
    return ref;
}

}  // namespace mmvm
