// Coefficient tables of the MMVM moment equations, generated once per order M
// on the host and uploaded to every device that uses them.
//
// Formulation (lambda-free, "lambda = 1" units; the kernels scale by powers
// of lambda at use):
//   * the self term uses the stream function psi of a Gaussian vortex:
//     u = (-d2 psi, d1 psi), so the appendix's H_1(a) = -Psi(a + e2) and
//     H_2(a) = Psi(a + e1) with Psi(a) = D^a psi.  At the origin psi is radial,
//     psi(r^2) = (ln r^2 + E1(r^2 / c)) / (4 pi), whose Taylor series gives
//     Psi0(2a, 2b) = f_{a+b} C(a+b, a) (2a)! (2b)!, f_n = -(-1)^n / (4 pi n n! c^n).
//     The table t0 holds Psi0 at c = 2 (the paper's 2 lambda^2 at lambda = 1).
//   * the stage-2 contraction uses the two lambda-free factor tables of
//     eq:FinalSingleI/II, f0[k][l][i] = C(l,i) 2^i k!/(k-i)! and
//     f1[k][l][i] = C(l,i) 2^{i+1} k!/(k-i-1)!.
//   * the pair kernel needs, for every shell n, the coefficients that turn
//     products of 1-D Gaussian derivatives into the two edge derivatives
//     Psi(0, n) and Psi(1, n-1) (see kappa below).
#pragma once
#include <vector>

namespace mmvm {

struct Tables {
    int M = 0;
    int K = 0;   // (M+1)(M+2)/2
    int P = 0;   // highest total derivative order of psi needed: max(3M, 1)
    int GM = 0;  // highest |gamma| of the velocity-derivative table: max(2M, 1)
    int KG = 0;  // (GM+1)(GM+2)/2
    int T0N = 0; // t0 is indexed by (a, b) with a + b <= T0N: tri(a, b)

    // Psi0 at the origin, c = 2, only even-even arguments: t0[tri(a,b)] = Psi0(2a, 2b).
    // Stored as a double-double pair (hi, lo) so that the high-order path can
    // use it at 106-bit accuracy.
    std::vector<double> t0_hi, t0_lo;
    // f0, f1: [M+1][M+1][M+1] (k, l, i), hi/lo pairs
    std::vector<double> f0_hi, f0_lo, f1_hi, f1_lo;
    // binomial coefficients C(l, i), [M+1][M+1] row-major (l, i); exact in FP64 for l <= 56
    std::vector<double> binom;
    // diagonals of the factor tables, [M+1][M+1] (k, i): fd0[k][i] = f0[k][i][i] = 2^i k!/(k-i)!,
    // fd1[k][i] = f1[k][i][i] = 2^{i+1} k!/(k-i-1)!, so that f[k][l][i] = C(l, i) fd[k][i]
    std::vector<double> fd0, fd1, fd0_lo, fd1_lo;
    // c1[k] = (-1)^{|k|} / (2^{|k|} k1! k2!)  (the projection constant at lambda = 1), hi/lo
    std::vector<double> c1_hi, c1_lo;
    // Edge coefficients of the pair kernel for shells n = 2..P:
    //   Psi(0, n)   = 2 Re(i^n     psi_{n0}) + sum_{c=0}^{n-2} kap0[n][c] h_c(s1) h_{n-2-c}(s2)
    //   Psi(1, n-1) = 2 Re(i^{n-1} psi_{n0}) + sum_{c=0}^{n-2} kap1[n][c] h_c(s1) h_{n-2-c}(s2)
    // where psi_{n0} = d^n psi (complex derivative), h_a(x) = d^a/dx^a exp(-x^2),
    // and the 1/(4 pi) of psi is folded in.  Layout: kap[(n*(n-1)/2 - 1) + c]...
    // simplified: kap0 and kap1 are [P+1][P+1] row-major (n, c).
    std::vector<double> kap0, kap1;
    // psi_{n0} prefactor: (-1)^{n-1} (n-1)! / (4 pi), n = 1..P ([P+1])
    std::vector<double> hol;
};

// Builds (and caches, thread-safe) the tables of order M.
const Tables& get_tables(int M);

inline int tri(int a, int b) { int s = a + b; return s * (s + 1) / 2 + b; }

}  // namespace mmvm
