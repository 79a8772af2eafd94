/*
 * oracle.h -- plain CPU evaluation of the multi-moment vortex method moment
 * equations (arXiv:1010.2475, appendix "Combinatorial formulae").
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product library.
 *
 * Layout: x[N][2]; mom[N][K] row-major, K = (M+1)(M+2)/2, shell-major
 * (ord k = k1+k2 ascending, then k2 ascending).  All buffers are host memory
 * owned by the caller.  Functions returning int return 0 on success and -1 on
 * invalid arguments (N < 1, M < 0 or M > 60, nu < 0, lambda0 <= 0).
 */
#ifndef MMVM_ORACLE_H
#define MMVM_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

int oracle_K(int M);
/* threads used by the parallel loops (no effect on results) */
void oracle_set_threads(int n);
int oracle_max_threads(void);
/* dM/dt and dx/dt at time t (eq:Final_CrossCoef, eq:xjdot_Final; for N = 1,
 * eq:moment_evolutionFinish).  lambda_j(t)^2 = lambda0_j^2 + 4 nu t. */
int oracle_rhs(int N, int M, double nu, const double* lambda0, double t, const double* x,
               const double* mom, double* dx, double* dmom);
/* the same for a list of (vortex j, coefficient k) rows only: out_dmom[r],
 * out_dx[2r..2r+1] = dx of vortex row_j[r] */
int oracle_rhs_rows(int N, int M, double nu, const double* lambda0, double t, const double* x,
                    const double* mom, int nrows, const int* row_j, const int* row_k,
                    double* out_dmom, double* out_dx);
/* nsteps classic RK4 steps of size dt from t0, in place on x and mom */
int oracle_rk4(int N, int M, double nu, const double* lambda0, double t0, double dt, long nsteps,
               double* x, double* mom);
/* single coefficients for the pins */
double oracle_H_origin(int comp, int a1, int a2, double Lam2);          /* H_1 (comp 1), H_2 (comp 2) */
double oracle_HB(int comp, int a1, int a2, double s1, double s2, double Lam2); /* H^B at s */
double oracle_gamma_tilde(int k1, int k2, int l1, int l2, int m1, int m2, double lam);
double oracle_ck(int k1, int k2, double lam);

/* adaptive Dormand-Prince 5(4) integration from t0 to t1 (error norm RMS of
 * e / (atol + rtol max(|y|, |y_new|)), safety 0.9, step factors in [0.2, 10]),
 * first step h0, in place on x and mom; counts of accepted and rejected steps */
int oracle_dopri5(int N, int M, double nu, const double* lambda0, double t0, double t1, double rtol, double atol,
                  double h0, double* x, double* mom, long* out_accepted, long* out_rejected);
/* vorticity omega(px[p], py[p]) reconstructed from the moments (eq:moment_expansion_def_tw0) */
int oracle_vorticity(int N, int M, double nu, const double* lambda0, double t, const double* x, const double* mom,
                     int npts, const double* px, const double* py, double* out);
/* non-axisymmetric enstrophy about (cx, cy) (eq:nonaxi_enstrophy): trapezoid in angle
 * (ntheta), composite Simpson in radius on [0, rmax] (nr even) */
int oracle_enstrophy_nonaxi(int N, int M, double nu, const double* lambda0, double t, const double* x,
                            const double* mom, double cx, double cy, double rmax, int nr, int ntheta, double* out_E);

#ifdef __cplusplus
}
#endif
#endif
