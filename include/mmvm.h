/*
 * mmvm.h -- C ABI of the MI355X (gfx950) library for the hot path of the
 * multi-moment vortex method (MMVM) of Uminsky, Wayne & Barbaro,
 * "A multi-moment vortex method for 2D viscous fluids" (arXiv:1010.2475).
 *
 * The method represents the vorticity as N Gaussian vortices, each carrying
 * Hermite moments M^j[k1,k2] up to total order M (eq:moment_expansion_def_tw0),
 * and evolves them by the quadratic moment ODE of the appendix:
 *   dM^j_k/dt = A + B + C              (eq:Final_CrossCoef)
 *     A: self interaction              (eq:FinalSingleI, eq:FinalSingleII, eq:moment_evolutionFinish)
 *     B: vortex-vortex interaction     (eq:FinalCrossI, eq:FinalCrossII)
 *     C: drift of the centre           (eq:last_termsimp)
 *   dx^j/dt                            (eq:xjdot_Final)
 * with core scales lambda_j(t)^2 = lambda_{j,0}^2 + 4 nu t (eq:phi00).
 *
 * Conventions shared by every entry point
 *  - Moments are stored shell-major: total order s = k1+k2 = 0..M, then k2
 *    ascending; index(k1,k2) = s(s+1)/2 + k2; K = (M+1)(M+2)/2 per vortex.
 *    mom is [n][K] row-major float64, x is [n][2] float64 (centres).
 *  - Readings of the paper fixed by this library: the pair term carries the
 *    target's moments on the binomial index l and the source's on the velocity
 *    index m; s_{j,j'} = x^j - x^{j'}; the centre velocity sums j' != j; every
 *    sum is truncated at total order <= M; vortex j uses its own lambda_j and
 *    a pair (j, j') uses Lambda^2 = lambda_j^2 + lambda_{j'}^2 in the kernel H^B.
 *  - Every function returns an mmvm_status and never throws across the ABI.
 *    Asynchronous entry points do not synchronise; an error found on the
 *    device (zero circulation, non-finite state) is latched and returned by
 *    mmvm_sync() or mmvm_poll().
 *  - The caller owns every buffer passed in.  The library owns only its
 *    internal workspaces and tables (device memory, cached per device and
 *    stream and grown on demand) and server slots.
 */
#ifndef MMVM_H
#define MMVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MMVM_OK = 0,
    MMVM_PENDING = 1,     /* mmvm_poll: request not finished yet */
    MMVM_EINVAL = -1,     /* bad pointer, size, nu < 0, lambda0 <= 0, dt or nsteps invalid */
    MMVM_ENOMEM = -2,     /* device or host allocation failed */
    MMVM_EORDER = -3,     /* n < 1, order < 0, order > MMVM_MAX_ORDER, or n > 1 and order > MMVM_MAX_PAIR_ORDER */
    MMVM_EZEROCIRC = -4,  /* a vortex of a multi-vortex problem has M^j_00 == 0 (eq:mass) */
    MMVM_EDEVICE = -5,    /* HIP runtime error */
    MMVM_ENOTFOUND = -6,  /* unknown ticket; tables of the order not prepared (mmvm_rhs_noalloc) */
    MMVM_EBUDGET = -7,    /* footprint exceeds the server budget or the no-alloc scratch array */
    MMVM_ENONFINITE = -8  /* NaN/Inf in the state */
} mmvm_status;

typedef enum {
    MMVM_FP64 = 0,  /* FP64 everywhere; double-double for the self contraction at high order */
    MMVM_MIXED = 1  /* FP32 pair interaction and FP64 self contraction; FP64 state and tables */
} mmvm_precision;

#define MMVM_MAX_ORDER 40
/* Interacting vortices (n > 1) up to this order.  Above it the pair term's
 * high-order derivatives (total order 3M) cancel in the contraction beyond
 * what FP64 holds: measured against the oracle, two vortices at distance ~1
 * core gave 3e-11 at order 20 and 2e-7 at order 30 (FP64 path). */
#define MMVM_MAX_PAIR_ORDER 16

/* One solve: n vortices of maximum total order `order`, viscosity nu = 1/Re,
 * initial core scales lambda0[n] (HOST pointer, all > 0). */
typedef struct {
    int32_t n;
    int32_t order;
    double nu;
    const double* lambda0;
} mmvm_problem;

/* ---------------------------------------------------------------------------
 * Coefficient tables (host).  kind:
 *   MMVM_TABLE_H        H_1 and H_2 of the appendix (derivatives of the two
 *                       velocity components of a Gaussian of squared width 2,
 *                       i.e. lambda = 1, at the origin) for total order
 *                       <= 3*order+1: double[2][T], T = (3*order+2)(3*order+3)/2,
 *                       shell-major like the moments.
 *   MMVM_TABLE_FACTORS  the lambda-free factors of eq:FinalSingleI/II:
 *                       f0[k][l][i] = C(l,i) 2^i k!/(k-i)! and
 *                       f1[k][l][i] = C(l,i) 2^{i+1} k!/(k-i-1)! (zero outside
 *                       their ranges): double[2][order+1][order+1][order+1].
 * With out == NULL only *needed_bytes is set.  MMVM_EINVAL if out_bytes is too
 * small or kind is unknown. */
#define MMVM_TABLE_H 0
#define MMVM_TABLE_FACTORS 1
mmvm_status mmvm_coeffs(int32_t order, int32_t kind, void* out, size_t out_bytes, size_t* needed_bytes);

/* Builds the coefficient tables of one order (the closed forms of H_1/H_2 and
 * the factor tables of eq:FinalSingleI/II, in double-double) on the host and
 * copies them to the current device, where every later call of that order
 * finds them.  Optional: the first call of an order does it by itself, which
 * puts the one-time build into that call (a served request, a timed loop).
 * The device copy is waited for on a stream of the library's own, so work in
 * flight on other streams is not synchronised.  MMVM_EORDER outside 0..40. */
mmvm_status mmvm_prepare(int32_t order);

/* ---------------------------------------------------------------------------
 * One right-hand side at time t (eq:Final_CrossCoef, eq:xjdot_Final):
 * x[n][2], mom[n][K] in, dx[n][2], dmom[n][K] out.  All four are DEVICE
 * pointers owned by the caller; stream is a hipStream_t (NULL = default
 * stream).  Asynchronous; dmom[:,0] is exactly 0 (circulation). */
mmvm_status mmvm_rhs(const mmvm_problem* prob, double t, const double* x, const double* mom,
                     double* dx, double* dmom, mmvm_precision prec, void* stream);

/* nsteps classic RK4 steps (c = 0, 1/2, 1/2, 1; weights 1/6, 1/3, 1/3, 1/6)
 * of size dt from t0, in place on the DEVICE arrays x and mom.  Asynchronous,
 * stream-ordered. */
mmvm_status mmvm_step(const mmvm_problem* prob, double t0, double dt, int64_t nsteps, double* x,
                      double* mom, mmvm_precision prec, void* stream);

/* A batch of independent single-vortex solves of one order (an ensemble, e.g. one
 * initial condition at several Reynolds numbers): member j is the problem of one
 * vortex with core lambda0[j] and viscosity nu[j] (HOST arrays [n]), and the
 * members do not interact.  Stepping a batch gives, for every member, the result
 * of stepping that vortex alone (same arithmetic), with one launch of each kernel
 * for the whole batch.  Section: the single-particle moment equations,
 * eq:moment_evolutionFinish; viscous core growth eq:phi00. */
typedef struct {
    int32_t n;             /* members, >= 1 */
    int32_t order;         /* M, 0..MMVM_MAX_ORDER */
    const double* nu;      /* [n] viscosity of each member, >= 0 */
    const double* lambda0; /* [n] initial core scale of each member, > 0 */
} mmvm_batch;

/* nsteps classic RK4 steps of every member of the batch, in place on the DEVICE
 * arrays x[n][2] (unchanged: a lone vortex does not move) and mom[n][K].
 * Asynchronous, stream-ordered; errors as mmvm_step (MMVM_EORDER, MMVM_EINVAL;
 * device-side checks latched for mmvm_sync). */
mmvm_status mmvm_step_batch(const mmvm_batch* batch, double t0, double dt, int64_t nsteps, double* x,
                            double* mom, mmvm_precision prec, void* stream);

/* Adaptive time stepping from t0 to t1 with the Dormand-Prince 5(4) pair, the
 * integrator of the paper's runs (section "A note on implementation and
 * performance": ode45, RelTol = AbsTol = 1e-8), on the DEVICE state x[n][2],
 * mom[n][K] in place, physical time.  Step-size control: the RMS over the state
 * of e / (atol + rtol max(|y|, |y_new|)), e the embedded fourth-order error
 * estimate, must be < 1; then h *= min(10, 0.9 err^-1/5) (no growth right after
 * a rejection), else the step is redone with h *= max(0.2, 0.9 err^-1/5); the
 * first step is h0 and the last one ends exactly at t1.  The host reads the
 * error norm once per step, so the call returns when the integration is done
 * (it synchronises `stream`).  stats (optional): accepted and rejected steps,
 * right-hand sides evaluated, the step size the controller would take next.
 * MMVM_EINVAL for t1 < t0, rtol < 0, atol <= 0, h0 <= 0 or a step below the
 * resolution of t; MMVM_ENONFINITE if the error norm is not finite. */
typedef struct {
    int64_t accepted, rejected, rhs_evals;
    double h_next;
} mmvm_adaptive_stats;
mmvm_status mmvm_integrate_adaptive(const mmvm_problem* prob, double t0, double t1, double rtol, double atol,
                                    double h0, double* x, double* mom, mmvm_precision prec, void* stream,
                                    mmvm_adaptive_stats* stats);

/* Waits for `stream` and returns (and clears) any error latched by device-side
 * checks of earlier calls on it: MMVM_EZEROCIRC or MMVM_ENONFINITE. */
mmvm_status mmvm_sync(void* stream);

/* ---------------------------------------------------------------------------
 * Serving: a continuous-batching solve server on the current device.
 * The server owns device memory up to hbm_budget_bytes and at most max_slots
 * resident requests.  mmvm_submit copies the HOST initial state (x0[n][2],
 * mom0[n][K], prob->lambda0) and returns at once with a ticket; requests are
 * admitted when a slot and their HBM footprint are free, run together with the
 * other resident requests step by step, and leave at completion.  Thread-safe.
 * The result of a request does not depend on what else is resident.
 * Requests are stepped on 4 HIP streams (the environment variable
 * MMVM_SERVER_STREAMS, 1-16, read at mmvm_server_create, changes that). */
typedef struct mmvm_server mmvm_server;
typedef struct {
    double t_arrive, t_admit, t_start, t_done; /* seconds, server clock */
    int64_t steps;
} mmvm_stats;

mmvm_status mmvm_server_create(size_t hbm_budget_bytes, int32_t max_slots, mmvm_server** out);
mmvm_status mmvm_submit(mmvm_server* srv, const mmvm_problem* prob, double t0, double dt,
                        int64_t nsteps, const double* x0, const double* mom0, mmvm_precision prec,
                        uint64_t* ticket);
/* MMVM_PENDING until done; then copies the final state into caller-owned HOST
 * buffers x_out[n][2], mom_out[n][K] (either may be NULL), fills *stats if
 * non-NULL, frees the slot and forgets the ticket. */
mmvm_status mmvm_poll(mmvm_server* srv, uint64_t ticket, double* x_out, double* mom_out,
                      mmvm_stats* stats);
/* Blocks until every submitted request has finished (results stay pollable). */
mmvm_status mmvm_server_drain(mmvm_server* srv);
mmvm_status mmvm_server_destroy(mmvm_server* srv);

/* ---------------------------------------------------------------------------
 * Kernel timing (profiling aid).  While enabled, every kernel launch of the
 * library is bracketed by HIP events on its stream; mmvm_timing_get waits for
 * them and returns the summed duration and launch count of one kernel
 * ("prep", "self", "pair", "stage2", "emit", "apply", "solo").  Enabling
 * clears the totals.  MMVM_ENOTFOUND if the kernel has not run while enabled.
 * The name "graph" returns, timing on or off, the number of replays of
 * captured stepping graphs since the process started (total_ms = 0): calls
 * of at least 9 steps on the large-order paths replay a captured graph (eight
 * steps on the matrix-core path, four on the double-double path) unless
 * timing is on or the environment variable MMVM_GRAPHS is 0. */
mmvm_status mmvm_timing_enable(int32_t on);
mmvm_status mmvm_timing_get(const char* kernel, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------------------
 * Launch-shape autotuning of the pair kernel (the all-pairs interaction of
 * eq:Final_CrossCoef): how many wavefronts share the sources of one target,
 * how many targets a workgroup holds, FP32 or FP64 arithmetic for the mixed
 * precision, the few-vortex kernel (16 lanes per pair), and whether 64-source
 * chunks lying wholly in a target's far field (beyond the Gaussian cores: the
 * pair field is then the harmonic multipole of the source) go to the cheaper
 * far-field kernel.  From 1024 vortices (orders 0-6) the sources of each call
 * are sorted in space (Hilbert order of the call's initial positions) and
 * every candidate uses the far-field split, which decides per chunk at run
 * time; the environment variable MMVM_PAIR_FAR=0 (or 1) restricts the
 * candidates to shapes without (with) it.  With sorted sources a far chunk
 * whose radius is small against its distance from the target enters through
 * the chunk's 41-term multipole expansion about its centre (truncation below
 * ~3e-14 of that chunk's contribution), and a cell of four consecutive chunks
 * that are all far through one expansion translated from theirs where that
 * converges as well; MMVM_FAR_CELLS=0 keeps the chunk expansions only, and
 * MMVM_FAR_M2P=0 every far pair on the pairwise form.  On by default (the environment
 * variable MMVM_AUTOTUNE=0 starts a process with it off).  The first launch
 * for a new key (order, precision, vortex count rounded up to a power of two)
 * times every candidate shape on the caller's stream with the caller's
 * inputs and synchronises that stream once; the fastest shape is kept for the
 * rest of the process, so a key always runs the same shape (and gives the
 * same bits).  Callers that capture launches into a graph should make one
 * uncaptured call per key first.  With tuning off a fixed default shape runs.
 * mmvm_autotune_report writes one text line per tuned key (shape, its time
 * and the default shape's time, in microseconds) into buf, NUL-terminated;
 * buf == NULL just sets *needed; MMVM_EINVAL if cap is too small. */
mmvm_status mmvm_autotune_enable(int32_t on);
mmvm_status mmvm_autotune_report(char* buf, size_t cap, size_t* needed);

/* ---------------------------------------------------------------------------
 * Diagnostics of the section "Shear diffusion / Results".
 *
 * mmvm_vorticity_grid: the vorticity reconstructed from the moments,
 *   omega(x) = sum_j sum_{|k| <= M} M^j_k phi_k(x - x^j; lambda_j(t))
 * (eq:moment_expansion_def_tw0, Hermite functions eq:Hermitedef of eq:phi00),
 * on the grid x = x0 + ix h, y = y0 + iy h: omega[iy][ix], iy < ny, ix < nx,
 * row-major, a DEVICE array of nx * ny doubles owned by the caller; x, mom are
 * the device state as for mmvm_rhs.  FP64.  Asynchronous on `stream`; the
 * library keeps a workspace per stream (grown on demand).  MMVM_EINVAL for bad
 * sizes or pointers, MMVM_EORDER outside 0..MMVM_MAX_ORDER. */
mmvm_status mmvm_vorticity_grid(const mmvm_problem* prob, double t, const double* x, const double* mom, double x0,
                                double y0, double h, int32_t nx, int32_t ny, double* omega, void* stream);

/* mmvm_enstrophy_nonaxi: the non-axisymmetric enstrophy about the centre
 * (cx, cy) (eq:nonaxi_enstrophy), E = int (omega - <omega>_theta)^2 dx over the
 * disc of radius rmax: the vorticity at ntheta equally spaced angles (exact
 * for the angular modes of a vortex centred at c when ntheta > 2M) on nr rings
 * whose squared radii are the Gauss-Legendre nodes of [0, rmax^2]
 * (int r dr = int d(r^2) / 2).  Writes E to the DEVICE double *E.
 * Asynchronous.  nr <= 4096, ntheta <= 8192. */
mmvm_status mmvm_enstrophy_nonaxi(const mmvm_problem* prob, double t, const double* x, const double* mom, double cx,
                                  double cy, double rmax, int32_t nr, int32_t ntheta, double* E, void* stream);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the right-hand side of
 * mmvm_rhs, same arguments and results (to rounding), with every workspace
 * region taken from one fixed array of MMVM_NOALLOC_SCRATCH_MB MiB that the
 * library holds on each device until the process ends.  It calls no hipMalloc,
 * hipFree or other allocating routine, and no host synchronisation:
 *  - the tables of the order must already be on the device: call
 *    mmvm_prepare(order) first (MMVM_ENOTFOUND otherwise);
 *  - a problem whose workspace exceeds the array returns MMVM_EBUDGET (e.g.
 *    orders <= 6 up to a few tens of thousands of vortices; one vortex at
 *    every order);
 *  - the pair kernel runs the launch shape the autotuner already chose for
 *    this (order, precision, vortex count) in the process, else the default
 *    shape: it never tunes;
 *  - lambda0 (host) is read during the call only;
 *  - device-side checks (zero circulation, non-finite state) are not
 *    reported: such inputs give non-finite outputs;
 *  - every call on a device shares that device's array: calls that overlap on
 *    one device (other streams, other threads) race and must be serialised by
 *    the caller. */
#define MMVM_NOALLOC_SCRATCH_MB 64
mmvm_status mmvm_rhs_noalloc(const mmvm_problem* prob, double t, const double* x, const double* mom,
                             double* dx, double* dmom, mmvm_precision prec, void* stream);

/* Human-readable name of a status code (static string). */
const char* mmvm_status_string(mmvm_status s);

#ifdef __cplusplus
}
#endif
#endif /* MMVM_H */
