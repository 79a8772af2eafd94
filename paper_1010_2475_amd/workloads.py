"""Seeded synthetic inputs for the multi-moment vortex method workloads.

This module only draws and lays out initial states; it holds none of the
method's arithmetic, so both the HIP path and the CPU oracle's tests use it.

Layout (shared by every consumer):
  x    [N, 2]  float64, vortex centres
  mom  [N, K]  float64, Hermite moments M^j_k, K = (M+1)(M+2)/2, shell-major
               (ord k = k1 + k2 ascending, then k2 ascending)
  lam0 [N]     float64, initial core scale lambda_{j,0} > 0
Viscosity nu = 1/Re (the paper's Re = M[0,0]/nu with unit circulation).

Workloads (all synthetic; the paper uses no dataset):
  single_quadrupole  Lamb-Oseen vortex with a quadrupole perturbation,
                     M00 = 1, M20 = 4 delta, M02 = -4 delta, lambda0 = 2
                     (section "Shear diffusion", eq:IC_sd); order 10, Re 1000.
  single_random      order 40; on top of Lamb-Oseen (M00 = 1, M10 = M01 = 0)
                     orthonormal coefficients a~_k ~ N(0,1) * 0.05 * 2^{-ord k/2}
                     for 2 <= ord k <= 40, drawn in shell-major order,
                     M_k = a~_k lambda0^{ord k} / sqrt(2^{ord k} k1! k2!).
  random_multi       N vortices, centres U([-5,5]^2), circulations U[-1,1],
                     core scales U[0.2,0.5], drawn per vortex in that order;
                     higher moments 0.
  two_clusters       2 x N/2 vortices at (-2,0) and (2,0), x ~ N(centre, I),
                     circulation 1/(N/2) each, core scales U[0.2,0.5].
  dilute_multi       N vortices uniform over a square of mean spacing 2
                     (most pairs in each other's far field).
  tripole_coarse     the large quadrupole perturbation (lambda0 = 1, delta = 0.25,
                     Re 1000) on a 6 x 6 grid of vortices over [-1,1]^2 of core
                     lambda0, circulations omega_0(x_j) times the node area
                     (eq:blurredIC), orders 0 or 2 (section "Tripole Relaxation").
  tripole_reference  that blurred initial vorticity as one particle of order 24
                     (moments of the 36 Gaussians about the centre).
  request_stream     Poisson arrivals of mixed single / multi-vortex solves.
"""
import math

import numpy as np


def K_of(M):
    return (M + 1) * (M + 2) // 2


def index(k1, k2):
    s = k1 + k2
    return s * (s + 1) // 2 + k2


def multi_indices(M):
    """[(k1, k2)] in storage order."""
    return [(s - k2, k2) for s in range(M + 1) for k2 in range(s + 1)]


def orthonormal_scale(M, lam):
    """n_k = sqrt(2^{ord k} k1! k2!) / lam^{ord k}: M_k * n_k is the coefficient
    of the L2(phi00^{-1})-orthonormal Hermite basis (weighted enstrophy norm)."""
    return np.array([math.sqrt(2.0 ** (a + b) * math.factorial(a) * math.factorial(b)) / lam ** (a + b)
                     for (a, b) in multi_indices(M)])


class Workload:
    def __init__(self, name, M, x, mom, lam0, nu, dt, steps):
        self.name = name
        self.M = int(M)
        self.x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
        self.mom = np.ascontiguousarray(mom, dtype=np.float64).reshape(self.x.shape[0], K_of(M))
        self.lam0 = np.ascontiguousarray(lam0, dtype=np.float64)
        self.nu = float(nu)
        self.dt = float(dt)
        self.steps = int(steps)

    @property
    def N(self):
        return self.x.shape[0]

    @property
    def K(self):
        return K_of(self.M)

    def moment_updates(self, steps=None):
        return self.N * self.K * (self.steps if steps is None else steps)

    def copy(self):
        return Workload(self.name, self.M, self.x.copy(), self.mom.copy(), self.lam0.copy(), self.nu,
                        self.dt, self.steps)


def single_quadrupole(M=10, delta=0.1, Re=1000.0, lam0=2.0, dt=1e-3, steps=1000):
    mom = np.zeros((1, K_of(M)))
    mom[0, 0] = 1.0
    if M >= 2:
        mom[0, index(2, 0)] = 4.0 * delta
        mom[0, index(0, 2)] = -4.0 * delta
    return Workload("single_quadrupole", M, np.zeros((1, 2)), mom, [lam0], 1.0 / Re, dt, steps)


def single_random(M=40, Re=1000.0, seed=2, lam0=2.0, amp=0.05, dt=1e-3, steps=2000):
    rng = np.random.default_rng(seed)
    ids = multi_indices(M)
    at = np.zeros(len(ids))
    at[0] = 1.0
    for i, (a, b) in enumerate(ids):
        if a + b >= 2:
            at[i] = rng.normal() * amp * 2.0 ** (-(a + b) / 2.0)
    mom = at / orthonormal_scale(M, lam0)
    return Workload("single_random", M, np.zeros((1, 2)), mom.reshape(1, -1), [lam0], 1.0 / Re, dt, steps)


def random_multi(N=64, M=6, Re=500.0, seed=3, box=5.0, dt=1e-3, steps=500):
    rng = np.random.default_rng(seed)
    x = np.zeros((N, 2))
    gam = np.zeros(N)
    lam0 = np.zeros(N)
    for j in range(N):
        x[j] = rng.uniform(-box, box, 2)
        gam[j] = rng.uniform(-1.0, 1.0)
        lam0[j] = rng.uniform(0.2, 0.5)
    mom = np.zeros((N, K_of(M)))
    mom[:, 0] = gam
    return Workload("random_multi", M, x, mom, lam0, 1.0 / Re, dt, steps)


def two_clusters(N=4096, M=4, Re=2000.0, seed=4, sep=4.0, sigma=1.0, dt=1e-3, steps=200):
    rng = np.random.default_rng(seed)
    h = N // 2
    x = np.zeros((N, 2))
    x[:h] = rng.normal(0.0, sigma, (h, 2)) + np.array([-sep / 2, 0.0])
    x[h:] = rng.normal(0.0, sigma, (N - h, 2)) + np.array([sep / 2, 0.0])
    lam0 = rng.uniform(0.2, 0.5, N)
    mom = np.zeros((N, K_of(M)))
    mom[:h, 0] = 1.0 / h
    mom[h:, 0] = 1.0 / (N - h)
    return Workload("two_clusters", M, x, mom, lam0, 1.0 / Re, dt, steps)


def dilute_multi(N=4096, M=4, Re=1000.0, seed=6, spacing=2.0, dt=1e-3, steps=100):
    """N vortices spread uniformly over a square whose mean spacing is
    `spacing` (most pairs far apart relative to their cores), circulations
    U[-1,1], core scales U[0.2,0.5], higher moments zero: the dilute field on
    which the pair interaction's far field dominates."""
    rng = np.random.default_rng(seed)
    half = 0.5 * spacing * math.sqrt(N)
    x = rng.uniform(-half, half, (N, 2))
    gam = rng.uniform(-1.0, 1.0, N)
    gam[np.abs(gam) < 1e-3] = 1e-3
    lam0 = rng.uniform(0.2, 0.5, N)
    mom = np.zeros((N, K_of(M)))
    mom[:, 0] = gam
    return Workload("dilute_multi", M, x, mom, lam0, 1.0 / Re, dt, steps)


def tripole_coarse(M=2, delta=0.25, lam0=1.0, Re=1000.0, n=6, dt=1e-3, steps=16000):
    """The large quadrupole perturbation of the Lamb-Oseen vortex on a coarse
    n x n grid of vortex centres over [-1, 1]^2 (section "Tripole Relaxation",
    eq:blurredIC): circulation M^j_00 = omega_0(x_j) * (node area), higher
    moments zero, every element of the one core size lambda0 (the paper's
    multi-vortex equations take one core size for all elements, and it states
    no other for this grid).  omega_0 = phi00 + 4 delta (phi20 - phi02)
    (eq:perturbM2) = phi00 (1 + 16 delta (x1^2 - x2^2) / lambda0^4), with
    phi00 = exp(-|x|^2 / lambda0^2) / (pi lambda0^2) (eq:phi00) and
    phi_k = D^k phi00 (eq:Hermitedef)."""
    g = np.linspace(-1.0, 1.0, n)
    hx = g[1] - g[0]
    X1, X2 = np.meshgrid(g, g, indexing="ij")
    x = np.stack([X1.ravel(), X2.ravel()], axis=1)
    r2 = (x ** 2).sum(1)
    phi00 = np.exp(-r2 / lam0 ** 2) / (math.pi * lam0 ** 2)
    omega0 = phi00 * (1.0 + 16.0 * delta * (x[:, 0] ** 2 - x[:, 1] ** 2) / lam0 ** 4)
    mom = np.zeros((n * n, K_of(M)))
    mom[:, 0] = omega0 * hx * hx
    return Workload("tripole_coarse", M, x, mom, np.full(n * n, lam0), 1.0 / Re, dt, steps)


def tripole_reference(M=24, delta=0.25, lam0=1.0, Re=1000.0, n=6, dt=1e-3, steps=16000):
    """The same blurred initial vorticity (the n x n grid of eq:blurredIC) as
    one particle of order M at the centre (the paper's order-24 reference
    solution of the identical initial conditions).  The elements share the
    particle's core, so each Gaussian's expansion about the centre is its
    Taylor series, phi00(x - a) = sum_k (-a)^k / k! D^k phi00(x), and the
    particle's moments are M_k = sum_j Gamma_j (-a_j1)^{k1} (-a_j2)^{k2} / (k1! k2!)
    (first moments zero by the grid's symmetry)."""
    c = tripole_coarse(M=0, delta=delta, lam0=lam0, Re=Re, n=n, dt=dt, steps=steps)
    mom = np.zeros((1, K_of(M)))
    for (k1, k2) in multi_indices(M):
        mom[0, index(k1, k2)] = np.sum(c.mom[:, 0] * (-c.x[:, 0]) ** k1 * (-c.x[:, 1]) ** k2
                                       / (math.factorial(k1) * math.factorial(k2)))
    return Workload("tripole_reference", M, np.zeros((1, 2)), mom, [lam0], 1.0 / Re, dt, steps)


def request_stream(n=2000, seed=5, mean_gap=5e-3, dt=1e-3):
    """Seeded served-stream requests: list of (t_arrive, Workload).

    50% single-particle (M ~ U{10..40}, delta ~ U[0.01,0.2], Re log-uniform
    [1e2,1e4]); 50% multi-vortex (N log-uniform in [16,1024], M ~ U{2..6},
    initial state as random_multi, Re log-uniform [1e2,1e4]); steps ~
    U{200..2000}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(mean_gap)
        steps = int(rng.integers(200, 2001))
        Re = float(10.0 ** rng.uniform(2.0, 4.0))
        if rng.uniform() < 0.5:
            M = int(rng.integers(10, 41))
            delta = float(rng.uniform(0.01, 0.2))
            w = single_quadrupole(M=M, delta=delta, Re=Re, dt=dt, steps=steps)
        else:
            N = int(round(math.exp(rng.uniform(math.log(16), math.log(1024)))))
            M = int(rng.integers(2, 7))
            w = random_multi(N=N, M=M, Re=Re, seed=int(rng.integers(1 << 31)), dt=dt, steps=steps)
        w.name = "req%d" % i
        out.append((t, w))
    return out
