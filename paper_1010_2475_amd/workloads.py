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
