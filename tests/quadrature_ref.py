"""Brute-force Galerkin projection of the vorticity equation by quadrature.

An independent check of the oracle's combinatorial formulas: the moment ODE is
by definition (eq:Galerkin, eq:mom_multi)

    dM^j_k/dt = -P_k[ u . grad w^j ] + P_k[ xdot^j . grad w^j ],
    P_k[f]     = c_k * int H_k(z; lambda_j) f(z) dz              (eq:coefficient)
    xdot^j     = (1/M^j_00) sum_{j' != j} int u^{j'}(z + s) w^j(z) dz   (eq:xjdot)

with w^j = sum_m M^j_m D^m phi00(.; lambda_j), u = sum_{j'} u^{j'}(z + s_{jj'}),
u^{j'} = sum_l M^{j'}_l D^l V00(.; lambda_{j'}), s_{jj'} = x^j - x^{j'}.  The
integrals are done with the trapezoid rule on a large square (spectrally
accurate for these Gaussian-decaying integrands).  Derivatives of V00 come
from sympy's chain rule on V00 = (-b2, b1) G(|b|^2), G(r) = (1 - e^{-r/L2})/(2 pi r),
with G^{(n)} from the regularised incomplete gamma function (scipy).
Shares nothing with the oracle or the HIP library.
"""
import math
from functools import lru_cache

import numpy as np
import scipy.special as sps
import sympy as sp

_b1, _b2 = sp.symbols("b1 b2", real=True)
_G = sp.Function("G")
_g = sp.symbols("g0:40")


@lru_cache(maxsize=None)
def _vel_deriv_fn(comp, l1, l2):
    r2 = _b1 ** 2 + _b2 ** 2
    base = -_b2 * _G(r2) if comp == 1 else _b1 * _G(r2)
    e = sp.diff(base, _b1, l1, _b2, l2) if (l1 or l2) else base
    reps = {}
    for d in e.atoms(sp.Subs):
        reps[d] = _g[d.expr.derivative_count]
    e = e.xreplace(reps).xreplace({_G(r2): _g[0]})
    nmax = l1 + l2 + 1
    return sp.lambdify((_b1, _b2) + tuple(_g[:nmax + 1]), e, "numpy"), nmax


def _G_derivs(r2, L2, nmax):
    """G^{(n)}(r2) for G(r) = (1 - exp(-r/L2)) / (2 pi r):
    d^n/dy^n (1-e^{-y})/y = (-1)^n n! P(n+1, y)/y^{n+1}."""
    y = r2 / L2
    out = []
    for n in range(nmax + 1):
        val = (-1) ** n * math.factorial(n) * sps.gammainc(n + 1, y) / y ** (n + 1)
        out.append(val / (2 * math.pi) / L2 ** (n + 1))
    return out


def velocity_derivative(comp, l1, l2, b1, b2, L2):
    """D^l of component comp (1 or 2) of V00(b; sqrt(L2)) at points b."""
    fn, nmax = _vel_deriv_fn(comp, l1, l2)
    gd = _G_derivs(b1 * b1 + b2 * b2, L2, nmax)
    return fn(b1, b2, *gd) * np.ones_like(b1)


def hermite_1d(n, z, lam):
    """H_n(z; lambda) = lambda^{-n} H_n^{phys}(z / lambda) (eq:Hermitepoly)."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    return np.polynomial.hermite.hermval(z / lam, c) / lam ** n


def dphi_1d(n, z, lam):
    """d^n/dz^n exp(-z^2/lambda^2)."""
    return (-1) ** n * hermite_1d(n, z, lam) * np.exp(-(z / lam) ** 2)


def galerkin_rhs(M, x, mom, lam, L=6.5, n=161):
    """dx [N,2], dM [N,K] by quadrature; lam = lambda_j at the evaluation time."""
    ids = [(s - k2, k2) for s in range(M + 1) for k2 in range(s + 1)]
    N = x.shape[0]
    K = len(ids)
    dM = np.zeros((N, K))
    dX = np.zeros((N, 2))
    for j in range(N):
        lj = lam[j]
        z1d = np.linspace(-L * lj, L * lj, n)
        h = z1d[1] - z1d[0]
        Z1, Z2 = np.meshgrid(z1d, z1d, indexing="ij")
        W = np.full(Z1.shape, h * h)
        W[0, :] *= 0.5
        W[-1, :] *= 0.5
        W[:, 0] *= 0.5
        W[:, -1] *= 0.5
        pref = 1.0 / (math.pi * lj * lj)
        # vorticity and its gradient
        w = np.zeros_like(Z1)
        gw1 = np.zeros_like(Z1)
        gw2 = np.zeros_like(Z1)
        for i, (m1, m2) in enumerate(ids):
            a = mom[j, i]
            if a == 0:
                continue
            w += a * pref * dphi_1d(m1, Z1, lj) * dphi_1d(m2, Z2, lj)
            gw1 += a * pref * dphi_1d(m1 + 1, Z1, lj) * dphi_1d(m2, Z2, lj)
            gw2 += a * pref * dphi_1d(m1, Z1, lj) * dphi_1d(m2 + 1, Z2, lj)
        # velocities
        u1 = np.zeros_like(Z1)
        u2 = np.zeros_like(Z1)
        xd = np.zeros(2)
        for jp in range(N):
            s = x[j] - x[jp]
            B1 = Z1 + s[0]
            B2 = Z2 + s[1]
            uj1 = np.zeros_like(Z1)
            uj2 = np.zeros_like(Z1)
            for i, (l1, l2) in enumerate(ids):
                a = mom[jp, i]
                if a == 0:
                    continue
                uj1 += a * velocity_derivative(1, l1, l2, B1, B2, lam[jp] ** 2)
                uj2 += a * velocity_derivative(2, l1, l2, B1, B2, lam[jp] ** 2)
            u1 += uj1
            u2 += uj2
            if jp != j:
                xd[0] += np.sum(W * uj1 * w)
                xd[1] += np.sum(W * uj2 * w)
        xd /= mom[j, 0]
        if N == 1:
            xd[:] = 0.0
        f = -(u1 * gw1 + u2 * gw2) + xd[0] * gw1 + xd[1] * gw2
        for i, (k1, k2) in enumerate(ids):
            ck = (-1) ** (k1 + k2) * lj ** (2 * (k1 + k2)) / (2 ** (k1 + k2) * math.factorial(k1) * math.factorial(k2))
            dM[j, i] = ck * np.sum(W * hermite_1d(k1, Z1, lj) * hermite_1d(k2, Z2, lj) * f)
        dX[j] = xd
    return dX, dM


def project(M, fvals, Z1, Z2, W, lam):
    """Moments M_k = P_k[f] of a sampled function (eq:coefficient)."""
    ids = [(s - k2, k2) for s in range(M + 1) for k2 in range(s + 1)]
    out = np.zeros(len(ids))
    for i, (k1, k2) in enumerate(ids):
        ck = (-1) ** (k1 + k2) * lam ** (2 * (k1 + k2)) / (2 ** (k1 + k2) * math.factorial(k1) * math.factorial(k2))
        out[i] = ck * np.sum(W * hermite_1d(k1, Z1, lam) * hermite_1d(k2, Z2, lam) * fvals)
    return out
