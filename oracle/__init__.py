"""Plain CPU oracle for the multi-moment vortex method (arXiv:1010.2475).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``; the product package never
imports it.  The arithmetic lives in ``oracle.c`` (quad precision, the paper's
appendix formulas term by term); this module only marshals numpy arrays.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=False):
    """Compile oracle.c with gcc (no GPU code involved)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src,
                               "-lquadmath", "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_K.argtypes = [ctypes.c_int]
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_rhs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double,
                                 dp, dp, dp, dp]
        L.oracle_rhs_rows.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double,
                                      dp, dp, ctypes.c_int, ip, ip, dp, dp]
        L.oracle_rk4.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_long, dp, dp]
        for f in (L.oracle_H_origin,):
            f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]
            f.restype = ctypes.c_double
        L.oracle_HB.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double]
        L.oracle_HB.restype = ctypes.c_double
        L.oracle_dopri5.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp,
                                    ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)]
        L.oracle_vorticity.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double, dp, dp,
                                       ctypes.c_int, dp, dp, dp]
        L.oracle_enstrophy_nonaxi.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ctypes.c_double, dp,
                                              dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_int, dp]
        L.oracle_gamma_tilde.argtypes = [ctypes.c_int] * 6 + [ctypes.c_double]
        L.oracle_gamma_tilde.restype = ctypes.c_double
        L.oracle_ck.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.oracle_ck.restype = ctypes.c_double
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def K_of(M):
    return (M + 1) * (M + 2) // 2


def rhs(M, nu, lambda0, t, x, mom):
    """dx/dt [N,2] and dM/dt [N,K] at time t (all vortices, all coefficients)."""
    lambda0 = np.ascontiguousarray(lambda0, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
    N = x.shape[0]
    mom = np.ascontiguousarray(mom, dtype=np.float64).reshape(N, K_of(M))
    dx = np.zeros_like(x)
    dm = np.zeros_like(mom)
    rc = lib().oracle_rhs(N, M, float(nu), _dp(lambda0), float(t), _dp(x), _dp(mom), _dp(dx), _dp(dm))
    if rc != 0:
        raise ValueError("oracle_rhs: invalid arguments")
    return dx, dm


def rhs_rows(M, nu, lambda0, t, x, mom, rows_j, rows_k):
    """dM^j_k/dt for the listed (j, k) rows, and dx^j/dt of each listed row's vortex."""
    lambda0 = np.ascontiguousarray(lambda0, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
    N = x.shape[0]
    mom = np.ascontiguousarray(mom, dtype=np.float64).reshape(N, K_of(M))
    rj = np.ascontiguousarray(rows_j, dtype=np.int32)
    rk = np.ascontiguousarray(rows_k, dtype=np.int32)
    out = np.zeros(len(rj))
    outx = np.zeros((len(rj), 2))
    rc = lib().oracle_rhs_rows(N, M, float(nu), _dp(lambda0), float(t), _dp(x), _dp(mom), len(rj),
                               _ip(rj), _ip(rk), _dp(out), _dp(outx))
    if rc != 0:
        raise ValueError("oracle_rhs_rows: invalid arguments")
    return out, outx


def rk4(M, nu, lambda0, t0, dt, nsteps, x, mom):
    """nsteps classic RK4 steps; returns new (x, mom) arrays."""
    lambda0 = np.ascontiguousarray(lambda0, dtype=np.float64)
    x = np.array(x, dtype=np.float64).reshape(-1, 2)
    N = x.shape[0]
    mom = np.array(mom, dtype=np.float64).reshape(N, K_of(M))
    rc = lib().oracle_rk4(N, M, float(nu), _dp(lambda0), float(t0), float(dt), int(nsteps),
                          _dp(x), _dp(mom))
    if rc != 0:
        raise ValueError("oracle_rk4: invalid arguments")
    return x, mom


def dopri5(M, nu, lambda0, t0, t1, rtol, atol, h0, x, mom):
    """Adaptive Dormand-Prince 5(4) from t0 to t1; returns (x, mom, accepted, rejected)."""
    lambda0 = np.ascontiguousarray(lambda0, dtype=np.float64)
    x = np.array(x, dtype=np.float64).reshape(-1, 2)
    N = x.shape[0]
    mom = np.array(mom, dtype=np.float64).reshape(N, K_of(M))
    acc, rej = ctypes.c_long(0), ctypes.c_long(0)
    rc = lib().oracle_dopri5(N, M, float(nu), _dp(lambda0), float(t0), float(t1), float(rtol), float(atol),
                             float(h0), _dp(x), _dp(mom), ctypes.byref(acc), ctypes.byref(rej))
    if rc != 0:
        raise ValueError("oracle_dopri5: invalid arguments")
    return x, mom, acc.value, rej.value


def vorticity(M, nu, lambda0, t, x, mom, px, py):
    """omega at the points (px, py) from the moments (eq:moment_expansion_def_tw0)."""
    lambda0 = np.ascontiguousarray(lambda0, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
    N = x.shape[0]
    mom = np.ascontiguousarray(mom, dtype=np.float64).reshape(N, K_of(M))
    px = np.ascontiguousarray(px, dtype=np.float64).ravel()
    py = np.ascontiguousarray(py, dtype=np.float64).ravel()
    out = np.zeros(len(px))
    rc = lib().oracle_vorticity(N, M, float(nu), _dp(lambda0), float(t), _dp(x), _dp(mom), len(px), _dp(px),
                                _dp(py), _dp(out))
    if rc != 0:
        raise ValueError("oracle_vorticity: invalid arguments")
    return out


def enstrophy_nonaxi(M, nu, lambda0, t, x, mom, cx, cy, rmax, nr, ntheta):
    """Non-axisymmetric enstrophy about (cx, cy) (eq:nonaxi_enstrophy)."""
    lambda0 = np.ascontiguousarray(lambda0, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
    N = x.shape[0]
    mom = np.ascontiguousarray(mom, dtype=np.float64).reshape(N, K_of(M))
    E = np.zeros(1)
    rc = lib().oracle_enstrophy_nonaxi(N, M, float(nu), _dp(lambda0), float(t), _dp(x), _dp(mom), float(cx),
                                       float(cy), float(rmax), int(nr), int(ntheta), _dp(E))
    if rc != 0:
        raise ValueError("oracle_enstrophy_nonaxi: invalid arguments")
    return float(E[0])


def set_threads(n):
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    lib().oracle_set_threads(int(n))


def max_threads():
    return int(lib().oracle_max_threads())


def H_origin(comp, a1, a2, Lam2):
    return lib().oracle_H_origin(comp, a1, a2, Lam2)


def HB(comp, a1, a2, s1, s2, Lam2):
    return lib().oracle_HB(comp, a1, a2, s1, s2, Lam2)


def gamma_tilde(k, l, m, lam):
    return lib().oracle_gamma_tilde(k[0], k[1], l[0], l[1], m[0], m[1], lam)


def ck(k, lam):
    return lib().oracle_ck(k[0], k[1], lam)
