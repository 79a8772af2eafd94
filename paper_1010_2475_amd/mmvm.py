"""ctypes binding of libmmvm (include/mmvm.h), same names as the C ABI.

Argument marshalling only: every step of the method runs in the HIP library.
Device arrays are torch tensors on a ROCm device (float64, contiguous); streams
are torch.cuda.Stream objects or raw hipStream_t integers (None = the current
torch stream).  There is no CPU fallback: if libmmvm.so is missing or fails to
load, every call raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmmvm.so")

FP64 = 0
MIXED = 1
TABLE_H = 0
TABLE_FACTORS = 1
MAX_ORDER = 40

OK, PENDING = 0, 1
_STATUS = {0: "MMVM_OK", 1: "MMVM_PENDING", -1: "MMVM_EINVAL", -2: "MMVM_ENOMEM", -3: "MMVM_EORDER",
           -4: "MMVM_EZEROCIRC", -5: "MMVM_EDEVICE", -6: "MMVM_ENOTFOUND", -7: "MMVM_EBUDGET",
           -8: "MMVM_ENONFINITE"}


class MMVMError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s" % (where, _STATUS.get(status, str(status))))


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("order", ctypes.c_int32), ("nu", ctypes.c_double),
                ("lambda0", ctypes.POINTER(ctypes.c_double))]


class Batch(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("order", ctypes.c_int32), ("nu", ctypes.POINTER(ctypes.c_double)),
                ("lambda0", ctypes.POINTER(ctypes.c_double))]


class AdaptiveStats(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int64), ("rejected", ctypes.c_int64), ("rhs_evals", ctypes.c_int64),
                ("h_next", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("steps", ctypes.c_int64)]


_lib = None

SYMBOLS = ["mmvm_coeffs", "mmvm_prepare", "mmvm_rhs", "mmvm_step", "mmvm_step_batch", "mmvm_sync", "mmvm_server_create", "mmvm_submit",
           "mmvm_poll", "mmvm_server_drain", "mmvm_server_destroy", "mmvm_timing_enable", "mmvm_timing_get",
           "mmvm_autotune_enable", "mmvm_autotune_report", "mmvm_rhs_noalloc", "mmvm_vorticity_grid",
           "mmvm_enstrophy_nonaxi", "mmvm_integrate_adaptive", "mmvm_status_string"]


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmmvm.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(Problem)
    L.mmvm_coeffs.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    L.mmvm_prepare.argtypes = [ctypes.c_int32]
    L.mmvm_rhs.argtypes = [pp, ctypes.c_double, vp, vp, vp, vp, ctypes.c_int, vp]
    L.mmvm_rhs_noalloc.argtypes = [pp, ctypes.c_double, vp, vp, vp, vp, ctypes.c_int, vp]
    L.mmvm_integrate_adaptive.argtypes = [pp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, vp, vp, ctypes.c_int, vp, ctypes.POINTER(AdaptiveStats)]
    L.mmvm_vorticity_grid.argtypes = [pp, ctypes.c_double, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int32, ctypes.c_int32, vp, vp]
    L.mmvm_enstrophy_nonaxi.argtypes = [pp, ctypes.c_double, vp, vp, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int32, ctypes.c_int32, vp, vp]
    L.mmvm_step.argtypes = [pp, ctypes.c_double, ctypes.c_double, ctypes.c_int64, vp, vp, ctypes.c_int, vp]
    L.mmvm_step_batch.argtypes = [ctypes.POINTER(Batch), ctypes.c_double, ctypes.c_double, ctypes.c_int64, vp, vp,
                                  ctypes.c_int, vp]
    L.mmvm_sync.argtypes = [vp]
    L.mmvm_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(vp)]
    L.mmvm_submit.argtypes = [vp, pp, ctypes.c_double, ctypes.c_double, ctypes.c_int64, dp, dp, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_uint64)]
    L.mmvm_poll.argtypes = [vp, ctypes.c_uint64, dp, dp, ctypes.POINTER(Stats)]
    L.mmvm_server_drain.argtypes = [vp]
    L.mmvm_server_destroy.argtypes = [vp]
    L.mmvm_timing_enable.argtypes = [ctypes.c_int32]
    L.mmvm_timing_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.mmvm_autotune_enable.argtypes = [ctypes.c_int32]
    L.mmvm_autotune_report.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    L.mmvm_status_string.argtypes = [ctypes.c_int]
    L.mmvm_status_string.restype = ctypes.c_char_p
    for name in SYMBOLS:
        if name != "mmvm_status_string":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc, where):
    if rc != OK:
        raise MMVMError(rc, where)


def K_of(M):
    return (M + 1) * (M + 2) // 2


def _problem(M, nu, lambda0):
    lam = np.ascontiguousarray(np.atleast_1d(lambda0), dtype=np.float64)
    p = Problem(len(lam), int(M), float(nu), lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return p, lam  # keep lam alive while p is used


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float64 device tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return ctypes.c_void_p(t.data_ptr())


def coeffs(order, kind):
    """Host copy of a coefficient table (see mmvm_coeffs)."""
    need = ctypes.c_size_t(0)
    _check(lib().mmvm_coeffs(order, kind, None, 0, ctypes.byref(need)), "mmvm_coeffs")
    out = np.zeros(need.value // 8)
    _check(lib().mmvm_coeffs(order, kind, out.ctypes.data_as(ctypes.c_void_p), need.value, None), "mmvm_coeffs")
    if kind == TABLE_FACTORS:
        return out.reshape(2, order + 1, order + 1, order + 1)
    return out.reshape(2, -1)


def rhs(M, nu, lambda0, t, x, mom, dx, dmom, prec=FP64, stream=None):
    p, lam = _problem(M, nu, lambda0)
    N, K = p.n, K_of(M)
    _check(lib().mmvm_rhs(ctypes.byref(p), float(t), _dev(x, (N, 2), "x"), _dev(mom, (N, K), "mom"),
                          _dev(dx, (N, 2), "dx"), _dev(dmom, (N, K), "dmom"), int(prec), _stream(stream)),
           "mmvm_rhs")


def rhs_noalloc(M, nu, lambda0, t, x, mom, dx, dmom, prec=FP64, stream=None):
    """mmvm_rhs_noalloc: mmvm_rhs on the library's fixed scratch array (no allocation;
    the order's tables must have been prepared)."""
    p, lam = _problem(M, nu, lambda0)
    N, K = p.n, K_of(M)
    _check(lib().mmvm_rhs_noalloc(ctypes.byref(p), float(t), _dev(x, (N, 2), "x"), _dev(mom, (N, K), "mom"),
                                  _dev(dx, (N, 2), "dx"), _dev(dmom, (N, K), "dmom"), int(prec),
                                  _stream(stream)), "mmvm_rhs_noalloc")


def integrate_adaptive(M, nu, lambda0, t0, t1, rtol, atol, h0, x, mom, prec=FP64, stream=None):
    """mmvm_integrate_adaptive: Dormand-Prince 5(4) from t0 to t1 in place on the device state;
    returns the step statistics (accepted, rejected, rhs_evals, h_next)."""
    p, lam = _problem(M, nu, lambda0)
    N, K = p.n, K_of(M)
    st = AdaptiveStats()
    _check(lib().mmvm_integrate_adaptive(ctypes.byref(p), float(t0), float(t1), float(rtol), float(atol), float(h0),
                                         _dev(x, (N, 2), "x"), _dev(mom, (N, K), "mom"), int(prec),
                                         _stream(stream), ctypes.byref(st)), "mmvm_integrate_adaptive")
    return {"accepted": st.accepted, "rejected": st.rejected, "rhs_evals": st.rhs_evals, "h_next": st.h_next}


def vorticity_grid(M, nu, lambda0, t, x, mom, x0, y0, h, nx, ny, omega, stream=None):
    """mmvm_vorticity_grid: omega[iy][ix] at (x0 + ix h, y0 + iy h) into the device tensor omega [ny, nx]."""
    p, lam = _problem(M, nu, lambda0)
    N, K = p.n, K_of(M)
    _check(lib().mmvm_vorticity_grid(ctypes.byref(p), float(t), _dev(x, (N, 2), "x"), _dev(mom, (N, K), "mom"),
                                     float(x0), float(y0), float(h), int(nx), int(ny),
                                     _dev(omega, (ny, nx), "omega"), _stream(stream)), "mmvm_vorticity_grid")


def enstrophy_nonaxi(M, nu, lambda0, t, x, mom, cx, cy, rmax, nr, ntheta, E, stream=None):
    """mmvm_enstrophy_nonaxi: the non-axisymmetric enstrophy about (cx, cy) into the device tensor E [1]."""
    p, lam = _problem(M, nu, lambda0)
    N, K = p.n, K_of(M)
    _check(lib().mmvm_enstrophy_nonaxi(ctypes.byref(p), float(t), _dev(x, (N, 2), "x"), _dev(mom, (N, K), "mom"),
                                       float(cx), float(cy), float(rmax), int(nr), int(ntheta), _dev(E, (1,), "E"),
                                       _stream(stream)), "mmvm_enstrophy_nonaxi")


def prepare(M):
    """Builds the tables of order M on the current device (mmvm_prepare)."""
    _check(lib().mmvm_prepare(int(M)), "mmvm_prepare")


def step(M, nu, lambda0, t0, dt, nsteps, x, mom, prec=FP64, stream=None):
    p, lam = _problem(M, nu, lambda0)
    N, K = p.n, K_of(M)
    _check(lib().mmvm_step(ctypes.byref(p), float(t0), float(dt), int(nsteps), _dev(x, (N, 2), "x"),
                           _dev(mom, (N, K), "mom"), int(prec), _stream(stream)), "mmvm_step")


def step_batch(M, nu, lambda0, t0, dt, nsteps, x, mom, prec=FP64, stream=None):
    """Steps a batch of independent single-vortex solves (mmvm_step_batch)."""
    lam = np.ascontiguousarray(np.atleast_1d(lambda0), dtype=np.float64)
    nuv = np.ascontiguousarray(np.broadcast_to(np.atleast_1d(np.asarray(nu, dtype=np.float64)), lam.shape))
    dp = ctypes.POINTER(ctypes.c_double)
    b = Batch(len(lam), int(M), nuv.ctypes.data_as(dp), lam.ctypes.data_as(dp))
    N, K = len(lam), K_of(M)
    _check(lib().mmvm_step_batch(ctypes.byref(b), float(t0), float(dt), int(nsteps), _dev(x, (N, 2), "x"),
                                 _dev(mom, (N, K), "mom"), int(prec), _stream(stream)), "mmvm_step_batch")


def sync(stream=None):
    _check(lib().mmvm_sync(_stream(stream)), "mmvm_sync")


def timing_enable(on):
    _check(lib().mmvm_timing_enable(1 if on else 0), "mmvm_timing_enable")


def autotune_enable(on):
    _check(lib().mmvm_autotune_enable(1 if on else 0), "mmvm_autotune_enable")


def autotune_report():
    """The tuned launch shapes, one text line per key."""
    need = ctypes.c_size_t(0)
    _check(lib().mmvm_autotune_report(None, ctypes.c_size_t(0), ctypes.byref(need)), "mmvm_autotune_report")
    buf = ctypes.create_string_buffer(need.value)
    _check(lib().mmvm_autotune_report(buf, ctypes.c_size_t(need.value), ctypes.byref(need)), "mmvm_autotune_report")
    return buf.value.decode()


def timing_get(kernel):
    """(total_ms, launches) of one kernel since timing was enabled."""
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    rc = lib().mmvm_timing_get(kernel.encode(), ctypes.byref(ms), ctypes.byref(n))
    if rc not in (OK, -6):
        _check(rc, "mmvm_timing_get")
    return ms.value, n.value


class Server:
    """Continuous-batching solve server (mmvm_server_*)."""

    def __init__(self, hbm_budget_bytes, max_slots):
        h = ctypes.c_void_p()
        _check(lib().mmvm_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)),
               "mmvm_server_create")
        self._h = h

    def submit(self, M, nu, lambda0, t0, dt, nsteps, x0, mom0, prec=MIXED):
        p, lam = _problem(M, nu, lambda0)
        x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(p.n, 2)
        mom0 = np.ascontiguousarray(mom0, dtype=np.float64).reshape(p.n, K_of(M))
        tk = ctypes.c_uint64(0)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().mmvm_submit(self._h, ctypes.byref(p), float(t0), float(dt), int(nsteps),
                                 x0.ctypes.data_as(dp), mom0.ctypes.data_as(dp), int(prec), ctypes.byref(tk)),
               "mmvm_submit")
        return tk.value

    def poll(self, ticket, N, M):
        x = np.zeros((N, 2))
        mom = np.zeros((N, K_of(M)))
        st = Stats()
        dp = ctypes.POINTER(ctypes.c_double)
        rc = lib().mmvm_poll(self._h, ctypes.c_uint64(ticket), x.ctypes.data_as(dp), mom.ctypes.data_as(dp),
                             ctypes.byref(st))
        if rc == PENDING:
            return None
        stats = {"t_arrive": st.t_arrive, "t_admit": st.t_admit, "t_start": st.t_start, "t_done": st.t_done,
                 "steps": st.steps}
        if rc != OK:
            err = MMVMError(rc, "mmvm_poll")
            err.stats = stats  # the request's timeline up to the error
            raise err
        return x, mom, stats

    def drain(self):
        _check(lib().mmvm_server_drain(self._h), "mmvm_server_drain")

    def close(self):
        if self._h:
            _check(lib().mmvm_server_destroy(self._h), "mmvm_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
