"""Host-only checks of the C ABI: the library loads, exports every function
that include/mmvm.h declares, validates arguments before touching a device,
and its coefficient tables (built by its own generator) agree with the
oracle's closed forms."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mm():
    from paper_1010_2475_amd import mmvm
    if not os.path.exists(mmvm.LIB_PATH):
        from paper_1010_2475_amd import build
        build.build()
    return mmvm


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "mmvm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mmvm_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(mm):
    L = mm.lib()
    names = _declared_functions()
    assert "mmvm_rhs" in names and "mmvm_step" in names and "mmvm_submit" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(mm.SYMBOLS)


def test_autotune_switch_and_report_without_device(mm):
    """The tuner's switch and report are host-only: with nothing tuned the
    report is empty, a NULL buffer only sizes it, a short buffer is rejected."""
    L = mm.lib()
    assert L.mmvm_autotune_enable(0) == 0
    assert L.mmvm_autotune_enable(1) == 0
    need = ctypes.c_size_t(0)
    assert L.mmvm_autotune_report(None, ctypes.c_size_t(0), ctypes.byref(need)) == 0
    assert need.value >= 1
    if need.value == 1:
        assert mm.autotune_report() == ""
    buf = ctypes.create_string_buffer(need.value)
    assert L.mmvm_autotune_report(buf, ctypes.c_size_t(need.value - 1), ctypes.byref(need)) == -1
    assert L.mmvm_autotune_report(buf, ctypes.c_size_t(need.value), ctypes.byref(need)) == 0


def test_graph_replay_count_without_device(mm):
    """The replay counter of captured stepping graphs is readable whatever the
    timing state; nothing has been replayed in a process without a GPU."""
    assert mm.timing_get("graph") == (0.0, 0)


def test_status_strings(mm):
    assert mm.lib().mmvm_status_string(-4) == b"MMVM_EZEROCIRC"


def test_argument_validation_without_device(mm):
    L = mm.lib()
    vp = ctypes.c_void_p
    lam = np.array([1.0, 1.0])
    dp = lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    # order out of range
    p = mm.Problem(1, 41, 0.01, dp)
    assert L.mmvm_rhs(ctypes.byref(p), 0.0, vp(8), vp(8), vp(8), vp(8), 0, None) == -3
    # no vortices
    p = mm.Problem(0, 2, 0.01, dp)
    assert L.mmvm_step(ctypes.byref(p), 0.0, 1e-3, 1, vp(8), vp(8), 0, None) == -3
    # negative viscosity, non-positive core
    p = mm.Problem(1, 2, -1.0, dp)
    assert L.mmvm_rhs(ctypes.byref(p), 0.0, vp(8), vp(8), vp(8), vp(8), 0, None) == -1
    bad = np.array([0.0])
    p = mm.Problem(1, 2, 0.01, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert L.mmvm_rhs(ctypes.byref(p), 0.0, vp(8), vp(8), vp(8), vp(8), 0, None) == -1
    # null device pointers
    p = mm.Problem(1, 2, 0.01, dp)
    assert L.mmvm_rhs(ctypes.byref(p), 0.0, None, vp(8), vp(8), vp(8), 0, None) == -1
    # multi-vortex problems take every order up to the interacting maximum, and no more
    p = mm.Problem(2, 17, 0.01, dp)
    assert L.mmvm_rhs(ctypes.byref(p), 0.0, vp(8), vp(8), vp(8), vp(8), 0, None) == -3
    # batches: null, empty, order out of range, bad member parameters, null state
    nu = np.array([0.01, 0.02])
    nup = nu.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.mmvm_step_batch(None, 0.0, 1e-3, 1, vp(8), vp(8), 0, None) == -1
    b = mm.Batch(0, 5, nup, dp)
    assert L.mmvm_step_batch(ctypes.byref(b), 0.0, 1e-3, 1, vp(8), vp(8), 0, None) == -3
    b = mm.Batch(2, 41, nup, dp)
    assert L.mmvm_step_batch(ctypes.byref(b), 0.0, 1e-3, 1, vp(8), vp(8), 0, None) == -3
    negnu = np.array([0.01, -1.0])
    b = mm.Batch(2, 5, negnu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), dp)
    assert L.mmvm_step_batch(ctypes.byref(b), 0.0, 1e-3, 1, vp(8), vp(8), 0, None) == -1
    b = mm.Batch(1, 5, nup, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert L.mmvm_step_batch(ctypes.byref(b), 0.0, 1e-3, 1, vp(8), vp(8), 0, None) == -1
    b = mm.Batch(2, 5, nup, dp)
    assert L.mmvm_step_batch(ctypes.byref(b), 0.0, 1e-3, 1, None, vp(8), 0, None) == -1
    # unknown table kind, too small buffer
    assert L.mmvm_coeffs(4, 7, None, 0, None) == -1
    buf = np.zeros(4)
    assert L.mmvm_coeffs(4, 0, buf.ctypes.data_as(ctypes.c_void_p), 32, None) == -1


@pytest.mark.parametrize("M", [0, 3, 10, 40])
def test_H_table_matches_paper_closed_form(mm, orc, M):
    """The library derives H_1, H_2 at the origin from the stream function's
    series; the oracle evaluates the appendix's closed forms."""
    H = mm.coeffs(M, mm.TABLE_H)
    nmax = 3 * M + 1
    worst = 0.0
    for s in range(nmax + 1):
        for a2 in range(s + 1):
            a1 = s - a2
            i = (s * (s + 1)) // 2 + a2
            for c in (1, 2):
                ref = orc.H_origin(c, a1, a2, 2.0)
                got = H[c - 1, i]
                if ref == 0.0:
                    assert got == 0.0
                else:
                    worst = max(worst, abs(got - ref) / abs(ref))
    assert worst < 1e-14, worst


@pytest.mark.parametrize("M", [1, 6, 40])
def test_factor_tables(mm, M):
    F = mm.coeffs(M, mm.TABLE_FACTORS)
    rng = np.random.default_rng(M)
    for _ in range(200):
        k, l, i = (int(v) for v in rng.integers(0, M + 1, 3))
        f0 = math.comb(l, i) * 2 ** i * math.factorial(k) // math.factorial(k - i) if (i <= l and i <= k) else 0
        f1 = (math.comb(l, i) * 2 ** (i + 1) * math.factorial(k) // math.factorial(k - i - 1)
              if (i <= l and i <= k - 1) else 0)
        for got, ref in ((F[0, k, l, i], f0), (F[1, k, l, i], f1)):
            assert (got == 0.0 and ref == 0) or abs(got - ref) <= 1e-15 * ref


def test_pair_constants_file_is_generated(tmp_path):
    """The pair kernel's edge-coefficient constants are exactly what their
    generator writes (no hand edits)."""
    import importlib.util
    import shutil
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_1010_2475_amd", "csrc")
    gen = os.path.join(here, "gen_pair_consts.py")
    shutil.copy(gen, tmp_path / "gen_pair_consts.py")
    spec = importlib.util.spec_from_file_location("gen_pair_consts_copy", tmp_path / "gen_pair_consts.py")
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.main()  # writes pair_consts.inc beside the copy
    with open(tmp_path / "pair_consts.inc") as f, open(os.path.join(here, "pair_consts.inc")) as g:
        assert f.read() == g.read()
