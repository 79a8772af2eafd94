"""GPU tests of the solve server (mmvm_server_*): results are identical alone
and in the mix, admission respects the HBM budget, errors are reported at
submit or poll."""
import os
import sys
import threading
import time

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1010_2475_amd import mmvm
    mmvm.lib()
    torch.cuda.init()
    return mmvm


def _requests():
    from paper_1010_2475_amd import workloads as wl
    reqs = [wl.single_quadrupole(M=12, delta=0.15, Re=800.0, steps=120),
            wl.random_multi(N=40, M=4, Re=300.0, seed=11, steps=90),
            wl.single_random(M=30, Re=2000.0, steps=60),
            wl.random_multi(N=150, M=3, Re=1000.0, seed=12, steps=50),
            wl.random_multi(N=20, M=6, Re=500.0, seed=13, steps=80),
            wl.single_random(M=9, Re=300.0, seed=5, steps=110)]  # persistent small-order kernel
    return reqs


def _solve_alone(mm, w, prec):
    srv = mm.Server(1 << 30, 4)
    tk = srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, prec)
    srv.drain()
    out = srv.poll(tk, w.N, w.M)
    srv.close()
    assert out is not None
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_same_alone_and_in_the_mix(mm, prec):
    reqs = _requests()
    alone = [_solve_alone(mm, w, prec) for w in reqs]
    srv = mm.Server(1 << 30, 3)  # fewer slots than requests: some queue
    tickets = []
    for i, w in enumerate(reqs):
        tickets.append(srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, prec))
        time.sleep(0.002 * i)  # staggered arrivals while others run
    srv.drain()
    for w, tk, (xa, ma, _) in zip(reqs, tickets, alone):
        x, m, st = srv.poll(tk, w.N, w.M)
        assert np.array_equal(x, xa) and np.array_equal(m, ma)
        assert st["steps"] == w.steps
        assert st["t_arrive"] <= st["t_admit"] <= st["t_start"] <= st["t_done"]
    srv.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_reused_buffers_do_not_change_results(mm, prec):
    """One slot: every request after the first runs in the workspace, device
    buffer and pinned buffer that an earlier request of another shape left in
    the server's pools; results equal solving each alone in a fresh server."""
    reqs = _requests()[::-1] + _requests()
    alone = [_solve_alone(mm, w, prec) for w in reqs]
    srv = mm.Server(1 << 30, 1)
    tickets = [srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, prec) for w in reqs]
    srv.drain()
    for i, (w, tk, (xa, ma, _)) in enumerate(zip(reqs, tickets, alone)):
        x, m, st = srv.poll(tk, w.N, w.M)
        assert np.array_equal(x, xa) and np.array_equal(m, ma), i
    srv.close()


def test_server_matches_direct_stepping(mm):
    import torch
    from paper_1010_2475_amd import workloads as wl
    w = wl.random_multi(N=30, M=4, Re=400.0, seed=21, steps=70)
    x_s, m_s, _ = _solve_alone(mm, w, 0)
    X = torch.tensor(w.x, device="cuda:0")
    Mo = torch.tensor(w.mom, device="cuda:0")
    mm.step(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, X, Mo, 0)
    mm.sync()
    m_d = Mo.cpu().numpy()
    assert np.abs(m_s - m_d).max() <= 1e-13 * np.abs(m_d).max()
    assert np.abs(x_s - X.cpu().numpy()).max() <= 1e-13


def test_admission_by_budget_and_slots(mm):
    from paper_1010_2475_amd import workloads as wl
    reqs = [wl.random_multi(N=64, M=6, Re=500.0, seed=30 + i, steps=40) for i in range(6)]
    # budget for two of them at a time (each: state + workspace, about 0.52 MB)
    srv = mm.Server(1_100_000, 8)
    tks = [srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, 1) for w in reqs]
    srv.drain()
    stats = [srv.poll(tk, w.N, w.M)[2] for tk, w in zip(tks, reqs)]
    # with room for at most two, the later requests were admitted only after earlier ones left
    admits = sorted(s["t_admit"] for s in stats)
    dones = sorted(s["t_done"] for s in stats)
    assert admits[2] >= dones[0]
    srv.close()


def test_over_budget_and_bad_inputs_rejected(mm):
    from paper_1010_2475_amd import workloads as wl
    srv = mm.Server(10_000, 2)
    w = wl.random_multi(N=200, M=6, steps=10)
    with pytest.raises(mm.MMVMError) as e:
        srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, 1)
    assert e.value.status == -7
    srv.close()
    srv = mm.Server(1 << 28, 2)
    w = wl.random_multi(N=5, M=2, steps=10)
    w.mom[2, 0] = 0.0
    with pytest.raises(mm.MMVMError) as e:
        srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, 1)
    assert e.value.status == -4
    w.mom[2, 0] = 1.0
    w.mom[3, 4] = float("inf")
    with pytest.raises(mm.MMVMError) as e:
        srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, 1)
    assert e.value.status == -8
    with pytest.raises(mm.MMVMError) as e:
        srv.poll(12345, 5, 2)
    assert e.value.status == -6
    srv.close()


def test_concurrent_submitters(mm):
    from paper_1010_2475_amd import workloads as wl
    srv = mm.Server(1 << 30, 6)
    reqs = [wl.random_multi(N=16 + 4 * i, M=2 + (i % 3), Re=700.0, seed=50 + i, steps=30) for i in range(12)]
    tickets = [None] * len(reqs)

    def go(i):
        w = reqs[i]
        tickets[i] = srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, 1)

    ths = [threading.Thread(target=go, args=(i,)) for i in range(len(reqs))]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    srv.drain()
    for tk, w in zip(tickets, reqs):
        x, m, st = srv.poll(tk, w.N, w.M)
        assert np.all(np.isfinite(m)) and st["steps"] == w.steps
        assert np.array_equal(m[:, 0], w.mom[:, 0])
    srv.close()


def _normwise(M, lam_t, ref, got):
    from paper_1010_2475_amd import workloads as wl
    worst = 0.0
    for j in range(ref.shape[0]):
        n = wl.orthonormal_scale(M, lam_t[j])
        worst = max(worst, np.abs((got[j] - ref[j]) * n).max() / np.abs(ref[j] * n).max())
    return worst


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-6)])
def test_served_results_match_oracle(mm, orc, prec, tol):
    """Requests served together (a multi-vortex and two single-vortex solves of
    different orders, submitted while the others run) against the oracle's RK4
    of each request alone."""
    from paper_1010_2475_amd import workloads as wl
    from test_gpu_parity import rand_workload
    multi = rand_workload(81, 3, 3)
    multi.dt, multi.steps = 2e-3, 12
    single = wl.single_random(M=9, Re=300.0, seed=82, steps=15)
    single.dt = 2e-3
    big = wl.single_random(M=14, Re=900.0, seed=83, steps=10)
    big.dt = 2e-3
    reqs = [multi, single, big]
    srv = mm.Server(1 << 30, 3)
    tks = []
    for w in reqs:
        print("submit N=%d M=%d prec=%d" % (w.N, w.M, prec), flush=True)
        tks.append(srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, prec))
    srv.drain()
    for w, tk in zip(reqs, tks):
        x, m, st = srv.poll(tk, w.N, w.M)
        x_r, m_r = orc.rk4(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom)
        lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * w.steps * w.dt)
        assert _normwise(w.M, lam_t, m_r, m) <= tol, (w.N, w.M)
        assert np.abs(x - x_r).max() <= tol * max(1.0, np.abs(x_r).max())
        assert np.array_equal(m[:, 0], w.mom[:, 0])
        assert st["steps"] == w.steps
    srv.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_single_vortex_batches_equal_alone(mm, prec):
    """Single-vortex requests of one order are stepped together as one batch
    (one launch of each kernel for the group, each member at its own time and
    with its own viscosity and core); with staggered arrivals and uneven step
    counts the groups change from chunk to chunk.  Every result equals solving
    that request alone, bit for bit: the persistent small-order kernel (order
    9), the matrix-core path (order 14) and, in FP64, the double-double path
    (order 28)."""
    from paper_1010_2475_amd import workloads as wl
    reqs = []
    for i in range(5):
        reqs.append(wl.single_random(M=9, Re=150.0 * (i + 1), seed=40 + i, steps=37 + 19 * i, lam0=1.0 + 0.2 * i))
        reqs.append(wl.single_random(M=14, Re=300.0 * (i + 1), seed=50 + i, steps=28 + 23 * i, lam0=1.5 + 0.1 * i))
    for i in range(3):
        reqs.append(wl.single_random(M=28, Re=500.0 * (i + 1), seed=60 + i, steps=30 + 11 * i, lam0=2.0 - 0.3 * i))
    alone = [_solve_alone(mm, w, prec) for w in reqs]
    srv = mm.Server(1 << 30, 16)
    tks = []
    for i, w in enumerate(reqs):
        print("submit M=%d steps=%d prec=%d" % (w.M, w.steps, prec), flush=True)
        tks.append(srv.submit(w.M, w.nu, w.lam0, 0.0, w.dt, w.steps, w.x, w.mom, prec))
        if i % 3 == 2:
            time.sleep(0.003)
    srv.drain()
    for i, (w, tk, (xa, ma, _)) in enumerate(zip(reqs, tks, alone)):
        x, m, st = srv.poll(tk, w.N, w.M)
        assert np.array_equal(m, ma), (i, w.M, np.abs(m - ma).max())
        assert np.array_equal(x, xa)
        assert st["steps"] == w.steps
    srv.close()
