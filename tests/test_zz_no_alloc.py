"""The entry point that allocates nothing (mmvm_rhs_noalloc) against mmvm_rhs:
same results to the parity bar, on two calls in a row (the second smaller, so
it runs in the scratch array the first left behind), for a multi-vortex and a
single-vortex problem; sizes beyond the array and unprepared orders rejected."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1010_2475_amd import mmvm
    mmvm.lib()
    return torch, mmvm


def _both(env, w, t, prec):
    torch, mm = env
    dev = torch.device("cuda:0")
    X = torch.tensor(w.x, device=dev)
    Mo = torch.tensor(w.mom, device=dev)
    out = []
    for fn in (mm.rhs, mm.rhs_noalloc):
        dX, dM = torch.full_like(X, 7.0), torch.full_like(Mo, 7.0)
        print("%s N=%d M=%d prec=%d" % (fn.__name__, w.N, w.M, prec), flush=True)
        fn(w.M, w.nu, w.lam0, t, X, Mo, dX, dM, prec)
        torch.cuda.synchronize()
        out.append((dX.cpu().numpy(), dM.cpu().numpy()))
    mm.sync()
    return out


def _normwise(M, lam_t, ref, got):
    from paper_1010_2475_amd import workloads as wl
    worst = 0.0
    for j in range(ref.shape[0]):
        n = wl.orthonormal_scale(M, lam_t[j])
        worst = max(worst, np.abs((got[j] - ref[j]) * n).max() / np.abs(ref[j] * n).max())
    return worst


@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 2e-6)])
@pytest.mark.parametrize("sizes", [((300, 4), (37, 4)), ((64, 6), (5, 3)), ((1, 40), (1, 12)), ((1, 30), (1, 9))])
def test_noalloc_matches_rhs_twice(env, prec, tol, sizes):
    torch, mm = env
    from test_gpu_parity import rand_workload
    for i, (N, M) in enumerate(sizes):  # the second call is smaller than the first
        mm.prepare(M)
        w = rand_workload(500 + 10 * i + N + M, N, M, spread=3.0)
        t = 0.3
        (dx_a, dm_a), (dx_b, dm_b) = _both(env, w, t, prec)
        lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t)
        assert np.all(dm_b[:, 0] == 0.0)
        assert _normwise(M, lam_t, dm_a, dm_b) <= tol, (N, M)
        if N > 1:
            assert np.abs(dx_b - dx_a).max() <= tol * max(1.0, np.abs(dx_a).max())
        else:
            assert np.all(dx_b == 0.0)


def test_noalloc_rejects_oversize_and_unprepared(env):
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    mm.prepare(6)
    w = wl.random_multi(N=100000, M=6)
    X = torch.zeros((w.N, 2), dtype=torch.float64, device="cuda:0")
    Mo = torch.zeros((w.N, w.K), dtype=torch.float64, device="cuda:0")
    with pytest.raises(mm.MMVMError) as e:
        mm.rhs_noalloc(w.M, w.nu, w.lam0, 0.0, X, Mo, torch.zeros_like(X), torch.zeros_like(Mo), 1)
    assert e.value.status == -7
    # an order whose tables were never built in this process
    w = wl.single_random(M=37)
    X = torch.zeros((1, 2), dtype=torch.float64, device="cuda:0")
    Mo = torch.tensor(w.mom, device="cuda:0")
    with pytest.raises(mm.MMVMError) as e:
        mm.rhs_noalloc(w.M, w.nu, w.lam0, 0.0, X, Mo, torch.zeros_like(X), torch.zeros_like(Mo), 0)
    assert e.value.status == -6
