"""GPU tests of the adaptive Dormand-Prince 5(4) integrator
(mmvm_integrate_adaptive; the paper's ode45 runs) against the oracle's
integrator with the same tableau, controller, first step and tolerances."""
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


def _gpu(env, w, t0, t1, rtol, atol, h0, prec):
    torch, mm = env
    X = torch.tensor(w.x, device="cuda:0")
    Mo = torch.tensor(w.mom, device="cuda:0")
    print("adaptive N=%d M=%d prec=%d tol=%g" % (w.N, w.M, prec, rtol), flush=True)
    st = mm.integrate_adaptive(w.M, w.nu, w.lam0, t0, t1, rtol, atol, h0, X, Mo, prec)
    return X.cpu().numpy(), Mo.cpu().numpy(), st


@pytest.mark.parametrize("case,prec", [("pair2", 0), ("single12", 0), ("multi4", 1)])
def test_adaptive_matches_oracle(env, orc, case, prec):
    from paper_1010_2475_amd import workloads as wl
    from test_gpu_parity import rand_workload, normwise
    if case == "pair2":
        w = rand_workload(91, 2, 2, spread=0.7)
        t1, tol, h0 = 0.8, 1e-8, 1e-2
    elif case == "single12":
        w = wl.single_random(M=12, Re=200.0, seed=92)
        t1, tol, h0 = 0.3, 1e-8, 1e-2
    else:
        w = rand_workload(93, 3, 4, spread=0.9)
        t1, tol, h0 = 0.4, 1e-6, 1e-2
    x_g, m_g, st = _gpu(env, w, 0.0, t1, tol, tol, h0, prec)
    x_r, m_r, acc, rej = orc.dopri5(w.M, w.nu, w.lam0, 0.0, t1, tol, tol, h0, w.x, w.mom)
    assert (st["accepted"], st["rejected"]) == (acc, rej)
    assert st["rhs_evals"] == 1 + 6 * (acc + rej)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t1)
    bar = 1e-12 if prec == 0 else 1e-6
    assert normwise(w.M, lam_t, m_r, m_g) <= bar
    assert np.abs(x_g - x_r).max() <= bar * max(1.0, np.abs(x_r).max())
    assert np.array_equal(m_g[:, 0], w.mom[:, 0])  # circulation bit for bit


def test_adaptive_tight_tolerance_matches_fine_rk4(env, orc):
    """At tight tolerances the adaptive solution is the ODE's: the fixed-step
    classic RK4 on the GPU with a fine step agrees."""
    torch, mm = env
    from test_gpu_parity import rand_workload, normwise
    w = rand_workload(94, 4, 3, spread=1.0)
    x_a, m_a, st = _gpu(env, w, 0.0, 0.5, 1e-11, 1e-11, 1e-3, 0)
    X = torch.tensor(w.x, device="cuda:0")
    Mo = torch.tensor(w.mom, device="cuda:0")
    mm.step(w.M, w.nu, w.lam0, 0.0, 2.5e-4, 2000, X, Mo, 0)
    mm.sync()
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * 0.5)
    assert normwise(w.M, lam_t, Mo.cpu().numpy(), m_a) <= 1e-9
    assert st["accepted"] > 0


def test_adaptive_rejects_bad_arguments(env):
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    w = wl.single_quadrupole(M=4)
    X = torch.tensor(w.x, device="cuda:0")
    Mo = torch.tensor(w.mom, device="cuda:0")
    for args in ((1.0, 0.5, 1e-8, 1e-8, 1e-3), (0.0, 1.0, 1e-8, 0.0, 1e-3), (0.0, 1.0, 1e-8, 1e-8, -1.0)):
        with pytest.raises(mm.MMVMError) as e:
            mm.integrate_adaptive(w.M, w.nu, w.lam0, *args, X, Mo, 0)
        assert e.value.status == -1
    st = mm.integrate_adaptive(w.M, w.nu, w.lam0, 0.5, 0.5, 1e-8, 1e-8, 1e-3, X, Mo, 0)
    assert st["accepted"] == 0
