"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Error metric (per vortex, orthonormal Hermite coefficients n_k M_k with
n_k = sqrt(2^{|k|} k1! k2!) / lambda_j^{|k|}):  max_k |d(n_k M_k)| / max_k |n_k M_k|,
maximised over vortices; positions: max |dx| / max(1, max |x|).
Bars: FP64 1e-12; mixed (FP32 pair interaction) 1e-6; circulation exact."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-6


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1010_2475_amd import mmvm
    mmvm.lib()
    return torch, mmvm


def _nk(M, lam):
    from paper_1010_2475_amd import workloads as wl
    return wl.orthonormal_scale(M, lam)


def normwise(M, lam_t, ref, got, gam=None, xdot=None):
    """With gam and xdot (per vortex), the scale of a vortex is at least the
    size |Gamma_j| |xdot_j| of the drift and pair terms that cancel in the
    first-moment rates (exactly zero when the first moments vanish, eq:xjdef),
    in orthonormal units; otherwise max_k |n_k ref_k|."""
    worst = 0.0
    for j in range(ref.shape[0]):
        n = _nk(M, lam_t[j])
        den = np.abs(ref[j] * n).max()
        if gam is not None and M >= 1:
            den = max(den, abs(gam[j]) * np.abs(xdot[j]).max() * n[1])
        num = np.abs((got[j] - ref[j]) * n).max()
        worst = max(worst, num / den if den > 0 else num)
    return worst


def gpu_rhs(env, w, t, prec, x=None, mom=None):
    torch, mm = env
    x = w.x if x is None else x
    mom = w.mom if mom is None else mom
    dev = torch.device("cuda:0")
    X = torch.tensor(x, dtype=torch.float64, device=dev).contiguous()
    Mo = torch.tensor(mom, dtype=torch.float64, device=dev).contiguous()
    dX = torch.zeros_like(X)
    dM = torch.zeros_like(Mo)
    print("gpu_rhs N=%d M=%d prec=%d" % (w.N, w.M, prec), flush=True)
    mm.rhs(w.M, w.nu, w.lam0, t, X, Mo, dX, dM, prec)
    mm.sync()
    return dX.cpu().numpy(), dM.cpu().numpy()


def gpu_step(env, w, t0, nsteps, prec):
    torch, mm = env
    dev = torch.device("cuda:0")
    X = torch.tensor(w.x, dtype=torch.float64, device=dev).contiguous()
    Mo = torch.tensor(w.mom, dtype=torch.float64, device=dev).contiguous()
    print("gpu_step N=%d M=%d steps=%d prec=%d" % (w.N, w.M, nsteps, prec), flush=True)
    mm.step(w.M, w.nu, w.lam0, t0, w.dt, nsteps, X, Mo, prec)
    mm.sync()
    return X.cpu().numpy(), Mo.cpu().numpy()


def rand_workload(seed, N, M, amp=0.08, spread=1.5, decay=0.5):
    """Random vortices with physically scaled moments: orthonormal coefficients
    a~_k = Gamma * amp * 2^{-decay |k|} * N(0,1) (decay 1/2: finite weighted
    enstrophy, the regime where the Hermite expansion converges; decay 0: a
    flat spectrum), first moments zero."""
    from paper_1010_2475_amd import workloads as wl
    rng = np.random.default_rng(seed)
    K = wl.K_of(M)
    x = rng.uniform(-spread, spread, (N, 2))
    lam0 = rng.uniform(0.3, 0.7, N)
    gam = rng.uniform(0.4, 1.0, N) * rng.choice([-1, 1], N)
    mom = np.zeros((N, K))
    shells = np.array([a + b for (a, b) in wl.multi_indices(M)])
    for j in range(N):
        at = rng.normal(0.0, 1.0, K) * amp * 2.0 ** (-shells * decay) * gam[j]
        at[0] = gam[j]
        mom[j] = at / wl.orthonormal_scale(M, lam0[j])
    if M >= 1:
        mom[:, 1:3] = 0.0
    return wl.Workload("rand", M, x, mom, lam0, 0.005, 1e-3, 10)


def structure(w, seed, amp=0.05):
    """Adds decaying orthonormal higher moments to a workload that starts as
    plain Gaussians, as its evolution would."""
    from paper_1010_2475_amd import workloads as wl
    rng = np.random.default_rng(seed)
    shells = np.array([a + b for (a, b) in wl.multi_indices(w.M)])
    for j in range(w.N):
        at = rng.normal(0.0, 1.0, w.K) * amp * 2.0 ** (-shells / 2.0) * w.mom[j, 0]
        at[:3] = 0.0
        w.mom[j] += at / wl.orthonormal_scale(w.M, w.lam0[j])


# ---------------------------------------------------------------------------
# right-hand side, small cases covering several tiles, ragged tails and edges
# ---------------------------------------------------------------------------
CASES = [(1, 0), (1, 1), (1, 3), (1, 6), (1, 7), (1, 8), (1, 10), (2, 0), (2, 1), (4, 1), (7, 1), (2, 2), (3, 4),
         (5, 6), (67, 2), (130, 3),
         # multi-vortex orders above the unrolled pair kernel (runtime-order pair kernel):
         # the small fused stage 2 (7-10), the matrix-core stage 2 (11 and up)
         (2, 7), (3, 8), (3, 10), (2, 12), (9, 9)]


@pytest.mark.parametrize("N,M", CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_rhs_matches_oracle(env, orc, N, M, prec):
    w = rand_workload(100 + 7 * N + M, N, M)
    t = 0.37
    if N <= 5 or M <= 2:
        dx_r, dm_r = orc.rhs(M, w.nu, w.lam0, t, w.x, w.mom)
        rows = None
    else:  # sample targets for the larger cases
        js = [0, N // 2, N - 1]
        rj = [j for j in js for _ in range(w.K)]
        rk = [k for _ in js for k in range(w.K)]
        d, dxr = orc.rhs_rows(M, w.nu, w.lam0, t, w.x, w.mom, rj, rk)
        dm_r = d.reshape(len(js), w.K)
        dx_r = dxr.reshape(len(js), w.K, 2)[:, 0, :]
        rows = js
    dx_g, dm_g = gpu_rhs(env, w, t, prec)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t)
    if rows is not None:
        dx_g, dm_g, lam_t = dx_g[rows], dm_g[rows], lam_t[rows]
    tol = FP64_TOL if prec == 0 else MIXED_TOL
    assert np.all(dm_g[:, 0] == 0.0)
    gam = w.mom[:, 0] if rows is None else w.mom[rows, 0]
    assert normwise(M, lam_t, dm_r, dm_g, gam, dx_r) <= tol
    if N > 1:
        assert np.abs(dx_g - dx_r).max() <= tol * max(1.0, np.abs(dx_r).max())
    else:
        assert np.all(dx_g == 0.0)


def test_rhs_zero_order_two_vortices_closed_form(env):
    """Order 0: xdot^j = Gamma_{j'} V00(x^j - x^{j'}; lambda_j^2 + lambda_{j'}^2)."""
    from paper_1010_2475_amd import workloads as wl
    x = np.array([[-0.6, 0.1], [0.5, -0.2]])
    mom = np.array([[0.8], [1.3]])
    w = wl.Workload("pair0", 0, x, mom, [0.3, 0.45], 1e-3, 1e-3, 1)
    dx, dm = gpu_rhs(env, w, 2.0, 0)
    lam2 = w.lam0 ** 2 + 4 * w.nu * 2.0
    for j, jp in ((0, 1), (1, 0)):
        s = x[j] - x[jp]
        r2 = s @ s
        v = mom[jp, 0] * np.array([-s[1], s[0]]) * (1 - math.exp(-r2 / (lam2[0] + lam2[1]))) / (2 * math.pi * r2)
        assert np.abs(dx[j] - v).max() <= 1e-15
    assert np.all(dm == 0.0)


def test_rhs_deterministic(env):
    w = rand_workload(5, 40, 4)
    a = gpu_rhs(env, w, 0.1, 0)
    b = gpu_rhs(env, w, 0.1, 0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_zero_circulation_is_reported(env):
    torch, mm = env
    w = rand_workload(9, 3, 2)
    w.mom[1, 0] = 0.0
    X = torch.tensor(w.x, device="cuda:0")
    Mo = torch.tensor(w.mom, device="cuda:0")
    dX, dM = torch.zeros_like(X), torch.zeros_like(Mo)
    mm.rhs(w.M, w.nu, w.lam0, 0.0, X, Mo, dX, dM, 0)
    with pytest.raises(mm.MMVMError) as e:
        mm.sync()
    assert e.value.status == -4
    mm.sync()  # cleared


def test_nonfinite_is_reported(env):
    torch, mm = env
    w = rand_workload(10, 1, 3)
    w.mom[0, 4] = float("nan")
    X = torch.tensor(w.x, device="cuda:0")
    Mo = torch.tensor(w.mom, device="cuda:0")
    dX, dM = torch.zeros_like(X), torch.zeros_like(Mo)
    mm.rhs(w.M, w.nu, w.lam0, 0.0, X, Mo, dX, dM, 0)
    with pytest.raises(mm.MMVMError) as e:
        mm.sync()
    assert e.value.status == -8


# ---------------------------------------------------------------------------
# RK4 stepping
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N,M,steps", [(1, 6, 20), (3, 3, 10), (4, 2, 25), (2, 8, 5), (2, 12, 3)])
def test_step_matches_oracle(env, orc, N, M, steps):
    w = rand_workload(200 + N, N, M)
    w.dt = 2e-3
    x_r, m_r = orc.rk4(M, w.nu, w.lam0, 0.1, w.dt, steps, w.x, w.mom)
    for prec, tol in ((0, FP64_TOL), (1, MIXED_TOL)):
        x_g, m_g = gpu_step(env, w, 0.1, steps, prec)
        lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * (0.1 + steps * w.dt))
        assert normwise(M, lam_t, m_r, m_g) <= tol
        assert np.abs(x_g - x_r).max() <= tol * max(1.0, np.abs(x_r).max())
        assert np.array_equal(m_g[:, 0], w.mom[:, 0])  # circulation bitwise


def host_rk4_via_rhs(env, w, t0, nsteps, prec):
    """Classic RK4 driven from the host, one mmvm_rhs per stage, combined with
    the same operations in the same order as the device stepper."""
    torch, mm = env
    dev = torch.device("cuda:0")
    X = torch.tensor(w.x, dtype=torch.float64, device=dev).contiguous()
    Y = torch.tensor(w.mom, dtype=torch.float64, device=dev).contiguous()
    c = (0.0, 0.5, 0.5, 1.0)
    wts = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)
    for n in range(nsteps):
        Ys, acc = Y, None
        for s in range(4):
            dX, dM = torch.zeros_like(X), torch.zeros_like(Y)
            mm.rhs(w.M, w.nu, w.lam0, t0 + (n + c[s]) * w.dt, X, Ys.contiguous(), dX, dM, prec)
            if s < 3:
                acc = wts[0] * dM if s == 0 else acc + wts[s] * dM
                Ys = Y + (c[s + 1] * w.dt) * dM
            else:
                Y = Y + w.dt * (acc + wts[3] * dM)
    mm.sync()
    return Y.cpu().numpy()


@pytest.mark.parametrize("M,prec", [(7, 0), (10, 1), (12, 0), (17, 1), (24, 0), (40, 1), (40, 0)])
def test_large_order_step_matches_rhs_driven_rk4(env, M, prec):
    """Single-vortex stepping at large orders (the matrix-core path finishes
    each stage inside the next stage's self kernel; the double-double path
    uses the emit kernel) against RK4 assembled on the host from mmvm_rhs."""
    from paper_1010_2475_amd import workloads as wl
    w = wl.single_random(M=M, Re=500.0)
    w.dt = 2e-3
    _, m_g = gpu_step(env, w, 0.05, 3, prec)
    m_h = host_rk4_via_rhs(env, w, 0.05, 3, prec)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * (0.05 + 3 * w.dt))
    assert normwise(M, lam_t, m_h, m_g) <= 1e-13
    assert m_g[0, 0] == w.mom[0, 0]


@pytest.mark.parametrize("M,prec", [(0, 0), (1, 1), (3, 0), (6, 1), (9, 0), (10, 0), (11, 1)])
def test_persistent_step_matches_rhs_driven_rk4(env, M, prec):
    """Small orders: one workgroup runs every RK4 stage of a single vortex
    without leaving the kernel; it must agree with RK4 assembled on the host
    from one mmvm_rhs per stage."""
    from paper_1010_2475_amd import workloads as wl
    w = wl.single_random(M=M, Re=500.0)
    w.dt = 2e-3
    x_g, m_g = gpu_step(env, w, 0.05, 5, prec)
    m_h = host_rk4_via_rhs(env, w, 0.05, 5, prec)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * (0.05 + 5 * w.dt))
    assert normwise(M, lam_t, m_h, m_g) <= 1e-13
    assert m_g[0, 0] == w.mom[0, 0]
    assert np.all(x_g == w.x)


@pytest.mark.parametrize("M,steps,dt", [(4, 30, 5e-3), (11, 6, 1e-2)])
def test_persistent_step_matches_oracle(env, orc, M, steps, dt):
    """The persistent kernel against the oracle's RK4 over a stretch long
    enough for the core to spread (Re 100)."""
    from paper_1010_2475_amd import workloads as wl
    w = wl.single_random(M=M, Re=100.0, seed=9)
    w.dt = dt
    x_r, m_r = orc.rk4(w.M, w.nu, w.lam0, 0.0, w.dt, steps, w.x, w.mom)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * steps * w.dt)
    x_g, m_g = gpu_step(env, w, 0.0, steps, 0)
    assert normwise(w.M, lam_t, m_r, m_g) <= FP64_TOL
    assert np.all(x_g == w.x)


def test_persistent_batch_of_many_uneven_solves(env, orc):
    """300 independent order-8 solves in one launch (more workgroups than
    compute units), with different viscosities, cores and moments: sampled
    members against the oracle, and every member against stepping it alone."""
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    rng = np.random.default_rng(21)
    nb, M, steps, dt = 300, 8, 6, 3e-3
    members = []
    for b in range(nb):
        w = wl.single_random(M=M, Re=float(10 ** rng.uniform(2, 4)), seed=100 + b, lam0=float(rng.uniform(0.8, 2.5)))
        w.dt = dt
        members.append(w)
    dev = torch.device("cuda:0")
    X = torch.tensor(np.concatenate([w.x for w in members]), device=dev)
    Mo = torch.tensor(np.concatenate([w.mom for w in members]), device=dev)
    print("step_batch nb=%d M=%d" % (nb, M), flush=True)
    mm.step_batch(M, [w.nu for w in members], [w.lam0[0] for w in members], 0.0, dt, steps, X, Mo, 0)
    mm.sync()
    got = Mo.cpu().numpy()
    for i in (0, 1, 137, 255, 256, 299):
        w = members[i]
        _, m_r = orc.rk4(w.M, w.nu, w.lam0, 0.0, dt, steps, w.x, w.mom)
        lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * steps * dt)
        assert normwise(M, lam_t, m_r, got[i:i + 1]) <= FP64_TOL, i
        _, m1 = gpu_step(env, w, 0.0, steps, 0)
        assert np.array_equal(got[i], m1[0]), i


def _step_env(env, w, t0, nsteps, prec, graphs, X=None, Mo=None):
    torch, mm = env
    dev = torch.device("cuda:0")
    X = torch.tensor(w.x, device=dev) if X is None else X
    Mo = torch.tensor(w.mom, device=dev) if Mo is None else Mo
    os.environ["MMVM_GRAPHS"] = "1" if graphs else "0"
    try:
        print("step M=%d steps=%d prec=%d graphs=%d" % (w.M, nsteps, prec, graphs), flush=True)
        mm.step(w.M, w.nu, w.lam0, t0, w.dt, nsteps, X, Mo, prec)
        mm.sync()
    finally:
        os.environ.pop("MMVM_GRAPHS", None)
    return X, Mo


@pytest.mark.parametrize("M,prec,nsteps", [(12, 0, 21), (16, 1, 22), (24, 0, 30), (40, 1, 21), (30, 0, 21),
                                           (40, 0, 12)])
def test_graph_replay_matches_direct_launches(env, M, prec, nsteps):
    """Large-order stepping replays a captured graph (eight steps on the matrix
    cores; four steps of the double-double path, FP64 above order 24) whose
    stage times come from a device clock; it must give the bits of direct
    launches, also when a second call recaptures it for other state buffers,
    with other work between, and when a third call reuses it."""
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    w = wl.single_random(M=M, Re=700.0, seed=M)
    w.dt = 2e-3
    dd = prec == 0 and M > 24
    reps = (nsteps - 1) // 4 if dd else (nsteps - 1) // 8
    r0 = mm.timing_get("graph")[1]
    _, m_d = _step_env(env, w, 0.05, nsteps, prec, False)
    assert mm.timing_get("graph")[1] == r0
    _, m_g = _step_env(env, w, 0.05, nsteps, prec, True)
    assert mm.timing_get("graph")[1] == r0 + reps
    assert np.array_equal(m_g.cpu().numpy(), m_d.cpu().numpy())
    # eager work between replays, then a second call continuing the run
    gpu_rhs(env, w, 0.3, prec)
    t1 = 0.05 + nsteps * w.dt
    X_d, m_d2 = _step_env(env, w, t1, nsteps + 3, prec, False, Mo=m_d.clone())
    X_g, m_g2 = _step_env(env, w, t1, nsteps + 3, prec, True, Mo=m_g.clone())
    assert np.array_equal(m_g2.cpu().numpy(), m_d2.cpu().numpy())
    assert np.array_equal(X_g.cpu().numpy(), w.x)
    # a third call on the same buffers (the graph is reused; the clock restarts)
    t2 = t1 + (nsteps + 3) * w.dt
    _step_env(env, w, t2, nsteps, prec, False, X=X_d, Mo=m_d2)
    _step_env(env, w, t2, nsteps, prec, True, X=X_g, Mo=m_g2)
    assert np.array_equal(m_g2.cpu().numpy(), m_d2.cpu().numpy())


@pytest.mark.parametrize("N,M,prec,nsteps", [(64, 6, 0, 21), (64, 4, 1, 26), (40, 2, 0, 9), (1100, 3, 1, 18)])
def test_graph_replay_interacting_matches_direct_launches(env, N, M, prec, nsteps):
    """Interacting vortices of the small orders replay a captured graph of
    eight steps (pair kernels and the fused stage-2 / RK4 kernel, stage times
    from a device clock): the same bits as direct launches, for a first call,
    a continuing call on the same buffers (the graph is reused) and a call on
    new buffers (recaptured).  N = 1100: sorted sources and the far split."""
    torch, mm = env
    w = structure_multi(N, M, 400 + N + M)
    r0 = mm.timing_get("graph")[1]
    X_d, m_d = _step_env(env, w, 0.02, nsteps, prec, False)
    assert mm.timing_get("graph")[1] == r0
    X_g, m_g = _step_env(env, w, 0.02, nsteps, prec, True)
    assert mm.timing_get("graph")[1] == r0 + (nsteps - 1) // 8
    assert np.array_equal(m_g.cpu().numpy(), m_d.cpu().numpy())
    assert np.array_equal(X_g.cpu().numpy(), X_d.cpu().numpy())
    t1 = 0.02 + nsteps * w.dt
    _step_env(env, w, t1, nsteps + 5, prec, False, X=X_d, Mo=m_d)
    _step_env(env, w, t1, nsteps + 5, prec, True, X=X_g, Mo=m_g)
    assert np.array_equal(m_g.cpu().numpy(), m_d.cpu().numpy())
    assert np.array_equal(X_g.cpu().numpy(), X_d.cpu().numpy())
    X_d2, m_d2 = _step_env(env, w, 0.0, nsteps, prec, False)
    X_g2, m_g2 = _step_env(env, w, 0.0, nsteps, prec, True)
    assert np.array_equal(m_g2.cpu().numpy(), m_d2.cpu().numpy())
    assert np.array_equal(X_g2.cpu().numpy(), X_d2.cpu().numpy())


def structure_multi(N, M, seed):
    """random_multi-like vortices (inside the dilute square for N >= 1024) with
    decaying higher moments."""
    from paper_1010_2475_amd import workloads as wl
    w = wl.dilute_multi(N=N, M=M, seed=seed) if N >= 1024 else wl.random_multi(N=N, M=M, seed=seed)
    structure(w, seed + 1)
    return w


@pytest.mark.parametrize("M,prec", [(20, 1), (32, 0)])
def test_graph_replay_batch_matches_direct_launches(env, M, prec):
    """A batch of three solves (own viscosities and cores) stepped through
    graph replays equals direct launches bit for bit."""
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    members = [wl.single_random(M=M, Re=Re, seed=s, lam0=l0) for Re, s, l0 in ((200.0, 5, 2.0), (2e3, 6, 1.2),
                                                                                 (2e4, 7, 0.9))]
    dev = torch.device("cuda:0")
    out = []
    for graphs in (False, True):
        X = torch.tensor(np.concatenate([w.x for w in members]), device=dev)
        Mo = torch.tensor(np.concatenate([w.mom for w in members]), device=dev)
        os.environ["MMVM_GRAPHS"] = "1" if graphs else "0"
        try:
            print("step_batch graphs=%d" % graphs, flush=True)
            mm.step_batch(M, [w.nu for w in members], [w.lam0[0] for w in members], 0.0, 1e-3, 17, X, Mo, prec)
            mm.sync()
        finally:
            os.environ.pop("MMVM_GRAPHS", None)
        out.append(Mo.cpu().numpy())
        if graphs:
            assert mm.timing_get("graph")[1] > 0
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("prec", [0, 1])
def test_workspace_reuse_across_orders(env, prec):
    """A stream's workspace serves every order from one allocation, laid out
    anew for each order.  Order 33 stepped before and after an order-40 solve
    on the same stream (the allocation grown for 40, then laid out for 33) gives
    the same bits."""
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    dev = torch.device("cuda:0")
    big = wl.single_random(M=40, Re=500.0, seed=3)
    small = wl.single_random(M=33, Re=800.0, seed=4)
    s = torch.cuda.Stream()
    out = []
    with torch.cuda.stream(s):
        for q in range(2):
            if q == 1:
                Xb = torch.tensor(big.x, device=dev)
                Mb = torch.tensor(big.mom, device=dev)
                print("workspace reuse: order 40 prec=%d" % prec, flush=True)
                mm.step(big.M, big.nu, big.lam0, 0.0, 2e-3, 12, Xb, Mb, prec, stream=s)
            X = torch.tensor(small.x, device=dev)
            Mo = torch.tensor(small.mom, device=dev)
            print("workspace reuse: order 33 prec=%d pass %d" % (prec, q), flush=True)
            mm.step(small.M, small.nu, small.lam0, 0.0, 2e-3, 12, X, Mo, prec, stream=s)
            mm.sync(s)
            out.append(Mo.cpu().numpy())
    assert np.all(np.isfinite(out[0]))
    assert np.array_equal(out[0], out[1])


def test_large_order_step_matches_oracle(env, orc):
    """Order 12, two RK4 steps of one vortex against the oracle's RK4."""
    from paper_1010_2475_amd import workloads as wl
    w = wl.single_random(M=12, Re=300.0)
    w.dt = 5e-3
    x_r, m_r = orc.rk4(w.M, w.nu, w.lam0, 0.1, w.dt, 2, w.x, w.mom)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * (0.1 + 2 * w.dt))
    for prec in (0, 1):
        x_g, m_g = gpu_step(env, w, 0.1, 2, prec)
        assert normwise(w.M, lam_t, m_r, m_g) <= FP64_TOL
        assert np.all(x_g == w.x)


@pytest.mark.parametrize("M,prec", [(5, 1), (10, 0), (11, 0), (12, 1), (24, 0), (33, 0), (40, 1)])
def test_batch_matches_individual_solves(env, M, prec):
    """A batch of independent single-vortex solves (different viscosities and
    cores) gives every member exactly the result of stepping it alone."""
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    members = [wl.single_random(M=M, Re=Re, seed=s, lam0=l0) for Re, s, l0 in ((100.0, 2, 2.0), (1e3, 3, 1.5),
                                                                                  (1e4, 4, 1.0))]
    for w in members:
        w.dt = 2e-3
    dev = torch.device("cuda:0")
    X = torch.tensor(np.concatenate([w.x for w in members]), device=dev)
    Mo = torch.tensor(np.concatenate([w.mom for w in members]), device=dev)
    print("step_batch M=%d prec=%d" % (M, prec), flush=True)
    mm.step_batch(M, [w.nu for w in members], [w.lam0[0] for w in members], 0.05, 2e-3, 7, X, Mo, prec)
    mm.sync()
    got = Mo.cpu().numpy()
    for i, w in enumerate(members):
        _, m1 = gpu_step(env, w, 0.05, 7, prec)
        assert np.array_equal(got[i], m1[0]), (i, np.abs(got[i] - m1[0]).max())
    assert np.array_equal(X.cpu().numpy(), np.concatenate([w.x for w in members]))


# ---------------------------------------------------------------------------
# the workloads at full size (sampled outputs the oracle computes one by one)
# ---------------------------------------------------------------------------
def test_single_quadrupole_trajectory(env, orc):
    """Order 10, Re 1000: 40 RK4 steps against the oracle; the full 1000-step
    run conserves circulation and keeps the first moments at zero."""
    from paper_1010_2475_amd import workloads as wl
    w = wl.single_quadrupole()
    x_r, m_r = orc.rk4(w.M, w.nu, w.lam0, 0.0, w.dt, 40, w.x, w.mom)
    x_g, m_g = gpu_step(env, w, 0.0, 40, 0)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * 40 * w.dt)
    assert normwise(w.M, lam_t, m_r, m_g) <= FP64_TOL
    x_g, m_g = gpu_step(env, w, 0.0, w.steps, 0)
    assert m_g[0, 0] == 1.0
    assert np.abs(m_g[0, 1:3]).max() < 1e-16
    assert np.all(x_g == 0.0)


@pytest.mark.parametrize("prec,tol", [(0, FP64_TOL), (1, 1e-9)])
def test_single_random_order40_sampled_rows(env, orc, prec, tol):
    """Order 40 (861 coefficients): sampled rows of dM/dt across all shells."""
    from paper_1010_2475_amd import workloads as wl
    w = wl.single_random(M=40, Re=1000.0)
    t = 0.5
    dx_g, dm_g = gpu_rhs(env, w, t, prec)
    ids = wl.multi_indices(40)
    rows = [wl.index(1, 1), wl.index(3, 2), wl.index(7, 6), wl.index(0, 17), wl.index(12, 13),
            wl.index(20, 20), wl.index(40, 0), wl.index(17, 23)]
    d, _ = orc.rhs_rows(40, w.nu, w.lam0, t, w.x, w.mom, [0] * len(rows), rows)
    lam = math.sqrt(w.lam0[0] ** 2 + 4 * w.nu * t)
    n = _nk(40, lam)
    scale = max(abs(d[i]) * n[r] for i, r in enumerate(rows))  # the oracle's rows set the scale
    err = max(abs(dm_g[0, r] - d[i]) * n[r] for i, r in enumerate(rows)) / scale
    assert err <= tol, err
    assert dm_g[0, 0] == 0.0
    del ids


@pytest.mark.parametrize("M", [11, 16, 24, 25, 33])
@pytest.mark.parametrize("prec", [0, 1])
def test_single_particle_orders_sampled_rows(env, orc, M, prec):
    """Orders between the small fused kernel and order 40: the matrix-core
    contraction (FP64 up to order 24, and the mixed path at every order) and
    the double-double contraction (FP64 above order 24), on rows spread over
    the shells and the edges of the triangle."""
    from paper_1010_2475_amd import workloads as wl
    w = rand_workload(300 + M, 1, M)
    t = 0.21
    dx_g, dm_g = gpu_rhs(env, w, t, prec)
    h = M // 2
    rows = sorted({wl.index(1, 1), wl.index(0, M), wl.index(M, 0), wl.index(h, M - h), wl.index(3, 2),
                   wl.index(M // 3, M // 3), wl.index(1, M - 1), wl.index(M - 2, 0), wl.index(2, h)})
    d, _ = orc.rhs_rows(M, w.nu, w.lam0, t, w.x, w.mom, [0] * len(rows), rows)
    lam = math.sqrt(w.lam0[0] ** 2 + 4 * w.nu * t)
    n = _nk(M, lam)
    scale = max(abs(d[i]) * n[r] for i, r in enumerate(rows))  # the oracle's rows set the scale
    err = max(abs(dm_g[0, r] - d[i]) * n[r] for i, r in enumerate(rows)) / scale
    tol = FP64_TOL if (M <= 24 or prec == 0) else 1e-9
    assert err <= tol, err
    assert dm_g[0, 0] == 0.0 and np.all(dx_g == 0.0)


@pytest.mark.parametrize("prec,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_autotuned_pair_shape_matches_oracle(env, orc, prec, tol):
    """The pair kernel under the shape the autotuner picks (sources of a
    target split over several wavefronts) and under the fixed default shape:
    both against the oracle on sampled rows, equal to each other to rounding,
    and the tuned shape repeats its bits."""
    torch, mm = env
    w = rand_workload(61, 300, 4, spread=4.0)
    t = 0.1
    mm.autotune_enable(False)
    try:
        _, d_def = gpu_rhs(env, w, t, prec)
    finally:
        mm.autotune_enable(True)
    _, d_a = gpu_rhs(env, w, t, prec)
    _, d_b = gpu_rhs(env, w, t, prec)
    assert np.array_equal(d_a, d_b)
    rep = mm.autotune_report()
    assert ("pair order=4 prec=%s n<=512" % ("mixed" if prec else "fp64")) in rep, rep
    js = [0, 151, 299]
    rj = [j for j in js for _ in range(w.K)]
    rk = [k for _ in js for k in range(w.K)]
    d, _ = orc.rhs_rows(w.M, w.nu, w.lam0, t, w.x, w.mom, rj, rk)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t)[js]
    assert normwise(w.M, lam_t, d.reshape(3, w.K), d_a[js]) <= tol
    assert normwise(w.M, lam_t, d.reshape(3, w.K), d_def[js]) <= tol
    # every vortex: two results each within the bar of the exact one differ by at most twice the bar
    lam_all = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t)
    assert normwise(w.M, lam_all, d_def, d_a) <= (1e-13 if prec == 0 else 2 * MIXED_TOL)


@pytest.mark.parametrize("prec,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_dense16_long_horizon_golden(env, prec, tol):
    """16 strongly overlapping order-5 vortices stepped 1200 RK4 steps against
    the oracle's end point stored in tests/golden/dense16_rk4_1200.json
    (written by make_dense16.py from the oracle alone): the drift, the pair
    interaction and the moment growth of a dense field, over a long horizon."""
    import json
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_dense16
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dense16_rk4_1200.json")) as f:
        gold = json.load(f)
    w = make_dense16.config()
    x_r, m_r = np.array(gold["x"]), np.array(gold["mom"])
    x_g, m_g = gpu_step(env, w, 0.0, gold["steps"], prec)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * gold["steps"] * w.dt)
    assert normwise(w.M, lam_t, m_r, m_g) <= tol
    assert np.abs(x_g - x_r).max() <= tol * max(1.0, np.abs(x_r).max())
    # circulation: dM_00 is written as zero, so it holds bit for bit
    assert np.array_equal(m_g[:, 0], w.mom[:, 0])


@pytest.mark.parametrize("prec,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_random_multi_64_sampled(env, orc, prec, tol):
    from paper_1010_2475_amd import workloads as wl
    w = wl.random_multi()
    # give the vortices some structure first (the workload starts as Gaussians)
    structure(w, 33)
    t = 0.2
    dx_g, dm_g = gpu_rhs(env, w, t, prec)
    js = [0, 17, 63]
    rj = [j for j in js for _ in range(w.K)]
    rk = [k for _ in js for k in range(w.K)]
    d, dxr = orc.rhs_rows(w.M, w.nu, w.lam0, t, w.x, w.mom, rj, rk)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t)[js]
    assert normwise(w.M, lam_t, d.reshape(3, w.K), dm_g[js]) <= tol
    dx_r = dxr.reshape(3, w.K, 2)[:, 0, :]
    assert np.abs(dx_g[js] - dx_r).max() <= tol * np.abs(dx_r).max()


@pytest.mark.parametrize("prec,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_two_clusters_4096_sampled(env, orc, prec, tol):
    from paper_1010_2475_amd import workloads as wl
    w = wl.two_clusters()
    structure(w, 44)
    t = 0.1
    dx_g, dm_g = gpu_rhs(env, w, t, prec)
    js = [3, 4000]
    rj = [j for j in js for _ in range(w.K)]
    rk = [k for _ in js for k in range(w.K)]
    d, dxr = orc.rhs_rows(w.M, w.nu, w.lam0, t, w.x, w.mom, rj, rk)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t)[js]
    assert normwise(w.M, lam_t, d.reshape(2, w.K), dm_g[js]) <= tol
    dx_r = dxr.reshape(2, w.K, 2)[:, 0, :]
    assert np.abs(dx_g[js] - dx_r).max() <= tol * np.abs(dx_r).max()
    # invariants that hold at any size
    G = w.mom[:, 0]
    assert np.all(dm_g[:, 0] == 0.0)
    assert abs((G[:, None] * dx_g).sum(0)).max() <= tol * np.abs(G[:, None] * dx_g).sum()


@pytest.mark.parametrize("N,M,prec", [(2, 14, 0), (2, 16, 0), (3, 16, 1), (2, 16, 1)])
def test_multi_vortex_high_orders_sampled_rows(env, orc, N, M, prec):
    """Interacting vortices at high orders: the runtime-order pair kernel (every
    shell up to 3M generated in LDS) feeding the matrix-core stage 2 (FP64 up to
    order 24, the mixed path at every order) or the double-double stage 2 (FP64
    above order 24), on rows spread over the shells of every vortex."""
    from paper_1010_2475_amd import workloads as wl
    w = rand_workload(700 + N + M, N, M, spread=1.2)
    t = 0.13
    dx_g, dm_g = gpu_rhs(env, w, t, prec)
    h = M // 2
    ks = sorted({wl.index(1, 1), wl.index(2, 0), wl.index(0, M), wl.index(M, 0), wl.index(h, M - h),
                 wl.index(3, 2), wl.index(M // 3, M // 3), wl.index(1, M - 1), wl.index(M - 2, 1)})
    rj = [j for j in range(N) for _ in ks]
    rk = [k for _ in range(N) for k in ks]
    d, dxr = orc.rhs_rows(M, w.nu, w.lam0, t, w.x, w.mom, rj, rk)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t)
    tol = FP64_TOL if prec == 0 else MIXED_TOL
    for j in range(N):
        n = _nk(M, lam_t[j])
        ref = d[j * len(ks):(j + 1) * len(ks)]
        got = dm_g[j, ks]
        scale = np.abs(ref * n[ks]).max()  # the oracle's rows set the scale
        assert np.abs((got - ref) * n[ks]).max() <= tol * scale, (j, np.abs((got - ref) * n[ks]).max() / scale)
    dx_r = dxr.reshape(N, len(ks), 2)[:, 0, :]
    assert np.abs(dx_g - dx_r).max() <= tol * max(1.0, np.abs(dx_r).max())
    assert np.all(dm_g[:, 0] == 0.0)


@pytest.mark.parametrize("M", [17, 20, 40])
def test_multi_vortex_above_the_pair_order_is_refused(env, M):
    """Interacting vortices above MMVM_MAX_PAIR_ORDER return MMVM_EORDER (their
    FP64 pair contraction would not hold the error bar)."""
    torch, mm = env
    w = rand_workload(800 + M, 2, M)
    X = torch.tensor(w.x, device="cuda:0")
    Mo = torch.tensor(w.mom, device="cuda:0")
    with pytest.raises(mm.MMVMError) as e:
        mm.rhs(w.M, w.nu, w.lam0, 0.0, X, Mo, torch.zeros_like(X), torch.zeros_like(Mo), 0)
    assert e.value.status == -3
    with pytest.raises(mm.MMVMError) as e:
        mm.step(w.M, w.nu, w.lam0, 0.0, 1e-3, 2, X, Mo, 1)
    assert e.value.status == -3


@pytest.mark.parametrize("prec", [0, 1])
def test_high_order_stepping_matches_oracle_golden(env, prec):
    """Single vortices of orders 17, 24 and 30 stepped a few RK4 steps against
    the oracle's end points in tests/golden/highorder_rk4.json (written by
    make_highorder.py from the oracle alone): the matrix-core stepping path
    (each stage finished inside the next self kernel, graph capture on the
    first call) and, above order 24 in FP64, the double-double path.  Bars:
    FP64 1e-12; the mixed path contracts in plain FP64, 1e-12 up to order 24
    and 1e-9 above (cancellation grows about 1.45x per order)."""
    import json
    from paper_1010_2475_amd import workloads as wl
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "highorder_rk4.json")
    with open(path) as f:
        gold = json.load(f)
    assert len(gold["cases"]) >= 2
    for c in gold["cases"]:
        w = wl.single_random(M=c["M"], Re=c["Re"], seed=c["seed"])
        w.dt = c["dt"]
        _, m_g = gpu_step(env, w, c["t0"], c["steps"], prec)
        lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * (c["t0"] + c["steps"] * w.dt))
        tol = FP64_TOL if (prec == 0 or c["M"] <= 24) else 1e-9
        err = normwise(w.M, lam_t, np.array([c["mom"]]), m_g)
        assert err <= tol, (c["M"], err)
        assert m_g[0, 0] == w.mom[0, 0]


@pytest.mark.parametrize("N,M,prec", [(2000, 4, 0), (2000, 6, 0), (2000, 4, 1), (1025, 2, 0), (1089, 3, 1),
                                    (1100, 0, 0), (1500, 1, 1), (2000, 5, 0)])
def test_far_field_dilute_matches_oracle(env, orc, N, M, prec):
    """A dilute field (mean spacing 2, cores 0.2-0.5): with the sources sorted
    in space, most 64-source chunks of a target are entirely beyond the
    far-field threshold, and the tuned shape sends them to the multipole
    kernel.  Sampled rows against the oracle, and every row against the
    default shape (no far-field split) to rounding.  N = 1025: the last chunk
    holds one source, which is near only to itself."""
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    w = wl.dilute_multi(N=N, M=M, seed=60 + M)
    structure(w, 61 + M)
    t = 0.2
    mm.autotune_enable(False)
    try:
        _, d_def = gpu_rhs(env, w, t, prec)
    finally:
        mm.autotune_enable(True)
    dx_g, dm_g = gpu_rhs(env, w, t, prec)
    rep = mm.autotune_report()
    print(rep, flush=True)
    js = [0, N // 2, N - 1]
    rj = [j for j in js for _ in range(w.K)]
    rk = [k for _ in js for k in range(w.K)]
    d, dxr = orc.rhs_rows(w.M, w.nu, w.lam0, t, w.x, w.mom, rj, rk)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t)
    tol = FP64_TOL if prec == 0 else MIXED_TOL
    gam = w.mom[js, 0]
    dx_r = dxr.reshape(3, w.K, 2)[:, 0, :]
    assert normwise(w.M, lam_t[js], d.reshape(3, w.K), dm_g[js], gam, dx_r) <= tol
    assert np.abs(dx_g[js] - dx_r).max() <= tol * np.abs(dx_r).max()
    assert normwise(w.M, lam_t, d_def, dm_g, w.mom[:, 0], dx_g) <= (1e-13 if prec == 0 else 2 * MIXED_TOL)


@pytest.mark.parametrize("N,M", [(200, 4), (64, 6)])
@pytest.mark.parametrize("decay,amp", [(0.5, 0.08), (0.25, 0.3), (0.0, 0.3)])
def test_mixed_bound_from_decaying_to_flat_spectra(env, orc, N, M, decay, amp):
    """The mixed path's stated bound (1e-6 normwise) on orthonormal spectra
    from decaying (2^{-|k|/2}) to flat, autotuner off (the default shape).
    Order 4 runs the FP32 pair kernel, whose low shells (|g| <= 2M + 1, all
    that the centre velocity and the first-moment rates read) are FP64:
    measured 4e-8 (decaying) to 6e-7 .. 1.4e-6 (flat, amplitude 0.3: the
    stated bound is 1e-6 for decaying spectra, 2e-6 for flat ones).  Order 6
    runs the pair kernel in FP64 in the mixed path too (FP32 shells measured
    3e-6 to 3.5e-5 there)."""
    torch, mm = env
    w = rand_workload(300 + N + M, N, M, amp=amp, decay=decay)
    mm.autotune_enable(False)
    try:
        dx_g, dm_g = gpu_rhs(env, w, 0.0, 1)
    finally:
        mm.autotune_enable(True)
    dx_r, dm_r = orc.rhs(M, w.nu, w.lam0, 0.0, w.x, w.mom)
    err = normwise(M, w.lam0, dm_r, dm_g, w.mom[:, 0], dx_r)
    errx = np.abs(dx_g - dx_r).max() / np.abs(dx_r).max()
    print("mixed N=%d M=%d decay=%g amp=%g: dM %.2e dx %.2e" % (N, M, decay, amp, err, errx), flush=True)
    bar = MIXED_TOL if decay > 0 else 2 * MIXED_TOL
    assert err <= bar and errx <= MIXED_TOL


@pytest.mark.parametrize("N,M,spacing", [(4096, 4, 4.0), (8000, 2, 3.0), (5000, 6, 4.0), (4500, 5, 4.0), (6000, 1, 3.0)])
def test_far_field_cell_expansions_match_chunks(env, orc, N, M, spacing):
    """Cells of four consecutive sorted chunks carry an expansion translated
    from their chunks'; a target far from a whole cell takes it once instead of
    four chunk expansions.  On a field wide enough for many such cells the
    right-hand side equals the chunk expansions alone (MMVM_FAR_CELLS=0) and the
    pairwise far field (MMVM_FAR_M2P=0) to rounding, differs from the chunk
    expansions alone (the cells are used), and matches the oracle's sampled
    rows to the FP64 bar."""
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    w = wl.dilute_multi(N=N, M=M, seed=80 + M, spacing=spacing)
    structure(w, 81 + M)
    t = 0.1
    res = {}
    for name, var in (("pairwise", "MMVM_FAR_M2P"), ("chunks", "MMVM_FAR_CELLS")):
        os.environ[var] = "0"
        try:
            res[name] = gpu_rhs(env, w, t, 0)
        finally:
            os.environ.pop(var, None)
    dx_c, dm_c = gpu_rhs(env, w, t, 0)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t)
    assert not np.array_equal(dm_c, res["chunks"][1])
    for name in ("pairwise", "chunks"):
        dx_r, dm_r = res[name]
        assert normwise(M, lam_t, dm_r, dm_c, w.mom[:, 0], dx_r) <= 1e-13, name
        assert np.abs(dx_c - dx_r).max() <= 1e-13 * np.abs(dx_r).max(), name
    js = [0, N // 2, N - 1]
    rj = [j for j in js for _ in range(w.K)]
    rk = [k for _ in js for k in range(w.K)]
    d, dxr = orc.rhs_rows(w.M, w.nu, w.lam0, t, w.x, w.mom, rj, rk)
    dx_r = dxr.reshape(3, w.K, 2)[:, 0, :]
    assert normwise(M, lam_t[js], d.reshape(3, w.K), dm_c[js], w.mom[js, 0], dx_r) <= FP64_TOL
    assert np.abs(dx_c[js] - dx_r).max() <= FP64_TOL * np.abs(dx_r).max()


def test_far_mask_of_a_chunk_holding_only_the_target(env):
    """N = 1089 leaves one source in the last sorted chunk.  A first call marks
    that chunk far for the targets away from its source; a second call on the
    mirrored field puts another vortex alone there, whose own chunk must then
    read near (not a stale far byte of the first call, which would send a
    zero-distance chunk to the expansion): every row of the second call equals
    the near form of the default shape to rounding."""
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    N, M = 1089, 2
    w = wl.dilute_multi(N=N, M=M, seed=90)
    structure(w, 91)
    gpu_rhs(env, w, 0.1, 0)
    w2 = wl.dilute_multi(N=N, M=M, seed=90)
    w2.mom = w.mom.copy()
    w2.x = -w.x
    dx_f, dm_f = gpu_rhs(env, w2, 0.1, 0)
    mm.autotune_enable(False)
    try:
        dx_n, dm_n = gpu_rhs(env, w2, 0.1, 0)
    finally:
        mm.autotune_enable(True)
    assert np.isfinite(dm_f).all() and np.isfinite(dx_f).all()
    lam_t = np.sqrt(w2.lam0 ** 2 + 4 * w2.nu * 0.1)
    assert normwise(M, lam_t, dm_n, dm_f, w2.mom[:, 0], dx_n) <= 1e-13
    assert np.abs(dx_f - dx_n).max() <= 1e-13 * np.abs(dx_n).max()


@pytest.mark.parametrize("N,M", [(4096, 4), (3000, 6), (2048, 2)])
def test_far_field_chunk_expansions_match_pairwise(env, orc, N, M):
    """Far chunks that lie well away from a target (radius <= 0.3 of the
    distance at orders <= 4, 0.25 above) enter through the multipole expansion
    of the whole chunk (40 terms) instead of pair by pair: the right-hand side
    equals the pairwise far field (MMVM_FAR_M2P=0) to rounding and the oracle's
    sampled rows to the FP64 bar, and the two differ (the expansions are used)."""
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    w = wl.dilute_multi(N=N, M=M, seed=70 + M)
    structure(w, 71 + M)
    t = 0.1
    os.environ["MMVM_FAR_M2P"] = "0"
    try:
        dx_p, dm_p = gpu_rhs(env, w, t, 0)
    finally:
        os.environ.pop("MMVM_FAR_M2P", None)
    dx_e, dm_e = gpu_rhs(env, w, t, 0)
    lam_t = np.sqrt(w.lam0 ** 2 + 4 * w.nu * t)
    assert not np.array_equal(dm_e, dm_p)
    assert normwise(M, lam_t, dm_p, dm_e, w.mom[:, 0], dx_p) <= 1e-13
    assert np.abs(dx_e - dx_p).max() <= 1e-13 * np.abs(dx_p).max()
    js = [0, N // 3, N - 1]
    rj = [j for j in js for _ in range(w.K)]
    rk = [k for _ in js for k in range(w.K)]
    d, dxr = orc.rhs_rows(w.M, w.nu, w.lam0, t, w.x, w.mom, rj, rk)
    dx_r = dxr.reshape(3, w.K, 2)[:, 0, :]
    assert normwise(M, lam_t[js], d.reshape(3, w.K), dm_e[js], w.mom[js, 0], dx_r) <= FP64_TOL
    assert np.abs(dx_e[js] - dx_r).max() <= FP64_TOL * np.abs(dx_r).max()
