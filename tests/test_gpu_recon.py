"""GPU tests of the diagnostics: the vorticity reconstructed on a grid
(eq:moment_expansion_def_tw0) and the non-axisymmetric enstrophy
(eq:nonaxi_enstrophy), against the oracle and the closed form of the
quadrupole initial condition eq:IC_sd."""
import math
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


def _grid(env, w, t, x0, y0, h, nx, ny):
    torch, mm = env
    dev = torch.device("cuda:0")
    X = torch.tensor(w.x, device=dev)
    Mo = torch.tensor(w.mom, device=dev)
    om = torch.full((ny, nx), 7.0, dtype=torch.float64, device=dev)
    print("vorticity_grid N=%d M=%d %dx%d" % (w.N, w.M, nx, ny), flush=True)
    mm.vorticity_grid(w.M, w.nu, w.lam0, t, X, Mo, x0, y0, h, nx, ny, om)
    torch.cuda.synchronize()
    return om.cpu().numpy()


@pytest.mark.parametrize("case", ["single24", "multi36", "multi300"])
def test_vorticity_grid_matches_oracle(env, orc, case):
    from paper_1010_2475_amd import workloads as wl
    from test_gpu_parity import rand_workload
    if case == "single24":
        w = wl.single_random(M=24, Re=700.0, seed=7)
        x0, y0, h, nx, ny = -9.0, -8.5, 0.11, 170, 153   # ragged tiles
    elif case == "multi36":
        w = rand_workload(12, 36, 2, spread=2.0)
        x0, y0, h, nx, ny = -3.5, -3.0, 0.037, 190, 170
    else:
        w = rand_workload(13, 300, 4, spread=3.0)
        x0, y0, h, nx, ny = -4.0, -4.0, 0.02, 400, 400
    t = 0.3
    om = _grid(env, w, t, x0, y0, h, nx, ny)
    rng = np.random.default_rng(3)
    ix = rng.integers(0, nx, 40)
    iy = rng.integers(0, ny, 40)
    ix[:2] = [0, nx - 1]
    iy[:2] = [ny - 1, 0]
    ref = orc.vorticity(w.M, w.nu, w.lam0, t, w.x, w.mom, x0 + h * ix, y0 + h * iy)
    got = om[iy, ix]
    scale = np.abs(om).max()
    assert np.abs(got - ref).max() <= 1e-12 * scale, np.abs(got - ref).max() / scale


def test_vorticity_grid_integrates_to_circulation(env):
    from test_gpu_parity import rand_workload
    w = rand_workload(14, 5, 6, spread=1.0)
    h = 0.02
    om = _grid(env, w, 0.0, -6.0, -6.0, h, 600, 600)
    total = om.sum() * h * h
    assert abs(total - w.mom[:, 0].sum()) <= 1e-10 * np.abs(w.mom[:, 0]).sum()


def test_vorticity_grid_many_vortices_in_chunks(env, orc):
    """Enough vortices that their tables are taken in several chunks (later
    chunks add to the grid)."""
    from test_gpu_parity import rand_workload
    w = rand_workload(15, 4000, 6, spread=4.0)
    x0, y0, h, n = -4.0, -4.0, 8.0 / 2047, 2048
    om = _grid(env, w, 0.1, x0, y0, h, n, n)
    rng = np.random.default_rng(4)
    ix, iy = rng.integers(0, n, 12), rng.integers(0, n, 12)
    ref = orc.vorticity(w.M, w.nu, w.lam0, 0.1, w.x, w.mom, x0 + h * ix, y0 + h * iy)
    assert np.abs(om[iy, ix] - ref).max() <= 1e-11 * np.abs(om).max()


def _enstrophy(env, w, t, cx, cy, rmax, nr, nth):
    torch, mm = env
    dev = torch.device("cuda:0")
    X = torch.tensor(w.x, device=dev)
    Mo = torch.tensor(w.mom, device=dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    print("enstrophy N=%d M=%d nr=%d nth=%d" % (w.N, w.M, nr, nth), flush=True)
    mm.enstrophy_nonaxi(w.M, w.nu, w.lam0, t, X, Mo, cx, cy, rmax, nr, nth, E)
    torch.cuda.synchronize()
    return float(E.cpu()[0])


@pytest.mark.parametrize("delta", [0.1, 0.02])
def test_enstrophy_quadrupole_closed_form(env, delta):
    from paper_1010_2475_amd import workloads as wl
    w = wl.single_quadrupole(M=10, delta=delta)
    E = _enstrophy(env, w, 0.0, 0.0, 0.0, 16.0, 48, 32)
    ref = 32 * delta ** 2 / (math.pi * 2.0 ** 6)
    assert abs(E - ref) <= 1e-12 * ref, (E, ref)


def test_enstrophy_matches_oracle(env, orc):
    from paper_1010_2475_amd import workloads as wl
    w = wl.single_random(M=10, Re=300.0, seed=9)
    t = 0.4
    E = _enstrophy(env, w, t, 0.0, 0.0, 18.0, 64, 48)
    # the oracle's composite Simpson in r has an O(h^4) error from the centre (the
    # first angular modes go as r^3 there): 4800 intervals put it near 1e-12
    Er = orc.enstrophy_nonaxi(w.M, w.nu, w.lam0, t, w.x, w.mom, 0.0, 0.0, 18.0, 4800, 48)
    assert abs(E - Er) <= 1e-10 * Er, (E, Er)
    # an axisymmetric state has none
    mom = np.zeros_like(w.mom)
    mom[0, 0] = 1.0
    mom[0, wl.index(2, 0)] = mom[0, wl.index(0, 2)] = 0.2
    w.mom = mom
    assert abs(_enstrophy(env, w, t, 0.0, 0.0, 18.0, 64, 48)) <= 1e-20


def test_diagnostics_reject_bad_arguments(env):
    torch, mm = env
    from paper_1010_2475_amd import workloads as wl
    w = wl.single_quadrupole(M=4)
    X = torch.tensor(w.x, device="cuda:0")
    Mo = torch.tensor(w.mom, device="cuda:0")
    with pytest.raises(mm.MMVMError) as e:
        mm.vorticity_grid(w.M, w.nu, w.lam0, 0.0, X, Mo, 0.0, 0.0, -1.0, 4, 4,
                          torch.zeros((4, 4), dtype=torch.float64, device="cuda:0"))
    assert e.value.status == -1
    with pytest.raises(mm.MMVMError) as e:
        mm.enstrophy_nonaxi(w.M, w.nu, w.lam0, 0.0, X, Mo, 0.0, 0.0, 5.0, 0, 8,
                            torch.zeros(1, dtype=torch.float64, device="cuda:0"))
    assert e.value.status == -1
