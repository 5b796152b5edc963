"""The first discrete semigroup (Section 2.2, eq. cost1) on the GPU
(lo_run_semigroup1) against the FP64 oracle's path-order definition.  The
GPU path sums come from prefix sums of tau V, so values agree to rounding
(tolerance 1e-12, far above the N eps max|tau V| ~ 1e-14 difference of the two
summation orders)."""
import numpy as np
import pytest

from paper_1210_4090_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _plan(torch, N, tau, P, V, period=1.0):
    from paper_1210_4090_amd.lo import Plan
    Vt = None if V is None else torch.as_tensor(V, device="cuda")
    p = Plan((N,), tau, (P,), period=(period,), V=Vt, method="brute")
    p._V = Vt
    return p


@pytest.mark.parametrize("N,tau,P,steps", [(256, 0.05, 0.0, 20), (1000, 0.02, 0.4, 8), (97, 0.1, -0.6, 12)])
def test_semigroup1_matches_oracle(torch_dev, orc, N, tau, P, steps):
    torch = torch_dev
    print("CASE semigroup1", N, tau, P, flush=True)
    u0 = wl.smooth_grid([N], 930) + 0.05 * wl.random_grid([N], 931)
    V = wl.smooth_grid([N], 932)
    ref = orc.semigroup1_run(u0, tau, P, steps, V=V)
    p = _plan(torch, N, tau, P, V)
    u = torch.as_tensor(u0, device="cuda").clone()
    p.run_semigroup1(u, steps)
    assert np.max(np.abs(u.cpu().numpy() - ref)) <= TOL


def test_semigroup1_paper_pendulum(torch_dev, orc):
    """The Section 5.1 data (period 2 pi, V = 1 - cos x, u0 = cos x) with a
    window that holds the minimisers, against the oracle."""
    torch = torch_dev
    w = wl.pendulum(256)
    steps = 40
    ref = orc.semigroup1_run(w.u0, w.tau, w.P[0], steps, V=w.V, period=w.period[0])
    p = _plan(torch, w.n[0], w.tau, w.P[0], w.V, period=w.period[0])
    u = torch.as_tensor(w.u0, device="cuda").clone()
    p.run_semigroup1(u, steps, window=200)
    assert np.max(np.abs(u.cpu().numpy() - ref)) <= TOL


def test_semigroup1_without_potential_is_the_scheme(torch_dev, orc):
    """V = 0: the first and the fully discrete semigroups coincide."""
    torch = torch_dev
    N, tau, P = 300, 0.04, 0.3
    u0 = wl.smooth_grid([N], 935)
    p = _plan(torch, N, tau, P, None)
    u = torch.as_tensor(u0, device="cuda").clone()
    p.run_semigroup1(u, 6)
    assert np.max(np.abs(u.cpu().numpy() - orc.run(u0, tau, [P], 6))) <= TOL


def test_semigroup1_window_and_support(torch_dev):
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan
    from paper_1210_4090_amd._lib import LoError, LO_ERR_WINDOW, LO_ERR_UNSUPPORTED, LO_ERR_INVALID
    N = 128
    u0 = 3.0 * wl.smooth_grid([N], 936)
    p = _plan(torch, N, 0.05, 0.0, wl.smooth_grid([N], 937))
    u = torch.as_tensor(u0, device="cuda").clone()
    with pytest.raises(LoError) as ei:
        p.run_semigroup1(u, 2, window=1)
    assert ei.value.status == LO_ERR_WINDOW
    with pytest.raises(LoError) as ei:
        p.run_semigroup1(u, 1, window=10 ** 6)
    assert ei.value.status == LO_ERR_INVALID
    p2 = Plan((32, 16), 0.05, (0.0, 0.0), method="brute")
    u2 = torch.zeros((16, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(LoError) as ei:
        p2.run_semigroup1(u2, 1)
    assert ei.value.status == LO_ERR_UNSUPPORTED
