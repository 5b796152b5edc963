"""Degenerate cases of the GPU path against the oracle, through the C ABI:
the smallest grids the boundary accepts (3 points per axis, where every
window spans the whole torus and lifts wrap several times), constant data
(every target's candidates tie, so the lowest-offset rule decides every
argmin) and runs of zero steps."""
import numpy as np
import pytest

from paper_1210_4090_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _plan(torch, n, tau, P, V, method):
    from paper_1210_4090_amd.lo import Plan
    Vt = torch.as_tensor(np.ascontiguousarray(V), device="cuda")
    p = Plan(n, tau, P, V=Vt, method=method)
    p._Vhold = Vt
    return p


@pytest.mark.parametrize("method", ["brute", "fast"])
@pytest.mark.parametrize("n", [(3,), (3, 3), (3, 3, 3), (3, 8, 5)])
def test_smallest_grids(torch_dev, orc, n, method):
    torch = torch_dev
    print("CASE smallest", n, method, flush=True)
    tau, P = 0.4, [0.3, -0.2, 0.1][: len(n)]
    u0 = wl.random_grid(list(n), 900)
    V = wl.random_grid(list(n), 901, 0.5)
    p = _plan(torch, n, tau, P, V, method)
    u = torch.as_tensor(u0, device="cuda").clone()
    arg = p.step(u, 0, argmin=True).cpu().numpy().astype(np.int64)
    ref, rarg = orc.step(u0, tau, P, V=V, with_argmin=True)
    got = u.cpu().numpy()
    if method == "brute":
        assert np.array_equal(got, ref)
    else:
        assert np.max(np.abs(got - ref)) <= 1e-12
    same = got == ref
    assert np.array_equal(arg[:, same], rarg[:, same].astype(np.int64))
    p.run(u, 5, n0=1)
    ref = orc.run(ref, tau, P, 5, V=V, n0=1)
    assert np.max(np.abs(u.cpu().numpy() - ref)) <= (0 if method == "brute" else 1e-12)


@pytest.mark.parametrize("method", ["brute", "fast"])
@pytest.mark.parametrize("n,P", [((64,), (0.0,)), ((40, 24), (0.25, -0.5))])
def test_constant_data_ties(torch_dev, orc, n, P, method):
    """u0 constant, V = 0: the minimum over offsets is the kinetic table's,
    tied across every target; argmins follow the lowest-offset rule exactly."""
    torch = torch_dev
    print("CASE constant", n, P, method, flush=True)
    tau = 0.05
    u0 = np.full(tuple(reversed(n)), 0.75)
    V = np.zeros_like(u0)
    p = _plan(torch, n, tau, list(P), V, method)
    u = torch.as_tensor(u0, device="cuda").clone()
    arg = p.step(u, 0, argmin=True).cpu().numpy().astype(np.int64)
    ref, rarg = orc.step(u0, tau, list(P), V=V, with_argmin=True)
    got = u.cpu().numpy()
    assert np.array_equal(got, ref)
    assert np.array_equal(arg, rarg.astype(np.int64))


@pytest.mark.parametrize("method", ["brute", "fast"])
def test_zero_steps_leave_u_unchanged(torch_dev, method):
    torch = torch_dev
    n = (96, 64)
    u0 = wl.smooth_grid(list(n), 910)
    p = _plan(torch, n, 0.02, [0.1, 0.2], wl.smooth_grid(list(n), 911), method)
    u = torch.as_tensor(u0, device="cuda").clone()
    p.run(u, 0)
    assert np.array_equal(u.cpu().numpy(), u0)
