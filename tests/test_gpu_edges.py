"""Degenerate cases of the GPU path against the oracle, through the C ABI:
the smallest grids the boundary accepts (3 points per axis, where every
window spans the whole torus and lifts wrap several times), constant data
(every target's candidates tie, so the lowest-offset rule decides every
argmin), runs of zero steps, caller tables whose window reaches the
table's end, and argmin offsets that do not fit int16."""
import numpy as np
import pytest

from paper_1210_4090_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _plan(torch, n, tau, P, V, method, **kw):
    from paper_1210_4090_amd.lo import Plan
    Vt = torch.as_tensor(np.ascontiguousarray(V), device="cuda")
    p = Plan(n, tau, P, V=Vt, method=method, **kw)
    p._Vhold = Vt
    return p


def _table(N, tau, half, P=0.0, q=0.0):
    """tau K*(s dx / tau) for K*(v) = v^2/2 + q v^4 - P v, s in [-half, half] (convex)."""
    d = np.arange(-half, half + 1) / N
    return tau * (0.5 * (d / tau) ** 2 + q * (d / tau) ** 4) - P * d


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


@pytest.mark.parametrize("method", ["brute", "fast"])
@pytest.mark.parametrize("n", [(96,), (40, 36)])
def test_caller_table_window_reaches_its_end(torch_dev, orc, n, method):
    """A caller table of half-width 8 under steep data: the rigorous window
    runs to the table's end (offsets past it cost +inf, so this is no error),
    and the brute kernels' blocked loop, which offers each target a few
    offsets past its window, must read +inf there.  Equal to the oracle bit
    for bit, values and argmins, over several steps."""
    torch = torch_dev
    print("CASE small table", n, method, flush=True)
    tau, half = 0.02, 8
    tabs = [_table(n[a], tau, half, P=0.1 * (a + 1)) for a in range(len(n))]
    u0 = 6.0 * wl.smooth_grid(list(n), 920, count=4, kmax=2) + 0.5 * wl.random_grid(list(n), 921)
    V = wl.smooth_grid(list(n), 922)
    P0 = [0.0] * len(n)
    p = _plan(torch, n, tau, P0, V, method, kstar_tabs=tabs)
    u = torch.as_tensor(u0, device="cuda").clone()
    arg = p.step(u, 0, argmin=True).cpu().numpy().astype(np.int64)
    ref, rarg = orc.step(u0, tau, P0, V=V, ktabs=tabs, with_argmin=True)
    assert np.array_equal(u.cpu().numpy(), ref)
    assert np.array_equal(arg, rarg.astype(np.int64))
    assert np.abs(rarg).max() == half            # minimisers do reach the end
    win, _ = p.diag()
    assert max(win) == half, win
    p.run(u, 4, n0=1)
    for k in range(4):
        ref = orc.step(ref, tau, P0, V=V, ktabs=tabs)
    assert np.array_equal(u.cpu().numpy(), ref)


def test_fixed_window_equal_to_the_table_half(torch_dev, orc):
    """A fixed window as wide as a caller table (the widest the plan accepts):
    gentle data whose minimisers stay inside it give the oracle's result bit
    for bit; steep data whose minimisers sit on its edge are reported."""
    torch = torch_dev
    from paper_1210_4090_amd._lib import LoError, LO_ERR_WINDOW
    N, tau, half = 64, 0.02, 8
    tab = _table(N, tau, half, P=0.2)
    V = wl.smooth_grid([N], 930)
    gentle = 0.05 * wl.smooth_grid([N], 931)
    p = _plan(torch, (N,), tau, [0.0], V, "brute", kstar_tabs=[tab], window=[half])
    u = torch.as_tensor(gentle, device="cuda").clone()
    arg = p.step(u, 0, argmin=True).cpu().numpy().astype(np.int64)
    ref, rarg = orc.step(gentle, tau, [0.0], V=V, ktabs=[tab], with_argmin=True)
    assert np.abs(rarg).max() < half
    assert np.array_equal(u.cpu().numpy(), ref)
    assert np.array_equal(arg, rarg.astype(np.int64))
    steep = 6.0 * wl.smooth_grid([N], 932, count=4, kmax=2)
    u = torch.as_tensor(steep, device="cuda").clone()
    with pytest.raises(LoError) as ei:
        p.step(u, 0, argmin=True)
    assert ei.value.status == LO_ERR_WINDOW


@pytest.mark.parametrize("method", ["brute", "fast"])
@pytest.mark.parametrize("N", [1000, 1001])
def test_argmin_offsets_beyond_int16_are_refused(torch_dev, orc, N, method):
    """A flat caller table with a strong drift: minimisers lie about 35000
    lifted cells away (the line wraps 35 times).  Values still equal the
    oracle's bit for bit; a step that asks for int16 argmins must refuse
    with LO_ERR_UNSUPPORTED instead of storing wrapped offsets.  N = 1000
    takes the row sweep, N = 1001 the one-line tile sweep."""
    torch = torch_dev
    from paper_1210_4090_amd._lib import LoError, LO_ERR_UNSUPPORTED
    print("CASE int16 range", N, method, flush=True)
    half, c, drift = 40000, 1e-6, 0.07
    s = np.arange(-half, half + 1, dtype=np.float64)
    tab = c * s * s - drift * s                      # convex; its minimum sits at s = 35000
    u0 = wl.smooth_grid([N], 940)
    V = wl.smooth_grid([N], 941)
    ref, rarg = orc.step(u0, 0.01, [0.0], V=V, ktabs=[tab], with_argmin=True)
    assert rarg.min() < -32767
    p = _plan(torch, (N,), 0.01, [0.0], V, method, kstar_tabs=[tab])
    u = torch.as_tensor(u0, device="cuda").clone()
    p.step(u, 0)
    assert np.array_equal(u.cpu().numpy(), ref)
    u = torch.as_tensor(u0, device="cuda").clone()
    with pytest.raises(LoError) as ei:
        p.step(u, 0, argmin=True)
    assert ei.value.status == LO_ERR_UNSUPPORTED
