"""The paper's own fast algorithm (Section 4) as a comparison path on the GPU
(lo_run_decomp): convex / concave pieces, each convolved in linear time,
minimum over the pieces.  With eta = 0 and a window holding the minimisers it
must reproduce the definition (the FP64 oracle) bit for bit: every value
written is a genuine candidate and the pair that attains the rounded minimum
is among them.  eta > 0 trades pieces for error (Section 4.3)."""
import numpy as np
import pytest

from paper_1210_4090_amd import workloads as wl

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _plan(torch, w, method="fast"):
    from paper_1210_4090_amd.lo import Plan
    if w.tcoef is not None:
        B = torch.as_tensor(w.basis, device="cuda")
        p = Plan(w.n, w.tau, w.P, period=w.period, basis=B, tcoef=w.tcoef, method=method)
        p._B = B
    else:
        V = torch.as_tensor(w.V, device="cuda")
        p = Plan(w.n, w.tau, w.P, period=w.period, V=V, method=method)
        p._V = V
    return p


def _oracle(orc, w, steps):
    if w.tcoef is not None:
        return orc.run(w.u0, w.tau, w.P, steps, period=w.period, basis=w.basis, tcoef=w.tcoef)
    return orc.run(w.u0, w.tau, w.P, steps, V=w.V, period=w.period)


def _claim_window(torch, w, steps):
    """The widest rigorous window of the run, from the claim path."""
    p = _plan(torch, w)
    u = torch.as_tensor(w.u0, device="cuda").clone()
    p.run(u, steps)
    return p.diag()[0][0]


@pytest.mark.parametrize("name", ["pendulum", "time_dependent"])
def test_decomposition_eta0_full_run_matches_oracle(torch_dev, orc, name):
    torch = torch_dev
    w = {"pendulum": wl.pendulum, "time_dependent": wl.time_dependent}[name](1024)
    print("CASE decomp", name, w.n, w.steps, flush=True)
    W = _claim_window(torch, w, w.steps) + 2
    ref = _oracle(orc, w, w.steps)
    p = _plan(torch, w)
    u = torch.as_tensor(w.u0, device="cuda").clone()
    pieces, breaks = p.run_decomp(u, w.steps, eta=0.0, window=W)
    got = u.cpu().numpy()
    assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))
    assert pieces >= w.steps and 0 <= breaks <= pieces


def test_decomposition_rough_data_whole_table(torch_dev, orc):
    """Rough data (many pieces) on a ragged 1000-point line, window = 0 (the
    plan's whole table)."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan
    n, tau, P = (1000,), 0.02, (0.4,)
    u0 = wl.smooth_grid(list(n), 920) + 0.05 * wl.random_grid(list(n), 921)
    V = wl.smooth_grid(list(n), 922)
    p = Plan(n, tau, P, V=torch.as_tensor(V, device="cuda"), method="fast")
    u = torch.as_tensor(u0, device="cuda").clone()
    pieces, breaks = p.run_decomp(u, 3, eta=0.0, window=0)
    ref = orc.run(u0, tau, P, 3, V=V)
    got = u.cpu().numpy()
    assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))
    assert breaks > 100   # rough data: many convex / concave alternations


def test_decomposition_tolerance_trades_pieces_for_error(torch_dev):
    """A larger tolerance merges pieces (fewer breaks) and moves the result
    away from the exact one."""
    torch = torch_dev
    w = wl.pendulum(2048)
    steps = 60
    W = _claim_window(torch, w, steps) + 2
    exact = None
    res = []
    for eta in (0.0, 0.01, 1.0):
        p = _plan(torch, w)
        u = torch.as_tensor(w.u0, device="cuda").clone()
        pieces, breaks = p.run_decomp(u, steps, eta=eta, window=W)
        got = u.cpu().numpy()
        if exact is None:
            exact = got
        res.append((eta, breaks, np.max(np.abs(got - exact))))
    print("CASE decomp eta", res, flush=True)
    assert res[0][2] == 0.0
    assert res[2][1] <= res[1][1] <= res[0][1]
    assert res[2][2] >= res[1][2]


def test_decomposition_rejects_what_it_does_not_cover(torch_dev):
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan
    from paper_1210_4090_amd._lib import LoError, LO_ERR_INVALID, LO_ERR_UNSUPPORTED
    p2 = Plan((32, 16), 0.05, (0.0, 0.0), method="fast")
    u2 = torch.zeros((16, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(LoError) as ei:
        p2.run_decomp(u2, 1)
    assert ei.value.status == LO_ERR_UNSUPPORTED
    p1 = Plan((64,), 0.05, (0.0,), method="fast")
    u1 = torch.zeros(64, dtype=torch.float64, device="cuda")
    for kw in ({"eta": -1.0}, {"window": 100000}):
        with pytest.raises(LoError) as ei:
            p1.run_decomp(u1, 1, **kw)
        assert ei.value.status == LO_ERR_INVALID
