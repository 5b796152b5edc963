"""lo_step_noalloc (one step with no plan and no device allocation, its work
memory in the library's static device array) against lo_step through the C
ABI: the same values and argmins bit for bit, on consecutive calls whose
second input is smaller, at the largest grid the static array holds, in
1-D to 3-D, for both methods; and several steps against lo_run and the
oracle."""
import numpy as np
import pytest

from paper_1210_4090_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _inputs(torch, n, seed):
    u0 = torch.as_tensor(wl.smooth_grid(list(n), seed), device="cuda")
    V = torch.as_tensor(wl.smooth_grid(list(n), seed + 1), device="cuda")
    return u0, V


def _compare(torch, n, tau, P, method, argmin, seed, step=0):
    """One lo_step on a plan against one lo_step_noalloc on the same data."""
    from paper_1210_4090_amd.lo import Plan, step_noalloc
    print("CASE noalloc", n, method, "argmin" if argmin else "", flush=True)
    u0, V = _inputs(torch, n, seed)
    plan = Plan(n, tau, P, V=V, method=method)
    ua = u0.clone()
    arg_a = plan.step(ua, step, argmin=argmin)
    plan.close()
    ub = u0.clone()
    tau_v = tau * V                      # fl(tau V), the plan's table
    arg_b = step_noalloc(ub, n, tau, P, tau_v=tau_v, step=step, method=method, argmin=argmin)
    torch.cuda.synchronize()
    assert torch.equal(ua, ub), float((ua - ub).abs().max())
    if argmin:
        assert torch.equal(arg_a, arg_b)


@pytest.mark.parametrize("method", ["fast", "brute"])
def test_two_calls_second_smaller(torch_dev, method):
    torch = torch_dev
    _compare(torch, (512, 384), 0.01, (0.3, 0.1), method, True, 11)
    _compare(torch, (200, 130), 0.02, (-0.4, 0.25), method, True, 13, step=3)


@pytest.mark.parametrize("method", ["fast", "brute"])
@pytest.mark.parametrize("n", [(4096,), (1000,), (64, 48, 40), (35, 3, 17)])
def test_grids_of_each_rank(torch_dev, n, method):
    P = [0.2, -0.1, 0.05][: len(n)]
    _compare(torch_dev, n, 0.02, P, method, True, 21)
    _compare(torch_dev, n, 0.02, P, method, False, 23)


def test_largest_grid_the_array_holds(torch_dev):
    from paper_1210_4090_amd._lib import LO_NOALLOC_MAX_POINTS
    assert 2048 * 2048 == LO_NOALLOC_MAX_POINTS
    _compare(torch_dev, (2048, 2048), 0.01, (0.3, 0.1), "fast", False, 31)
    _compare(torch_dev, (1024, 512), 0.01, (0.3, 0.1), "fast", True, 33)


@pytest.mark.parametrize("method", ["fast", "brute"])
def test_steps_against_run_and_oracle(torch_dev, orc, method):
    """Ten calls, step index n = 0..9 (a time-independent potential): the same
    values as lo_run over ten steps, and the oracle's (bitwise on the brute
    path, within 1e-12 on the fast path)."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan, step_noalloc
    n, tau, P, steps = (300, 260), 0.02, (0.3, -0.2), 10
    print("CASE noalloc run", n, method, flush=True)
    u0, V = _inputs(torch, n, 41)
    plan = Plan(n, tau, P, V=V, method=method)
    ua = u0.clone()
    plan.run(ua, steps)
    plan.close()
    ub = u0.clone()
    tau_v = tau * V
    for k in range(steps):
        step_noalloc(ub, n, tau, P, tau_v=tau_v, step=k, method=method)
    torch.cuda.synchronize()
    assert torch.equal(ua, ub), float((ua - ub).abs().max())
    ref = orc.run(u0.cpu().numpy(), tau, P, steps, V=V.cpu().numpy())
    err = float(np.max(np.abs(ub.cpu().numpy() - ref)))
    assert err <= (0.0 if method == "brute" else 1e-12), err


def test_rejections(torch_dev):
    """Beyond the static array, and caller tables, are refused before any
    device work; u is left as it was."""
    torch = torch_dev
    from paper_1210_4090_amd._lib import LO_ERR_UNSUPPORTED, LoError
    from paper_1210_4090_amd.lo import step_noalloc
    u = torch.zeros((2049, 2048), dtype=torch.float64, device="cuda")
    with pytest.raises(LoError) as e:
        step_noalloc(u, (2048, 2049), 0.01, (0.0, 0.0))
    assert e.value.status == LO_ERR_UNSUPPORTED
    assert float(u.abs().max()) == 0.0
