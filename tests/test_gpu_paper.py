"""The paper's own experiments (Section 5) on the GPU path, through the C ABI.

Pendulum (Section 5.1: P = 0, V = 1 - cos x) and time-dependent potential
(Section 5.2: P = 1, V = cos 2x sin t), u0 = cos x on the 2 pi torus, space
step h = pi / K, time step about sqrt(h), T = 8.  Full runs are checked
against the FP64 oracle (bit for bit on the brute path, 1e-12 on the fast
path); the self-convergence study checks the O(sqrt h) order the paper
reports for tau = sqrt(h).  Grids of 2048 points take the row sweep; 4096
points take the one-line tile sweep.
"""
import math

import numpy as np
import pytest

from paper_1210_4090_amd import workloads as wl

pytestmark = pytest.mark.gpu

FAST_TOL = 1e-12
GEN = {"pendulum": wl.pendulum, "time_dependent": wl.time_dependent}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _solve(torch, w, method, steps=None):
    from paper_1210_4090_amd.lo import Plan
    if w.tcoef is not None:
        B = torch.as_tensor(w.basis, device="cuda")
        p = Plan(w.n, w.tau, w.P, period=w.period, basis=B, tcoef=w.tcoef, method=method)
    else:
        V = torch.as_tensor(w.V, device="cuda")
        p = Plan(w.n, w.tau, w.P, period=w.period, V=V, method=method)
    u = torch.as_tensor(w.u0, device="cuda").clone()
    p.run(u, w.steps if steps is None else steps)
    return u.cpu().numpy()


def _oracle(orc, w):
    if w.tcoef is not None:
        return orc.run(w.u0, w.tau, w.P, w.steps, period=w.period, basis=w.basis, tcoef=w.tcoef)
    return orc.run(w.u0, w.tau, w.P, w.steps, V=w.V, period=w.period)


@pytest.mark.parametrize("method", ["brute", "fast"])
@pytest.mark.parametrize("K", [1024, 2048])
@pytest.mark.parametrize("name", ["pendulum", "time_dependent"])
def test_paper_experiment_full_run(torch_dev, orc, name, K, method):
    w = GEN[name](K)
    print("CASE", name, w.n, w.steps, method, flush=True)
    ref = _oracle(orc, w)
    got = _solve(torch_dev, w, method)
    if method == "brute":
        assert np.array_equal(got, ref), np.max(np.abs(got - ref))
    else:
        assert np.max(np.abs(got - ref)) <= FAST_TOL, np.max(np.abs(got - ref))


@pytest.mark.parametrize("name", ["pendulum", "time_dependent"])
def test_paper_self_convergence_order(torch_dev, name):
    """Relative max-norm error at T = 8 against the 2^17-point solution, for
    2K = 2^4 .. 2^12 points: it decreases with h, and the fitted order is
    near the 1/2 the paper observes for tau = sqrt(h)."""
    Kref = 2 ** 16
    ref = _solve(torch_dev, GEN[name](Kref), "fast")
    hs, errs = [], []
    for n in range(3, 12):
        K = 2 ** n
        u = _solve(torch_dev, GEN[name](K), "fast")
        r = ref[:: Kref // K]
        errs.append(np.max(np.abs(u - r)) / np.max(np.abs(r)))
        hs.append(math.pi / K)
    print("CASE", name, ["%.3e" % e for e in errs], flush=True)
    assert all(b < a for a, b in zip(errs, errs[1:]))
    order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 0.4 < order < 0.75, order
