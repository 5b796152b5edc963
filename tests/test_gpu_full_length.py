"""Whole runs of the benchmark workloads against the oracle (eq. uN over every
step), in the plans and launch shapes the benchmark uses.

The oracle takes minutes to hours on these grids, so its results were
written once by tests/golden/make_full_runs.py (which calls only oracle/ and
the seeded input generators) at 8192 seeded sample points of the final field
plus the first line along axis 0.  The brute path must match them bit for
bit, the fast path within 1e-12 absolute; the adjoint within 1e-8 relative
(max norm over the samples, against the full gradient's max norm)."""
import os

import numpy as np
import pytest

from paper_1210_4090_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FAST_TOL = 1e-12
ADJ_TOL = 1e-8


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def golden(name):
    with np.load(os.path.join(GOLDEN, name + ".npz"), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _run(torch, w, steps, method):
    from paper_1210_4090_amd.lo import Plan
    V = torch.as_tensor(w.V, device="cuda")
    p = Plan(w.n, w.tau, w.P, V=V, method=method)
    u = torch.as_tensor(w.u0, device="cuda").clone()
    p.run(u, steps)
    torch.cuda.synchronize()
    return u.reshape(-1).cpu().numpy(), p.diag()[0]


def _compare(name, got, g, method):
    ref = g["val"]
    err = float(np.max(np.abs(got[g["idx"]] - ref)))
    print("MEASURED %s %s: max |gpu - oracle| over %d samples = %.3g (|u| up to %.3g)"
          % (name, method, ref.shape[0], err, float(g["absmax"])), flush=True)
    if method == "brute":
        assert np.array_equal(got[g["idx"]], ref), err
    else:
        assert err <= FAST_TOL, err


@pytest.mark.parametrize("method", ["fast", "brute"])
def test_3d_workload_all_200_steps(torch_dev, method):
    g = golden("c3_200")
    w = wl.config3()
    print("CASE full length 3-D", method, flush=True)
    got, win = _run(torch_dev, w, int(g["steps"]), method)
    print("windows", win, flush=True)
    _compare("c3_200", got, g, method)


@pytest.mark.parametrize("method", ["fast", "brute"])
def test_2d_data_on_2048x1280_400_steps(torch_dev, method):
    """The 2-D workload's data on a grid with as many tiles on both axes as
    the headline has (its 256-thread launch shapes), 400 steps: the windows
    settle within the first 30, so most of the run is the steady state."""
    g = golden("c2_2048x1280_400")
    w = wl.config2(2048, n1=1280)
    print("CASE full length 2048x1280", method, flush=True)
    got, _ = _run(torch_dev, w, int(g["steps"]), method)
    _compare("c2_2048x1280_400", got, g, method)


@pytest.mark.parametrize("method", ["fast", "brute"])
def test_2d_workload_full_grid_30_steps(torch_dev, method):
    g = golden("c2_2048sq_30")
    w = wl.config2()
    print("CASE full grid 2048^2", method, flush=True)
    got, _ = _run(torch_dev, w, int(g["steps"]), method)
    _compare("c2_2048sq_30", got, g, method)


@pytest.mark.parametrize("ckpt_every", [50, 0])
def test_adjoint_workload_one_segment(torch_dev, ckpt_every):
    """The differentiation workload (1024^2, 64 modes) over one whole 50-step
    segment: checkpointed (recompute of the segment from its checkpoint) and
    recorded argmins, fast path, against the oracle's adjoint."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan
    g = golden("c5_adjoint_50")
    w, _ = wl.config5()
    steps = int(g["steps"])
    print("CASE adjoint one segment", ckpt_every, flush=True)
    B = torch.as_tensor(w.basis, device="cuda")
    p = Plan(w.n, w.tau, w.P, basis=B, coef=w.coef, method="fast")
    u = torch.as_tensor(w.u0, device="cuda").clone()
    gT = torch.as_tensor(np.random.default_rng(int(g["grad_seed"])).standard_normal(w.u0.shape), device="cuda")
    if ckpt_every:
        ck = p.run(u, steps, 0, ckpt_every)
        gu, gc = p.backward(ck, steps, ckpt_every, gT)
    else:
        E = p.run_record(u, steps)
        gu, gc = p.backward_recorded(E, steps, gT)
    torch.cuda.synchronize()
    _compare("c5_adjoint_50 u(T)", u.reshape(-1).cpu().numpy(), g, "fast")
    gu = gu.reshape(-1).cpu().numpy()[g["idx"]]
    rel_u = float(np.max(np.abs(gu - g["gu"]))) / float(g["gu_absmax"])
    rel_c = float(np.max(np.abs(gc - g["gc"]))) / float(np.max(np.abs(g["gc"])))
    print("MEASURED c5_adjoint_50 relative error: grad u0 %.3g, grad coef %.3g" % (rel_u, rel_c), flush=True)
    assert rel_u <= ADJ_TOL and rel_c <= ADJ_TOL, (rel_u, rel_c)


def test_batched_instance_1024_first_100_steps(torch_dev):
    """The first side-1024 instance of the batched workload, 100 steps in a
    plan of its own (the batch advances it bit for bit as such a plan does:
    test_gpu_hbar), against the oracle."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan
    g = golden("c4_inst_1024_100")
    bw = wl.config4()
    i = int(g["instance"])
    print("CASE batched instance", i, bw.P[i], flush=True)
    V = torch.as_tensor(bw.V_by_side[1024], device="cuda")
    p = Plan([1024, 1024], bw.tau, bw.P[i], V=V, method="fast")
    u = torch.zeros((1024, 1024), dtype=torch.float64, device="cuda")
    p.run(u, int(g["steps"]))
    torch.cuda.synchronize()
    _compare("c4_inst_1024_100", u.reshape(-1).cpu().numpy(), g, "fast")
