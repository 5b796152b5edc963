"""Batched discrete effective Hamiltonian (lo_effective_H) vs the oracle.

Each instance starts from u0 = 0 on its own grid and rotation vector P; after
T/tau steps the library reports the bracket [-max D, -min D] of
D = u(T) - u(T - 1) and its midpoint.  The oracle runs every instance alone
with the plain definition; the brute path must match it bit for bit, the
fast path within 1e-12 (each test prints the error it measured).
"""
import numpy as np
import pytest

from paper_1210_4090_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def print_case(*a):
    print("CASE", *a, flush=True)


def _V_dev(torch, bw):
    return {int(s): torch.as_tensor(v, dtype=torch.float64, device="cuda") for s, v in bw.V_by_side.items()}


def _oracle_bracket(orc, side, P, V, tau, T):
    m = int(round(1.0 / tau))
    K = int(round(T / tau))
    u0 = np.zeros((side, side))
    u1 = orc.run(u0, tau, P, K - m, V=V)
    u2 = orc.run(u1, tau, P, m, V=V)
    D = u2 - u1
    return np.array([-D.max(), -(D.max() + D.min()) * 0.5, -D.min()])


FAST_TOL = 1e-12


def _fast_check(tag, got, ref):
    err = float(np.max(np.abs(got - ref)))
    print("MEASURED %s: max |gpu - oracle| = %.3g" % (tag, err), flush=True)
    assert err <= FAST_TOL, (tag, got - ref)


@pytest.mark.parametrize("method", ["brute", "fast"])
def test_small_batch_matches_oracle(torch_dev, orc, method):
    torch = torch_dev
    from paper_1210_4090_amd.lo import effective_H
    bw = wl.config4(ninst_p1=4, ninst_p2=3, sides=(16, 24, 40), tau=0.1, T=3.0, seed=11)
    bw.P = bw.P * 4.0          # most of these lie outside the flat piece of H around P = 0
    print_case("hbar small", method, bw.ninst)
    Vd = _V_dev(torch, bw)
    out = effective_H(bw.sides, bw.P, Vd, bw.tau, bw.T, method=method)
    for i in range(bw.ninst):
        s = int(bw.sides[i])
        ref = _oracle_bracket(orc, s, bw.P[i], bw.V_by_side[s], bw.tau, bw.T)
        if method == "brute":
            assert np.array_equal(out[i], ref), (i, out[i], ref)
        else:
            _fast_check("small batch instance %d" % i, out[i], ref)
        assert out[i][0] <= out[i][1] <= out[i][2]


def test_small_odd_sides_one_line_tiles(torch_dev, orc):
    """Sides below 16 and not multiples of 8: both axes sweep in one-line
    tiles, and each instance's next windows come from a search block of its
    own (block 0 of its row of the launch grid)."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import effective_H
    bw = wl.config4(ninst_p1=3, ninst_p2=2, sides=(10, 12, 14), tau=0.1, T=3.0, seed=13)
    bw.P = bw.P * 3.0
    print_case("hbar one-line tiles", bw.ninst)
    Vd = _V_dev(torch, bw)
    out = effective_H(bw.sides, bw.P, Vd, bw.tau, bw.T, method="fast")
    for i in range(bw.ninst):
        s = int(bw.sides[i])
        ref = _oracle_bracket(orc, s, bw.P[i], bw.V_by_side[s], bw.tau, bw.T)
        _fast_check("one-line tiles instance %d (side %d)" % (i, s), out[i], ref)
        assert out[i][0] <= out[i][1] <= out[i][2]


def test_zero_rotation_gives_max_potential(torch_dev):
    """P = 0: the cheapest cycle rests at the maximum of V (zero kinetic
    cost), so the discrete effective Hamiltonian is max V on the grid and
    the bracket contains it."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import effective_H
    sides = np.array([32, 48, 32])
    P = np.zeros((3, 2))
    Vs = {32: wl.smooth_grid([32, 32], 5), 48: wl.smooth_grid([48, 48], 5)}
    Vd = {k: torch.as_tensor(v, device="cuda") for k, v in Vs.items()}
    out = effective_H(sides, P, Vd, 0.05, 4.0, method="fast")
    for i, s in enumerate(sides):
        vmax = Vs[int(s)].max()
        assert out[i][0] - 1e-12 <= vmax <= out[i][2] + 1e-12, (out[i], vmax)


@pytest.mark.parametrize("method", ["brute", "fast"])
def test_batched_equals_individual_runs(torch_dev, method):
    """The batch advances every instance exactly as a plan of its own would."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan, effective_H
    bw = wl.config4(ninst_p1=3, ninst_p2=3, sides=(64, 96), tau=0.05, T=2.0, seed=12)
    print_case("hbar batched vs individual", method)
    Vd = _V_dev(torch, bw)
    out = effective_H(bw.sides, bw.P, Vd, bw.tau, bw.T, method=method)
    for i in range(bw.ninst):
        s = int(bw.sides[i])
        p = Plan([s, s], bw.tau, bw.P[i], V=Vd[s], method=method)
        u = torch.zeros((s, s), dtype=torch.float64, device="cuda")
        p.run(u, 20)
        snap = u.clone()
        p.run(u, 20, n0=20)
        D = (u - snap).cpu().numpy()
        ref = np.array([-D.max(), -(D.max() + D.min()) * 0.5, -D.min()])
        assert np.array_equal(out[i], ref), (i, out[i] - ref)


def test_large_rotation_full_length_vs_oracle(torch_dev, orc):
    """256^2 grids, tau = 0.02, T = 20 (1000 steps) at rotation vectors
    outside the flat piece of H, where the bracket is not trivially max V."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import effective_H
    bw = wl.config4(ninst_p1=2, ninst_p2=2, sides=(256,), seed=13)
    bw.P = np.array([[3.0, 1.5], [-2.5, 3.5], [4.0, -0.5], [0.5, 0.25]])
    Vd = _V_dev(torch, bw)
    out = effective_H(bw.sides, bw.P, Vd, bw.tau, bw.T, method="fast")
    for i in (0, 1):
        ref = _oracle_bracket(orc, 256, bw.P[i], bw.V_by_side[256], bw.tau, bw.T)
        print("P", bw.P[i], out[i], ref, out[i] - ref, flush=True)
        assert ref[1] > bw.V_by_side[256].max() + 0.1
        _fast_check("P = %s, 1000 steps" % bw.P[i], out[i], ref)


def test_invalid_time_step_rejected(torch_dev):
    torch = torch_dev
    from paper_1210_4090_amd._lib import LoError
    from paper_1210_4090_amd.lo import effective_H
    V = {16: torch.zeros((16, 16), dtype=torch.float64, device="cuda")}
    with pytest.raises(LoError):
        effective_H([16], np.zeros((1, 2)), V, 0.03, 3.0)     # 1/tau not an integer
    with pytest.raises(LoError):
        effective_H([16], np.zeros((1, 2)), V, 0.1, 0.05)     # T shorter than one time unit


def test_full_batch_512_instances(torch_dev, orc):
    """The full workload (512 instances, sides 256..1024, tau = 0.02,
    T = 20): brackets are ordered and contain max V (every P of the workload
    lies in the flat piece of the effective Hamiltonian around P = 0, where it
    equals max V), P and -P on the same grid agree (V is even), a side-1024
    instance equals a plan of its own bit for bit, and the 256^2 instance of
    largest |P| is recomputed by the oracle in full."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan, effective_H
    bw = wl.config4()
    print_case("hbar full", bw.ninst)
    Vd = _V_dev(torch, bw)
    out = effective_H(bw.sides, bw.P, Vd, bw.tau, bw.T, method="fast")
    assert np.all(np.isfinite(out))
    assert np.all(out[:, 0] <= out[:, 1]) and np.all(out[:, 1] <= out[:, 2])
    vmax = np.array([bw.V_by_side[int(s)].max() for s in bw.sides])
    assert np.all(out[:, 0] - FAST_TOL <= vmax) and np.all(vmax <= out[:, 2] + FAST_TOL), \
        np.flatnonzero((out[:, 0] - FAST_TOL > vmax) | (vmax > out[:, 2] + FAST_TOL))
    width = out[:, 2] - out[:, 0]
    print("MEASURED bracket width: max %.3g, median %.3g; max |mid - max V| %.3g"
          % (width.max(), np.median(width), np.max(np.abs(out[:, 1] - vmax))), flush=True)
    i = int(np.flatnonzero(bw.sides == 1024)[0])
    steps, unit = int(round(bw.T / bw.tau)), int(round(1.0 / bw.tau))
    p = Plan([1024, 1024], bw.tau, bw.P[i], V=Vd[1024], method="fast")
    u = torch.zeros((1024, 1024), dtype=torch.float64, device="cuda")
    p.run(u, steps - unit)
    snap = u.clone()
    p.run(u, unit, n0=steps - unit)
    D = (u - snap).cpu().numpy()
    alone = np.array([-D.max(), -(D.max() + D.min()) * 0.5, -D.min()])
    assert np.array_equal(out[i], alone), (i, out[i] - alone)
    pairs = 0
    for i in range(bw.ninst):
        j = int(np.argmin(np.sum(np.abs(bw.P + bw.P[i]), axis=1)))
        if np.allclose(bw.P[j], -bw.P[i]) and bw.sides[j] == bw.sides[i] and j > i:
            assert abs(out[i, 1] - out[j, 1]) <= 1e-8, (i, j, out[i], out[j])
            pairs += 1
    print("mirror pairs checked:", pairs, flush=True)
    cand = np.flatnonzero(bw.sides == 256)
    i = int(cand[np.argmax(np.sum(bw.P[cand] ** 2, axis=1))])   # far from the flat piece around P = 0
    ref = _oracle_bracket(orc, 256, bw.P[i], bw.V_by_side[256], bw.tau, bw.T)
    print("instance", i, out[i], ref, out[i] - ref, flush=True)
    _fast_check("instance %d of the full batch" % i, out[i], ref)


def test_autotuned_batches_bitwise_identical(torch_dev):
    """The launch-shape tuner applied to every batch changes no bracket."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import effective_H
    bw = wl.config4(ninst_p1=3, ninst_p2=2, sides=(128, 192), tau=0.05, T=4.0, seed=14)
    print_case("hbar autotuned")
    Vd = _V_dev(torch, bw)
    a = effective_H(bw.sides, bw.P, Vd, bw.tau, bw.T, method="fast")
    b = effective_H(bw.sides, bw.P, Vd, bw.tau, bw.T, method="fast", autotune=True)
    assert np.array_equal(a, b), a - b
