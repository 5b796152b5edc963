"""Reverse pass (lo_backward) vs the oracle's adjoint, through the C ABI.

The oracle stores every argmin of the forward run and scatters the upstream
gradient back in a sequential loop over the grid; the library recomputes
segments from checkpoints and sums each source's run of targets.  On the
brute path the argmins are bitwise those of the oracle and the additions
happen in the same order, so the gradient with respect to u0 is compared
bit for bit; the potential's gradient differs only in the order of its final
reduction.  The fast path must agree within 1e-8 (relative, max norm).
"""
import numpy as np
import pytest

from paper_1210_4090_amd import workloads as wl

pytestmark = pytest.mark.gpu

ADJ_TOL = 1e-8
COEF_TOL_EXACT_ARGMIN = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _gpu(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def print_case(*a):
    print("CASE", *a, flush=True)


def _basis(n, count, seed):
    """`count` seeded Fourier modes (cos and sin of integer wave vectors)."""
    ndim = len(n)
    ks = wl.wave_vectors(ndim, 3.0)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(ks.shape[0], size=count, replace=False))
    kinds = ["cos" if i % 2 == 0 else "sin" for i in range(count)]
    return wl.basis_tables(n, ks[idx], kinds)


def _rel(got, ref):
    return np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)


def _run_adjoint(torch, n, tau, P, basis, coef, u0, gT, nsteps, every, method):
    from paper_1210_4090_amd.lo import Plan
    B = _gpu(torch, basis)
    p = Plan(n, tau, P, basis=B, coef=coef, method=method)
    u = _gpu(torch, u0)
    ck = p.run(u, nsteps, 0, every)
    gu, gc = p.backward(ck, nsteps, every, _gpu(torch, gT))
    return u.cpu().numpy(), gu.cpu().numpy(), gc, p


CASES = [
    # (n, tau, P, steps, checkpoint spacing)
    ((64,), 0.05, (0.3,), 30, 7),
    ((257,), 0.02, (-0.7,), 25, 25),
    ((48, 40), 0.04, (0.2, -0.1), 20, 6),
    ((130, 96), 0.01, (0.3, 0.1), 12, 5),
    ((12, 10, 16), 0.05, (0.1, -0.2, 0.3), 6, 4),
]


@pytest.mark.parametrize("method", ["brute", "fast"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_adjoint_matches_oracle(torch_dev, orc, case, method):
    torch = torch_dev
    n, tau, P, steps, every = CASES[case]
    print_case("adjoint", n, steps, every, method)
    basis = _basis(n, 6, 100 + case)
    coef = np.random.default_rng(200 + case).standard_normal(basis.shape[0]) * 0.5
    u0 = wl.smooth_grid(list(n), 300 + case)
    gT = np.random.default_rng(400 + case).standard_normal(u0.shape)
    uT_ref, gu_ref, gc_ref = orc.adjoint(u0, tau, P, steps, basis, coef, gT)
    uT, gu, gc, _ = _run_adjoint(torch, n, tau, P, basis, coef, u0, gT, steps, every, method)
    if method == "brute":
        assert np.array_equal(uT, uT_ref)
        assert np.array_equal(gu, gu_ref), "max diff %g" % np.max(np.abs(gu - gu_ref))
        assert _rel(gc, gc_ref) <= COEF_TOL_EXACT_ARGMIN, _rel(gc, gc_ref)
    else:
        assert _rel(gu, gu_ref) <= ADJ_TOL, _rel(gu, gu_ref)
        assert _rel(gc, gc_ref) <= ADJ_TOL, _rel(gc, gc_ref)


def test_adjoint_rough_data_wide_windows(torch_dev, orc):
    """Random (rough) data: windows cover most of the line, many runs wrap."""
    torch = torch_dev
    n, tau, P, steps, every = (40, 33), 0.3, (0.7, -0.4), 8, 3
    print_case("adjoint rough", n)
    basis = _basis(n, 4, 7)
    coef = np.array([0.3, -0.2, 0.5, 0.1])
    u0 = wl.random_grid(list(n), 8)
    gT = np.random.default_rng(9).standard_normal(u0.shape)
    _, gu_ref, gc_ref = orc.adjoint(u0, tau, P, steps, basis, coef, gT)
    _, gu, gc, p = _run_adjoint(torch, n, tau, P, basis, coef, u0, gT, steps, every, "brute")
    assert np.array_equal(gu, gu_ref), "max diff %g" % np.max(np.abs(gu - gu_ref))
    assert _rel(gc, gc_ref) <= COEF_TOL_EXACT_ARGMIN
    win, amax = p.diag()
    assert min(amax) >= 1


def test_adjoint_zero_steps_is_identity(torch_dev):
    torch = torch_dev
    n = (32, 24)
    basis = _basis(n, 2, 1)
    u0 = wl.smooth_grid(list(n), 2)
    gT = np.random.default_rng(3).standard_normal(u0.shape)
    _, gu, gc, _ = _run_adjoint(torch, n, 0.05, (0.1, 0.2), basis, np.ones(2), u0, gT, 0, 5, "brute")
    assert np.array_equal(gu, gT)
    assert np.all(gc == 0.0)


def test_adjoint_mass_and_linearity(torch_dev):
    """Each reverse sweep moves every target's gradient to exactly one
    source, so sum(grad_u0) = sum(grad_uT) up to rounding; and the adjoint is
    linear in the upstream gradient (same argmins)."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan
    n, tau, P = (96, 80), 0.02, (0.3, -0.2)
    basis = _basis(n, 4, 11)
    B = _gpu(torch, basis)
    p = Plan(n, tau, P, basis=B, coef=np.array([0.5, -0.3, 0.2, 0.1]), method="fast")
    u = _gpu(torch, wl.smooth_grid(list(n), 12))
    ck = p.run(u, 40, 0, 10)
    rng = np.random.default_rng(13)
    g1, g2 = rng.standard_normal((2,) + u.shape)
    a1, c1 = p.backward(ck, 40, 10, _gpu(torch, g1))
    a2, c2 = p.backward(ck, 40, 10, _gpu(torch, g2))
    a12, c12 = p.backward(ck, 40, 10, _gpu(torch, 2.0 * g1 - g2))
    a1, a2, a12 = (t.cpu().numpy() for t in (a1, a2, a12))
    assert abs(a1.sum() - g1.sum()) <= 1e-11 * np.abs(g1).sum()
    assert np.max(np.abs(a12 - (2.0 * a1 - a2))) <= 1e-12 * np.max(np.abs(a12))
    assert np.max(np.abs(c12 - (2.0 * c1 - c2))) <= 1e-10 * np.max(np.abs(c12))


def test_autograd_function(torch_dev):
    """LaxOleinik.apply gives the library's adjoint through torch.autograd."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import LaxOleinik, Plan
    n, tau, P, steps, every = (64, 48), 0.03, (0.2, 0.1), 15, 4
    basis = _basis(n, 4, 21)
    B = _gpu(torch, basis)
    c0 = np.array([0.4, -0.1, 0.3, 0.2])
    p = Plan(n, tau, P, basis=B, coef=c0, method="fast")
    u0 = _gpu(torch, wl.smooth_grid(list(n), 22)).requires_grad_(True)
    coef = torch.tensor(c0, dtype=torch.float64, device="cuda", requires_grad=True)
    wgt = _gpu(torch, np.random.default_rng(23).standard_normal(u0.shape))
    uT = LaxOleinik.apply(u0, coef, p, steps, every)
    loss = (uT * wgt).sum()
    gu, gc = torch.autograd.grad(loss, [u0, coef])
    ck = p.run(u0.detach().clone(), steps, 0, every)
    ru, rc = p.backward(ck, steps, every, wgt)
    assert torch.equal(gu, ru)
    assert np.array_equal(gc.cpu().numpy(), rc)


def test_finite_differences_full_size(torch_dev):
    """1024^2 differentiation workload (500 steps, checkpoints every 50):
    the adjoint's directional derivatives in u0 and in the coefficients
    against central differences (the map is piecewise affine, so they agree
    up to the few argmins that switch between the perturbed runs)."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan
    w, _ = wl.config5()
    print_case("config5 fd", w.n, w.steps)
    B = _gpu(torch, w.basis)
    c = np.asarray(w.coef)
    p = Plan(w.n, w.tau, w.P, basis=B, coef=c, method="fast")
    u0 = _gpu(torch, w.u0)
    wgt = _gpu(torch, np.random.default_rng(31).standard_normal(w.u0.shape))

    def loss(du, dc):
        p.set_coef(c + dc)
        u = u0 + du
        p.run(u, w.steps)
        return float((u * wgt).sum())

    u = u0.clone()
    p.set_coef(c)
    ck = p.run(u, w.steps, 0, 50)
    gu, gc = p.backward(ck, w.steps, 50, wgt)
    assert abs(float(gu.sum()) - float(wgt.sum())) <= 1e-9 * float(wgt.abs().sum())
    rng = np.random.default_rng(32)
    du = _gpu(torch, wl.smooth_grid(list(w.n), 33))
    dc = rng.standard_normal(c.shape[0]) / (1.0 + np.arange(c.shape[0]))
    eps = 1e-6
    fd_u = (loss(eps * du, 0 * dc) - loss(-eps * du, 0 * dc)) / (2 * eps)
    fd_c = (loss(0 * du, eps * dc) - loss(0 * du, -eps * dc)) / (2 * eps)
    ad_u = float((gu * du).sum())
    ad_c = float(np.dot(gc, dc))
    print("fd_u %.12g ad_u %.12g fd_c %.12g ad_c %.12g" % (fd_u, ad_u, fd_c, ad_c), flush=True)
    assert abs(fd_u - ad_u) <= 1e-5 * abs(ad_u)
    assert abs(fd_c - ad_c) <= 1e-5 * abs(ad_c)


def test_config5_full_size_first_steps_vs_oracle(torch_dev, orc):
    """Full 1024^2 grid of the differentiation workload, 4 steps, two
    checkpoint segments, in the launch configuration the benchmark uses."""
    torch = torch_dev
    w, _ = wl.config5()
    steps = 4
    print_case("config5 oracle", w.n, steps)
    gT = np.random.default_rng(41).standard_normal(w.u0.shape)
    _, gu_ref, gc_ref = orc.adjoint(w.u0, w.tau, w.P, steps, w.basis, w.coef, gT)
    _, gu, gc, _ = _run_adjoint(torch, w.n, w.tau, w.P, w.basis, w.coef, w.u0, gT, steps, 2, "fast")
    assert _rel(gu, gu_ref) <= ADJ_TOL, _rel(gu, gu_ref)
    assert _rel(gc, gc_ref) <= ADJ_TOL, _rel(gc, gc_ref)


def test_autotuned_plan_same_gradients(torch_dev):
    """The launch-shape tuner leaves the forward values and the adjoint unchanged."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan
    n, tau, P, steps, every = (256, 192), 0.01, (0.3, 0.1), 24, 8
    basis = _basis(n, 6, 71)
    B = _gpu(torch, basis)
    coef = np.random.default_rng(72).standard_normal(6) * 0.5
    u0 = _gpu(torch, wl.smooth_grid(list(n), 73))
    gT = _gpu(torch, np.random.default_rng(74).standard_normal(u0.shape))
    res = []
    for tune in (False, True):
        p = Plan(n, tau, P, basis=B, coef=coef, method="fast", autotune=tune)
        u = u0.clone()
        ck = p.run(u, steps, 0, every)
        gu, gc = p.backward(ck, steps, every, gT)
        res.append((u.cpu().numpy(), gu.cpu().numpy(), gc))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])
    assert np.array_equal(res[0][2], res[1][2])


@pytest.mark.parametrize("method", ["brute", "fast"])
@pytest.mark.parametrize("case", [0, 2, 4])
def test_recorded_argmins_adjoint(torch_dev, orc, case, method):
    """Forward pass recording every step's argmins (lo_run_record), then the
    reverse pass without recomputation (lo_backward_recorded): the same
    forward result and the same gradients as the checkpointed adjoint, bit
    for bit, and the oracle's adjoint within the usual tolerance."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan
    n, tau, P, steps, every = CASES[case]
    print_case("recorded adjoint", n, steps, method)
    basis = _basis(n, 6, 100 + case)
    coef = np.random.default_rng(200 + case).standard_normal(basis.shape[0]) * 0.5
    u0 = wl.smooth_grid(list(n), 300 + case)
    gT = np.random.default_rng(400 + case).standard_normal(u0.shape)
    uT, gu, gc, _ = _run_adjoint(torch, n, tau, P, basis, coef, u0, gT, steps, every, method)
    p = Plan(n, tau, P, basis=_gpu(torch, basis), coef=coef, method=method)
    u = _gpu(torch, u0)
    E = p.run_record(u, steps)
    gu2, gc2 = p.backward_recorded(E, steps, _gpu(torch, gT))
    np.testing.assert_array_equal(u.cpu().numpy(), uT)
    np.testing.assert_array_equal(gu2.cpu().numpy(), gu)
    np.testing.assert_array_equal(gc2, gc)
    _, ogu, ogc = orc.adjoint(u0, tau, list(P), steps, basis, coef, gT)
    assert _rel(gu2.cpu().numpy(), ogu) <= ADJ_TOL
    assert _rel(gc2, ogc) <= ADJ_TOL


def test_recorded_argmins_autograd(torch_dev):
    """LaxOleinik with ckpt_every = 0 (recorded argmins) gives the
    checkpointed gradients."""
    torch = torch_dev
    from paper_1210_4090_amd.lo import Plan, LaxOleinik
    n, tau, P, steps = (48, 40), 0.04, (0.2, -0.1), 16
    basis = _gpu(torch, _basis(n, 6, 150))
    grads = []
    for every in (4, 0):
        p = Plan(n, tau, P, basis=basis, coef=np.zeros(6), method="fast")
        u0 = _gpu(torch, wl.smooth_grid(list(n), 151)).requires_grad_(True)
        coef = torch.tensor(np.random.default_rng(152).standard_normal(6) * 0.5, dtype=torch.float64,
                            requires_grad=True)
        uT = LaxOleinik.apply(u0, coef, p, steps, every)
        (uT * uT).sum().backward()
        grads.append((u0.grad.cpu().numpy(), coef.grad.cpu().numpy()))
    np.testing.assert_array_equal(grads[0][0], grads[1][0])
    np.testing.assert_array_equal(grads[0][1], grads[1][1])
