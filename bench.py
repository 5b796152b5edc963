#!/usr/bin/env python3
"""Benchmark of the fully discrete Lax--Oleinik step on one MI355X.

A bench "step" is one full run of the 2-D workload (2048^2 torus, P = (0.3,
0.1), V = cos2pi x + cos2pi y + 0.5 cos2pi(x+y), u0 = 8 seeded Fourier modes,
tau = 0.01, 1000 time steps): every time step is the row sweep, the column
sweep and the fused potential step, all in the library's HIP kernels.  u0 and
V are resident in HBM before the timed region.  Printed: one JSON line with
grid-point updates/s, the roofline of the dominant kernel (HIP events on the
kernels' stream), the CPU oracle's rate on a bounded sample, and secondary
measurements (brute vs fast, the 3-D workload, batched effective
Hamiltonians, forward + adjoint).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VALU_PEAK = 39.3e12       # non-FMA FP64 lane ops/s: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_bytes(ndim: int, npts: int):
    """Algorithmic HBM bytes per launch of each axis sweep: read u, write u
    (16 B/point), plus the tau*V table (8 B/point) in the last axis."""
    return [npts * (16 + (8 if a == ndim - 1 else 0)) for a in range(ndim)]


# kernel that sweeps axis a of the 2-D headline workload on the fast path
FAST_2D_KERNELS = {0: "k_claim_row<0,0,8,256,false>", 1: "k_claim_tile<1,0,16,false,256,16>"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "claim_sweeps_2d_2048sq_hbm_traffic.txt")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernel sources have
    changed since the counters were taken."""
    import hashlib
    if kernel is None or not os.path.exists(TRAFFIC_FILE):
        return None
    vals, srcs, digest = {}, [], None
    for line in open(TRAFFIC_FILE):
        if line.startswith("traffic_bytes_per_launch "):
            k, v = line[len("traffic_bytes_per_launch "):].rsplit(":", 1)
            vals[k.strip()] = float(v)
        elif line.startswith("kernel_source_sha256:"):
            digest = line.split(":", 1)[1].strip()
        elif line.startswith("kernel_sources:"):
            srcs = line.split(":", 1)[1].split()
    h = hashlib.sha256()
    for f in srcs:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if not srcs or h.hexdigest() != digest:
        return None
    return vals.get(kernel)


def timed_runs(torch, plan, u0, steps, K, W):
    u = torch.empty_like(u0)
    for _ in range(W):
        u.copy_(u0)
        plan.run(u, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        u.copy_(u0)
        plan.run(u, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, u


def measure_workload(torch, w, method, K, W, steps=None, autotune=False):
    from paper_1210_4090_amd.lo import Plan
    steps = w.steps if steps is None else steps
    V = torch.as_tensor(w.V, device="cuda")
    u0 = torch.as_tensor(w.u0, device="cuda")
    plan = Plan(w.n, w.tau, w.P, V=V, method=method, autotune=autotune)
    dt, u = timed_runs(torch, plan, u0, steps, K, W)
    rate = w.npts * steps * K / dt
    # per-kernel durations over one full run from u0, HIP events on the stream
    u.copy_(u0)
    ms = plan.time_kernels(u, steps)
    wins, _ = plan.diag()
    nb = sweep_bytes(w.ndim, w.npts)
    dom = int(max(range(w.ndim), key=lambda a: ms[a]))
    gbs = nb[dom] / (ms[dom] * 1e-3) / 1e9
    return {"rate": rate, "dt": dt, "ms_per_run": dt / K * 1e3, "kernel_ms": [float(x) for x in ms],
            "dominant_axis": dom, "dominant_GBs": gbs, "bytes_per_launch": nb[dom],
            "all_axis_GBs": [nb[a] / (ms[a] * 1e-3) / 1e9 for a in range(w.ndim)],
            "window_max": wins, "plan": plan, "V": V, "u0": u0}


def brute_valu(torch, w, plan, V, u0):
    """FP64 VALU work of the brute sweeps over one run: every step's windows
    (read back after each step) give 2 (2 W + 1) lane operations per point and
    axis (one add and one min per candidate)."""
    u = u0.clone()
    ops = 0.0
    for n in range(w.steps):
        plan.run(u, 1, n0=n)
        wins, _ = plan.diag()
        ops += sum(2.0 * (2 * W + 1) for W in wins) * w.npts
    return ops


def copy_ceiling(torch, mib=1024, reps=20):
    """A plain device copy of `mib` MiB (read and write: twice the 256 MB
    last-level cache), timed with HIP events: the practical HBM ceiling."""
    n = mib * (1 << 20) // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return {"bytes_per_copy": 2 * n * 8, "us_per_copy": ms * 1e3, "GBs": 2 * n * 8 / (ms * 1e-3) / 1e9,
            "how": "torch copy_ of %d MiB (read + write), mean of %d" % (mib, reps)}


def measure_adjoint(torch, method, every=50, reps=2, autotune=False, record=False):
    """Differentiation workload (1024^2, 500 steps, 64 Fourier modes of V):
    forward with FP64 checkpoints every `every` steps, then the reverse pass
    (segment recompute with int16 argmins, reverse sweeps, projection); with
    record, the forward pass keeps every step's argmins instead (2 GB here)
    and the reverse pass recomputes nothing."""
    import numpy as np
    from paper_1210_4090_amd import workloads as wl
    from paper_1210_4090_amd.lo import Plan
    w, _ = wl.config5()
    B = torch.as_tensor(w.basis, device="cuda")
    plan = Plan(w.n, w.tau, w.P, basis=B, coef=w.coef, method=method, autotune=autotune)
    u0 = torch.as_tensor(w.u0, device="cuda")
    gT = torch.as_tensor(np.random.default_rng(5).standard_normal(w.u0.shape), device="cuda")
    u = torch.empty_like(u0)
    best = None
    for _ in range(reps + 1):
        u.copy_(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ck = plan.run_record(u, w.steps) if record else plan.run(u, w.steps, 0, every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if record:
            plan.backward_recorded(ck, w.steps, gT)
        else:
            plan.backward(ck, w.steps, every, gT)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if best is None or t2 - t0 < best[0] + best[1]:
            best = (t1 - t0, t2 - t1)
        del ck
    fwd, bwd = best
    return {"forward_ms": fwd * 1e3, "backward_ms": bwd * 1e3,
            "fwd_adjoint_updates_per_s": w.npts * w.steps / (fwd + bwd),
            "checkpoint_every": 0 if record else every, "recorded_argmins": bool(record),
            "nmodes": int(w.basis.shape[0])}


def measure_hbar(torch, method, subset=None):
    """Batched effective Hamiltonians (512 instances, sides 256..1024,
    tau = 0.02, T = 20): the batched library call over the whole set, and
    one plan per instance run back to back over the first `subset` instances
    (all by default)."""
    import numpy as np
    from paper_1210_4090_amd import workloads as wl
    from paper_1210_4090_amd.lo import Plan, effective_H
    bw = wl.config4()
    Vd = {int(s): torch.as_tensor(v, device="cuda") for s, v in bw.V_by_side.items()}
    steps = int(round(bw.T / bw.tau))
    per_unit = int(round(1.0 / bw.tau))
    pts = bw.sides.astype(np.float64) ** 2

    def batched(idx):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        effective_H(bw.sides[idx], bw.P[idx], Vd, bw.tau, bw.T, method=method)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    all_idx = np.arange(bw.ninst)
    subset = bw.ninst if subset is None else subset
    sub = all_idx[:subset]
    batched(all_idx[:8])              # warm-up (code objects, allocator)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = effective_H(bw.sides, bw.P, Vd, bw.tau, bw.T, method=method)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    t_sub = t_all if subset == bw.ninst else batched(sub)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in sub:
        s = int(bw.sides[i])
        p = Plan([s, s], bw.tau, bw.P[i], V=Vd[s], method=method)
        u = torch.zeros((s, s), dtype=torch.float64, device="cuda")
        p.run(u, steps - per_unit)
        snap = u.clone()
        p.run(u, per_unit, n0=steps - per_unit)
        float((u - snap).max())
        p.close()
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    # algorithmic bytes of every step of every instance: two sweeps of 16 B a
    # point and the tau V table (8 B a point), over the whole job's time
    step_bytes = float(sum(sweep_bytes(2, 1)))
    width = out[:, 2] - out[:, 0]
    vmax = np.array([bw.V_by_side[int(s)].max() for s in bw.sides])
    return {"instances": bw.ninst, "steps": steps, "total_points": float(pts.sum()),
            "bracket_width": {"max": float(width.max()), "median": float(np.median(width)),
                              "p90": float(np.quantile(width, 0.9)), "min": float(width.min())},
            "max_abs_mid_minus_maxV": float(np.max(np.abs(out[:, 1] - vmax))),
            "batched_s": t_all, "hbar_per_s": bw.ninst / t_all,
            "updates_per_s": float(pts.sum()) * steps / t_all,
            "effective_GBs_whole_job": float(pts.sum()) * steps * step_bytes / t_all / 1e9,
            "hbm_frac_whole_job": float(pts.sum()) * steps * step_bytes / t_all / 1e9 / HBM_PEAK_GBS,
            "per_instance_loop_instances": int(subset), "per_instance_loop_batched_s": t_sub,
            "per_instance_loop_s": t_loop, "speedup_batched_vs_loop": t_loop / t_sub}


def hbar_batched_only(torch, method, steps):
    """The batched call alone over `steps` steps (a whole number of time
    units, for profiling)."""
    from paper_1210_4090_amd import workloads as wl
    from paper_1210_4090_amd.lo import effective_H
    bw = wl.config4()
    T = steps * bw.tau
    Vd = {int(s): torch.as_tensor(v, device="cuda") for s, v in bw.V_by_side.items()}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    effective_H(bw.sides, bw.P, Vd, bw.tau, T, method=method)
    torch.cuda.synchronize()
    return {"instances": bw.ninst, "steps": steps, "batched_s": time.perf_counter() - t0}


def measure_hbar_autotuned(torch):
    """The batched effective-Hamiltonian call with and without the launch-shape
    tuner, timed in alternation (a first tuned call tunes every batch and keeps
    the choices for the process); best of two each."""
    from paper_1210_4090_amd import workloads as wl
    from paper_1210_4090_amd.lo import effective_H
    bw = wl.config4()
    Vd = {int(s): torch.as_tensor(v, device="cuda") for s, v in bw.V_by_side.items()}
    effective_H(bw.sides, bw.P, Vd, bw.tau, bw.T, autotune=True)
    best = {"default_s": float("inf"), "tuned_s": float("inf")}
    for order in ((("default_s", False), ("tuned_s", True)), (("tuned_s", True), ("default_s", False))):
        for key, at in order:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            effective_H(bw.sides, bw.P, Vd, bw.tau, bw.T, autotune=at)
            torch.cuda.synchronize()
            best[key] = min(best[key], time.perf_counter() - t0)
    return best


def compare_tuned(measure):
    """measure(autotune) with fresh plans, default and tuned in alternation,
    best of two each.  A plan's speed depends slightly on where its arrays
    land: the first plan of a workload's size in a process can land in memory
    no plan has used and run a few percent faster than those after it (the
    256^3 row sweep 57 against 61 us), so a throwaway plan takes that place,
    and the two rounds take the shapes in opposite orders."""
    measure(False)
    best = {}
    for order in ((("default", False), ("tuned", True)), (("tuned", True), ("default", False))):
        for key, at in order:
            r = measure(at)
            if key not in best or r["ms"] < best[key]["ms"]:
                best[key] = r
    return best


# The paper's one timing (Section 5.1): the pendulum on 2^18 points to T = 8 in
# about 19 minutes of MATLAB on a 2.3 GHz Core i7 laptop, with its approximate
# decomposition (tolerance eta = h).  Context only: other hardware, other method.
PAPER_PENDULUM_S = 19 * 60.0


def measure_paper_pendulum(torch, method, K=2 ** 17, reps=None):
    """The paper's pendulum (Section 5.1) on 2K points to T = 8 (tau about
    sqrt(h)), the run timed on the device; best of `reps`."""
    from paper_1210_4090_amd import workloads as wl
    from paper_1210_4090_amd.lo import Plan
    w = wl.pendulum(K)
    p = Plan(w.n, w.tau, w.P, period=w.period, V=torch.as_tensor(w.V, device="cuda"), method=method)
    u0 = torch.as_tensor(w.u0, device="cuda")
    best = None
    reps = reps if reps is not None else (3 if method == "fast" else 1)
    for _ in range(reps + 1):   # the first run warms up
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.run(u, w.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None or dt < best else best
    p.close()
    return {"grid_points": w.npts, "steps": w.steps, "tau": w.tau, "ms_per_run": best * 1e3,
            "updates_per_s": w.npts * w.steps / best, "paper_reported_s": PAPER_PENDULUM_S,
            "paper_setting": "MATLAB, 2.3 GHz Intel Core i7 laptop, approximate decomposition eta = h"}


def measure_decomposition(torch, K=2 ** 13, etas=(0.0, 0.01, 1.0)):
    """The paper's own algorithm (Section 4; lo_run_decomp) on the pendulum
    with 2K points to T = 8, for tolerances eta (on slope increments; eta = 1
    is the paper's eta = h on raw increments), against the exact claim path:
    device time, pieces and convex/concave breaks per step, relative error."""
    import numpy as np
    from paper_1210_4090_amd import workloads as wl
    from paper_1210_4090_amd.lo import Plan
    w = wl.pendulum(K)
    p = Plan(w.n, w.tau, w.P, period=w.period, V=torch.as_tensor(w.V, device="cuda"), method="fast")
    u0 = torch.as_tensor(w.u0, device="cuda")

    def timed(fn):
        u = u0.clone()
        fn(u, 2)                  # warm-up
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn(u, w.steps)
        torch.cuda.synchronize()
        return u, time.perf_counter() - t0, r

    exact, tc, _ = timed(lambda u, k: p.run(u, k))
    window = p.diag()[0][0] + 2
    ex = exact.cpu().numpy()
    runs = []
    for eta in etas:
        u, dt, (pieces, breaks) = timed(lambda u, k, e=eta: p.run_decomp(u, k, eta=e, window=window))
        runs.append({"eta": eta, "ms_per_run": dt * 1e3, "pieces_per_step": pieces / w.steps,
                     "breaks_per_step": breaks / w.steps,
                     "max_rel_err_vs_exact": float(np.max(np.abs(u.cpu().numpy() - ex)) / np.max(np.abs(ex)))})
    p.close()
    return {"grid_points": w.npts, "steps": w.steps, "window": int(window), "claim_path_ms": tc * 1e3,
            "decomposition": runs}


def cpu_baseline(w, nsteps=30):
    from oracle import oracle
    t0 = time.perf_counter()
    oracle.run(w.u0, w.tau, w.P, nsteps, V=w.V)
    dt = time.perf_counter() - t0
    return {"value": w.npts * nsteps / dt, "unit": "grid-point updates/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": "first %d time steps of the %s workload, full grid (%.1f s)"
            % (nsteps, w.name, dt)}


def _only_run(torch, w, method, steps):
    """One run of `steps` steps of the workload from its u0 (for profiling)."""
    from paper_1210_4090_amd.lo import Plan
    V = torch.as_tensor(w.V, device="cuda")
    plan = Plan(w.n, w.tau, w.P, V=V, method=method)
    u = torch.as_tensor(w.u0, device="cuda").clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(u, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": w.name, "steps": steps, "ms_per_run": dt * 1e3, "updates_per_s": w.npts * steps / dt}


def _only_3d(torch, method, steps=None):
    from paper_1210_4090_amd import workloads as wl
    w = wl.config3()
    if steps:
        return _only_run(torch, w, method, steps)
    m = measure_workload(torch, w, method, 2, 1)
    return {"updates_per_s": m["rate"], "ms_per_run": m["ms_per_run"], "kernel_ms": m["kernel_ms"],
            "all_axis_GBs": m["all_axis_GBs"]}


def _only_2d(torch, method, steps=None):
    from paper_1210_4090_amd import workloads as wl
    w = wl.config2()
    return _only_run(torch, w, method, steps or w.steps)


# one secondary workload at a time (python bench.py --only NAME [--run-steps N]), for profiling runs
ONLY = {
    "2d": _only_2d,
    "3d": _only_3d,
    "copy": lambda torch, method, steps=None: copy_ceiling(torch),
    "hbar": lambda torch, method, steps=None: measure_hbar(torch, method) if not steps else hbar_batched_only(
        torch, method, steps),
    "adjoint": lambda torch, method, steps=None: measure_adjoint(torch, method, reps=1),
    "adjoint_recorded": lambda torch, method, steps=None: measure_adjoint(torch, method, reps=1, record=True),
    "pendulum": lambda torch, method, steps=None: measure_paper_pendulum(torch, method, reps=1),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--method", default="fast", choices=["fast", "brute"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="only the headline workload")
    ap.add_argument("--only", choices=sorted(ONLY), default=None,
                    help="measure one workload and print its figures (for profiling runs); no "
                         "headline line")
    ap.add_argument("--run-steps", type=int, default=None,
                    help="with --only 2d / 3d: one run of this many steps from u0; with --only hbar: the "
                         "batched call alone over this many steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1210_4090_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.only:
        print(json.dumps({"workload": args.only, "figures": ONLY[args.only](torch, args.method, args.run_steps)}),
              flush=True)
        return
    w = wl.config2()
    log("workload %s steps=%d method=%s K=%d W=%d" % (w.name, w.steps, args.method, args.steps, args.warmup))
    m = measure_workload(torch, w, args.method, args.steps, args.warmup)
    log("headline: %.4g updates/s, %.2f ms per run, kernels %s ms, windows %s"
        % (m["rate"], m["ms_per_run"], m["kernel_ms"], m["window_max"]))
    kname = FAST_2D_KERNELS.get(m["dominant_axis"]) if args.method == "fast" else None
    traffic = measured_traffic(kname)
    ceil = copy_ceiling(torch)
    log("copy ceiling: %.1f GB/s" % ceil["GBs"])
    out = {
        "metric": "grid-point min-plus updates/sec + HBM GB/s, plain vs batched H̄(P) vs fwd+adjoint",
        "value": m["rate"],
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_run"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Fourier modes)",
        "config": {"workload": "2d_torus_2048x2048_tau0.01_1000steps", "grid": [2048, 2048],
                   "time_steps_per_run": w.steps, "method": args.method, "P": list(w.P),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": m["dominant_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": m["dominant_GBs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "axis-%d sweep %s" % (m["dominant_axis"], kname or ""),
                     "algorithmic_bytes_per_launch": m["bytes_per_launch"],
                     "kernel_ms": m["kernel_ms"],
                     "timing": "mean interval of a HIP event pair around each launch, on the plan's stream, "
                               "over one full run (never below the kernel's own duration)",
                     "copy_ceiling_GBs": ceil["GBs"], "frac_of_copy_ceiling": m["dominant_GBs"] / ceil["GBs"]},
        "effective_GBs_whole_step": sum(sweep_bytes(w.ndim, w.npts)) * w.steps / (m["ms_per_run"] * 1e-3) / 1e9,
        "hbm_copy_ceiling": ceil,
    }
    if not args.no_extras:
        extras = {}
        other = "brute" if args.method == "fast" else "fast"
        mb = measure_workload(torch, w, other, 1, 0)
        extras["headline_workload_" + other] = {"updates_per_s": mb["rate"], "ms_per_run": mb["ms_per_run"],
                                               "kernel_ms": mb["kernel_ms"], "window_max": mb["window_max"]}
        bm = mb if other == "brute" else m
        ops = brute_valu(torch, w, bm["plan"], bm["V"], bm["u0"])
        extras["headline_workload_brute_valu"] = {
            "lane_ops_per_run": ops, "ops_per_s": ops / (bm["ms_per_run"] * 1e-3),
            "peak_ops_per_s": FP64_VALU_PEAK, "frac": ops / (bm["ms_per_run"] * 1e-3) / FP64_VALU_PEAK,
            "count": "2 (2W + 1) FP64 add/min lane operations per point and axis, W each step's window"}
        log("%s: %.4g updates/s; brute VALU %s" % (other, mb["rate"], extras["headline_workload_brute_valu"]))
        del mb, bm
        w3 = wl.config3()
        m3 = measure_workload(torch, w3, args.method, 2, 1)
        whole3 = sum(sweep_bytes(w3.ndim, w3.npts)) * w3.steps / (m3["ms_per_run"] * 1e-3) / 1e9
        extras["3d_torus_256^3_200steps"] = {
            "updates_per_s": m3["rate"], "ms_per_run": m3["ms_per_run"], "kernel_ms": m3["kernel_ms"],
            "all_axis_GBs": m3["all_axis_GBs"], "hbm_frac_dominant": m3["dominant_GBs"] / HBM_PEAK_GBS,
            "effective_GBs_whole_run": whole3, "hbm_frac_whole_run": whole3 / HBM_PEAK_GBS,
            "frac_of_copy_ceiling_whole_run": whole3 / ceil["GBs"], "window_max": m3["window_max"]}
        log("3-D: %.4g updates/s, axis GB/s %s" % (m3["rate"], m3["all_axis_GBs"]))
        del m3
        extras["batched_hbar_512"] = measure_hbar(torch, args.method)
        extras["batched_hbar_512"]["frac_of_copy_ceiling_whole_job"] = \
            extras["batched_hbar_512"]["effective_GBs_whole_job"] / ceil["GBs"]
        log("batched hbar: %s" % extras["batched_hbar_512"])
        extras["fwd_adjoint_1024^2_500steps"] = measure_adjoint(torch, args.method)
        extras["fwd_adjoint_1024^2_500steps_recorded_argmins"] = measure_adjoint(torch, args.method, record=True)
        log("fwd+adjoint, recorded argmins: %s" % extras["fwd_adjoint_1024^2_500steps_recorded_argmins"])
        extras["paper_pendulum_2^18"] = measure_paper_pendulum(torch, args.method)
        log("paper pendulum: %s" % extras["paper_pendulum_2^18"])
        extras["paper_decomposition_pendulum_2^14"] = measure_decomposition(torch)
        log("paper decomposition: %s" % extras["paper_decomposition_pendulum_2^14"])
        if args.method == "fast":
            # default against tuned, each pair measured side by side
            def run2(wk, at):
                m = measure_workload(torch, wk, "fast", 2, 1, autotune=at)
                return {"ms": m["ms_per_run"], "updates_per_s": m["rate"], "kernel_ms": m["kernel_ms"]}

            def adj(at):
                r = measure_adjoint(torch, "fast", autotune=at)
                r["ms"] = r["forward_ms"] + r["backward_ms"]
                return r

            extras["headline_workload_autotuned"] = compare_tuned(lambda at: run2(w, at))
            extras["3d_torus_256^3_200steps_autotuned"] = compare_tuned(lambda at: run2(w3, at))
            extras["fwd_adjoint_1024^2_500steps_autotuned"] = compare_tuned(adj)
            extras["batched_hbar_512_autotuned"] = measure_hbar_autotuned(torch)
            log("autotuned: %s" % {k: v for k, v in extras.items() if "autotuned" in k})
        log("fwd+adjoint: %s" % extras["fwd_adjoint_1024^2_500steps"])
        out["extras"] = extras
    if not args.no_cpu:
        cb = cpu_baseline(w)
        log("cpu oracle: %.4g updates/s on %d threads" % (cb["value"], cb["cores"]))
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
