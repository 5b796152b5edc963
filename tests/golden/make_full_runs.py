"""Writes the oracle's results for the full-length parity tests.

The FP64 CPU oracle (oracle/, the definition written out: Section 2.3,
eq. eqconvol, split as in Remark rk28, composed as in eq. uN; its adjoint
is the derivative of eq. uN) takes minutes to hours on these grids, too long
for a GPU test, so its results are stored here once: at 8192 seeded sample
points of the final field (plus the whole first line along axis 0), with the
field's max-norm.  Nothing here comes from the GPU path: only oracle/ and the
seeded input generators of workloads.py are called.

    python tests/golden/make_full_runs.py [name ...]

writes tests/golden/<name>.npz for each run (all by default).  The oracle's
result does not depend on its thread count (rows are independent and each
is evaluated in a fixed order).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_1210_4090_amd import workloads as wl  # noqa: E402

NSAMPLE = 8192


def sample_index(shape, seed):
    """Seeded flat indices: NSAMPLE random points and the first line along axis 0."""
    npts = int(np.prod(shape))
    rnd = np.random.default_rng(seed).choice(npts, size=min(NSAMPLE, npts), replace=False)
    line = np.arange(shape[-1], dtype=np.int64)
    return np.unique(np.concatenate([rnd.astype(np.int64), line]))


def forward(w, steps, seed):
    t0 = time.time()
    u = oracle.run(w.u0, w.tau, w.P, steps, V=w.V)
    idx = sample_index(u.shape, seed)
    return dict(idx=idx, val=u.reshape(-1)[idx], absmax=np.max(np.abs(u)), steps=steps,
                grid=np.array(w.n, dtype=np.int64), seconds=time.time() - t0)


def c3_200():
    """The 3-D workload (256^3, tau = 0.02), all 200 steps."""
    return forward(wl.config3(), 200, 3001)


def c2_2048x1280_400():
    """The 2-D workload's data on a 2048 x 1280 grid, 400 steps (the windows
    settle within the first 30)."""
    return forward(wl.config2(2048, n1=1280), 400, 3002)


def c2_2048sq_30():
    """The 2-D workload at full size (2048^2), its first 30 steps."""
    return forward(wl.config2(), 30, 3003)


def c5_adjoint_50():
    """The differentiation workload (1024^2, 64 potential modes): one 50-step
    segment, the loss gradient seeded N(0, 1).  Stores u(50), dL/du0 at the
    sample points and the whole coefficient gradient."""
    t0 = time.time()
    w, _ = wl.config5()
    steps = 50
    gT = np.random.default_rng(5050).standard_normal(w.u0.shape)
    uT, gu, gc = oracle.adjoint(w.u0, w.tau, w.P, steps, w.basis, w.coef, gT)
    idx = sample_index(uT.shape, 3005)
    return dict(idx=idx, val=uT.reshape(-1)[idx], absmax=np.max(np.abs(uT)), gu=gu.reshape(-1)[idx],
                gu_absmax=np.max(np.abs(gu)), gc=gc, steps=steps, grad_seed=5050,
                grid=np.array(w.n, dtype=np.int64), seconds=time.time() - t0)


def c4_inst_1024_100():
    """The first side-1024 instance of the batched effective-Hamiltonian
    workload (u0 = 0, its P, V as the 2-D workload, tau = 0.02): 100 steps."""
    t0 = time.time()
    bw = wl.config4()
    i = int(np.flatnonzero(bw.sides == 1024)[0])
    steps = 100
    u = oracle.run(np.zeros((1024, 1024)), bw.tau, bw.P[i], steps, V=bw.V_by_side[1024])
    idx = sample_index(u.shape, 3004)
    return dict(idx=idx, val=u.reshape(-1)[idx], absmax=np.max(np.abs(u)), steps=steps, instance=i,
                grid=np.array([1024, 1024], dtype=np.int64), seconds=time.time() - t0)


RUNS = {f.__name__: f for f in (c2_2048sq_30, c5_adjoint_50, c4_inst_1024_100, c2_2048x1280_400, c3_200)}


def main(names):
    for name in names or list(RUNS):
        print("oracle run %s on %d threads" % (name, oracle.num_threads()), flush=True)
        res = RUNS[name]()
        np.savez(os.path.join(HERE, name + ".npz"), **{k: np.asarray(v) for k, v in res.items()})
        print("  wrote %s.npz (%.0f s)" % (name, res["seconds"]), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
