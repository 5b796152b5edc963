"""Seeded synthetic inputs for the fully discrete Lax--Oleinik scheme.

This module only *draws* inputs: grids, initial data u0, potential samples V on
the grid, Fourier basis tables and rotation vectors P.  It holds none of the
scheme's arithmetic (no kinetic cost, no min-plus, no potential step), so both
the HIP path and the CPU oracle may consume what it produces.

The workloads follow the paper's setting: a mechanical Hamiltonian
H = |p + P|^2 / 2 + V on a periodic grid (Section 1, eq. HPV; Section 3,
hypothesis (iii)), with smooth periodic V given by a few Fourier modes and the
experiments' analytic data (Section 5).  The paper measures on no public data
set; everything here is synthetic.

Conventions: a grid has `ndim` axes, axis 0 varies fastest in memory, axis a
has n[a] points x_a = i_a * period[a] / n[a].  Arrays are float64, shape
(n[ndim-1], ..., n[0]) in numpy order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------
# Fourier fields on the grid
# ----------------------------------------------------------------------------
def _axis_phases(n: Sequence[int], period: Sequence[float]) -> List[np.ndarray]:
    """x_a / period_a for every axis a (float64, length n[a])."""
    return [np.arange(na, dtype=np.float64) / float(na) for na in n]


def fourier_field(n: Sequence[int], kvecs: np.ndarray, amps: np.ndarray,
                  phases: np.ndarray, period: Optional[Sequence[float]] = None,
                  kind: Optional[Sequence[str]] = None) -> np.ndarray:
    """sum_m amps[m] * cos(2 pi k_m . x / period + phases[m]) on the grid.

    kvecs: (M, ndim) integer wave vectors (component a pairs with axis a).
    kind: optional per-mode 'cos' or 'sin' (sin(theta) = cos(theta - pi/2)).
    Evaluated through per-axis complex exponentials (separable factors).
    """
    n = list(n)
    ndim = len(n)
    if period is None:
        period = [1.0] * ndim
    kvecs = np.asarray(kvecs, dtype=np.int64).reshape(-1, ndim)
    amps = np.asarray(amps, dtype=np.float64).reshape(-1)
    phases = np.asarray(phases, dtype=np.float64).reshape(-1)
    xs = _axis_phases(n, period)
    shape = tuple(reversed(n))
    out = np.zeros(shape, dtype=np.float64)
    for m in range(kvecs.shape[0]):
        ph = phases[m]
        if kind is not None and kind[m] == "sin":
            ph = ph - 0.5 * math.pi
        acc = np.exp(1j * ph) * np.ones((1,) * ndim, dtype=np.complex128)
        for a in range(ndim):
            fac = np.exp(1j * TWO_PI * kvecs[m, a] * xs[a])
            sh = [1] * ndim
            sh[ndim - 1 - a] = n[a]
            acc = acc * fac.reshape(sh)
        out += amps[m] * np.real(acc)
    return out


def wave_vectors(ndim: int, kmax: float) -> np.ndarray:
    """All k in Z^ndim with 0 < |k| <= kmax, in lexicographic order."""
    r = int(math.floor(kmax))
    rng = range(-r, r + 1)
    ks = []
    for k in np.array(np.meshgrid(*([list(rng)] * ndim), indexing="ij")).reshape(ndim, -1).T:
        q = float(np.dot(k, k))
        if 0 < q <= kmax * kmax + 1e-12:
            ks.append(tuple(int(v) for v in k))
    ks.sort()
    return np.array(ks, dtype=np.int64)


def random_modes(ndim: int, count: int, kmax: float, rng: np.random.Generator
                 ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """`count` wave vectors drawn without replacement from 0<|k|<=kmax,
    amplitude 1/|k|^2, uniform phase in [0, 2 pi)."""
    ks = wave_vectors(ndim, kmax)
    idx = rng.choice(ks.shape[0], size=count, replace=False)
    kv = ks[np.sort(idx)]
    amp = 1.0 / np.sum(kv.astype(np.float64) ** 2, axis=1)
    ph = rng.uniform(0.0, TWO_PI, size=count)
    return kv, amp, ph


def half_plane_basis(count_k: int) -> Tuple[np.ndarray, List[str]]:
    """First `count_k` 2-D wave vectors of the half plane (k1 > 0, or k1 == 0
    and k2 > 0), sorted by (|k|^2, k1, k2); each gives a cos and a sin mode.
    Returns (kvecs (2*count_k, 2), kinds)."""
    cands = []
    r = 8
    for k1 in range(0, r + 1):
        for k2 in range(-r, r + 1):
            if k1 > 0 or (k1 == 0 and k2 > 0):
                cands.append((k1 * k1 + k2 * k2, k1, k2))
    cands.sort()
    ks = [(c[1], c[2]) for c in cands[:count_k]]
    kv, kinds = [], []
    for k in ks:
        kv.append(k)
        kinds.append("cos")
        kv.append(k)
        kinds.append("sin")
    return np.array(kv, dtype=np.int64), kinds


def basis_tables(n: Sequence[int], kvecs: np.ndarray, kinds: Sequence[str]) -> np.ndarray:
    """phi_m on the grid, shape (M, *grid_shape), phi = cos or sin of 2 pi k.x."""
    M = kvecs.shape[0]
    out = np.empty((M,) + tuple(reversed(list(n))), dtype=np.float64)
    for m in range(M):
        out[m] = fourier_field(n, kvecs[m:m + 1], np.ones(1), np.zeros(1), kind=[kinds[m]])
    return out


# ----------------------------------------------------------------------------
# Workload descriptions
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    """One synthetic problem: grid, time step, rotation vector, u0 and V."""
    name: str
    n: Tuple[int, ...]
    tau: float
    P: Tuple[float, ...]
    steps: int
    u0: np.ndarray
    V: np.ndarray
    period: Tuple[float, ...] = None
    basis: Optional[np.ndarray] = None      # (M, *grid) Fourier basis, if V = sum c_m phi_m
    coef: Optional[np.ndarray] = None       # (M,) coefficients of V in that basis
    tcoef: Optional[np.ndarray] = None      # (steps, M): V(t_n) = sum_m tcoef[n, m] phi_m

    def __post_init__(self):
        if self.period is None:
            self.period = tuple([1.0] * len(self.n))

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def npts(self) -> int:
        return int(np.prod(self.n))


def _c2_potential(n: Sequence[int]) -> np.ndarray:
    kv = np.array([[1, 0], [0, 1], [1, 1]])
    return fourier_field(n, kv, np.array([1.0, 1.0, 0.5]), np.zeros(3))


def config1(n: int = 256, steps: int = 200) -> Workload:
    """1-D torus, P = 0, V = cos 2 pi x, u0 = sin 2 pi x, tau = 0.05."""
    V = fourier_field([n], np.array([[1]]), np.ones(1), np.zeros(1))
    u0 = fourier_field([n], np.array([[1]]), np.ones(1), np.array([-0.5 * math.pi]))
    return Workload("1d_torus_n%d" % n, (n,), 0.05, (0.0,), steps, u0, V)


def config2(n: int = 2048, steps: int = 1000, seed: int = 2, n1: Optional[int] = None) -> Workload:
    """2-D torus, P = (0.3, 0.1), V = cos2pi x + cos2pi y + 0.5 cos2pi(x+y),
    u0 = 8 seeded Fourier modes |k| <= 4 with amplitude 1/|k|^2, tau = 0.01.
    The grid is n x n, or n points on axis 0 by n1 on axis 1."""
    rng = np.random.default_rng(seed)
    kv, amp, ph = random_modes(2, 8, 4.0, rng)
    shape = [n, n if n1 is None else int(n1)]
    u0 = fourier_field(shape, kv, amp, ph)
    return Workload("2d_torus_%dx%d" % tuple(shape), tuple(shape), 0.01, (0.3, 0.1), steps, u0,
                    _c2_potential(shape))


def config3(n: int = 256, steps: int = 200, seed: int = 3) -> Workload:
    """3-D torus, P = (0.2, -0.1, 0.05), u0 = 0, V = 16 seeded modes |k| <= 4
    with amplitude 1/|k|^2, tau = 0.02."""
    rng = np.random.default_rng(seed)
    kv, amp, ph = random_modes(3, 16, 4.0, rng)
    V = fourier_field([n, n, n], kv, amp, ph)
    return Workload("3d_torus_%d^3" % n, (n, n, n), 0.02, (0.2, -0.1, 0.05), steps,
                    np.zeros((n, n, n)), V)


# ----------------------------------------------------------------------------
# The paper's own experiments (Section 5): 1-D, period 2 pi, space step
# h = pi / K (2K points), time step about sqrt(h), final time T = 8.
# ----------------------------------------------------------------------------
def paper_time_step(h: float, T: float = 8.0) -> Tuple[float, int]:
    """A time step near sqrt(h) (the experiments' choice) that divides T, so
    runs on different grids end at the same time: tau = T / ceil(T / sqrt(h))."""
    steps = int(math.ceil(T / math.sqrt(h)))
    return T / steps, steps


def pendulum(K: int, T: float = 8.0) -> Workload:
    """Section 5.1: P = 0, V = 1 - cos x, u0 = cos x on the 2 pi torus with
    h = pi / K (2K grid points) and tau ~ sqrt(h), run to T."""
    n = 2 * K
    tau, steps = paper_time_step(math.pi / K, T)
    cosx = fourier_field([n], np.array([[1]]), np.ones(1), np.zeros(1))
    return Workload("pendulum_%d" % n, (n,), tau, (0.0,), steps, cosx.copy(), 1.0 - cosx,
                    period=(TWO_PI,))


def time_dependent(K: int, T: float = 8.0) -> Workload:
    """Section 5.2: P = 1, V(t, x) = cos 2x sin t, u0 = cos x, same grids and
    time steps as the pendulum.  V is given as one basis table (cos 2x) with
    the coefficient sin(t_n) at step n, t_n = n tau."""
    n = 2 * K
    tau, steps = paper_time_step(math.pi / K, T)
    cosx = fourier_field([n], np.array([[1]]), np.ones(1), np.zeros(1))
    basis = fourier_field([n], np.array([[2]]), np.ones(1), np.zeros(1))[None]
    tcoef = np.sin(tau * np.arange(steps, dtype=np.float64))[:, None]
    return Workload("time_dependent_%d" % n, (n,), tau, (1.0,), steps, cosx, None,
                    period=(TWO_PI,), basis=basis, tcoef=tcoef)


@dataclasses.dataclass
class BatchWorkload:
    """Many effective-Hamiltonian instances on uneven 2-D grids."""
    sides: np.ndarray          # (ninst,)
    P: np.ndarray              # (ninst, 2)
    tau: float
    T: float
    V_by_side: dict            # side -> V grid
    name: str = "batched_hbar"

    @property
    def ninst(self) -> int:
        return int(self.sides.shape[0])


def config4(ninst_p1: int = 32, ninst_p2: int = 16, sides=(256, 384, 512, 768, 1024),
            tau: float = 0.02, T: float = 20.0, seed: int = 4) -> BatchWorkload:
    """Batched effective Hamiltonian: P on a ninst_p1 x ninst_p2 grid in
    [-1, 1]^2, square sides drawn uniformly from `sides`, V as config2, u0 = 0."""
    rng = np.random.default_rng(seed)
    p1 = np.linspace(-1.0, 1.0, ninst_p1)
    p2 = np.linspace(-1.0, 1.0, ninst_p2)
    P = np.array([(a, b) for a in p1 for b in p2], dtype=np.float64)
    sd = rng.choice(np.asarray(sides, dtype=np.int64), size=P.shape[0], replace=True)
    Vs = {int(s): _c2_potential([int(s), int(s)]) for s in np.unique(sd)}
    return BatchWorkload(sd, P, tau, T, Vs, name="batched_hbar_%d" % P.shape[0])


def config5(n: int = 1024, steps: int = 500, nk: int = 32, seed_u0: int = 5,
            seed_star: int = 55, seed_eval: int = 56):
    """Differentiation workload: V = sum_m c_m phi_m over the first `nk`
    half-plane wave vectors (cos and sin each), hidden c* ~ N(0,1)/|k|^2,
    evaluation point c = c* + 0.3 N(0,1)/|k|^2, u0 as config2, tau = 0.01,
    P = (0.3, 0.1).  Returns (workload at c, c_star)."""
    kv, kinds = half_plane_basis(nk)
    k2 = np.sum(kv.astype(np.float64) ** 2, axis=1)
    c_star = np.random.default_rng(seed_star).standard_normal(kv.shape[0]) / k2
    c = c_star + 0.3 * np.random.default_rng(seed_eval).standard_normal(kv.shape[0]) / k2
    basis = basis_tables([n, n], kv, kinds)
    rng = np.random.default_rng(seed_u0)
    ukv, uamp, uph = random_modes(2, 8, 4.0, rng)
    u0 = fourier_field([n, n], ukv, uamp, uph)
    w = Workload("2d_adjoint_%dx%d" % (n, n), (n, n), 0.01, (0.3, 0.1), steps, u0,
                 None, basis=basis, coef=c)
    return w, c_star


def random_grid(n: Sequence[int], seed: int, scale: float = 1.0) -> np.ndarray:
    """Uniform random values in [-scale, scale] on the grid (rough data)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=tuple(reversed(list(n))))


def smooth_grid(n: Sequence[int], seed: int, count: int = 6, kmax: float = 3.0) -> np.ndarray:
    """A seeded smooth periodic field (a few Fourier modes)."""
    rng = np.random.default_rng(seed)
    ndim = len(n)
    count = min(count, wave_vectors(ndim, kmax).shape[0])
    kv, amp, ph = random_modes(ndim, count, kmax, rng)
    return fourier_field(n, kv, amp, ph)
