"""ctypes front end of the FP64 CPU oracle (lo_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product package never does.

Every function follows the plain definition of the fully discrete
Lax--Oleinik scheme (Section 2.3, eq. eqconvol; Remark rk28 for the axis
splitting; eq. uN for the composition), or, for semigroup1_*, of the first
discrete semigroup (Section 2.2, eq. cost1); see lo_oracle.c for the exact
floating-point evaluation order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lo_oracle.c")
_LIB = os.path.join(_HERE, "liblo_oracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_sweep.argtypes = [ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, _f64p, ctypes.c_int64, _f64p, _f64p, _i32p]
        L.orc_step.argtypes = [ctypes.c_int, _i64p, _f64p, ctypes.c_double, _f64p,
                               ctypes.POINTER(_f64p), _i64p, _f64p, _f64p, _i32p]
        L.orc_run.argtypes = [ctypes.c_int, _i64p, _f64p, ctypes.c_double, _f64p,
                              ctypes.POINTER(_f64p), _i64p, _f64p, ctypes.c_int, _f64p, _f64p,
                              ctypes.c_int64, ctypes.c_int64, _f64p]
        L.orc_joint_step.argtypes = [ctypes.c_int, _i64p, _f64p, ctypes.c_double, _f64p, _f64p, _f64p]
        L.orc_potential.argtypes = [ctypes.c_int64, ctypes.c_int, _f64p, _f64p, _f64p]
        L.orc_adjoint.argtypes = [ctypes.c_int, _i64p, _f64p, ctypes.c_double, _f64p, ctypes.c_int64,
                                  _f64p, ctypes.c_int, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p]
        L.orc_num_threads.argtypes = []
        L.orc_semigroup1_step.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          _f64p, ctypes.c_int64, _f64p, _f64p, _f64p, _i32p]
        for f in ("orc_sweep", "orc_step", "orc_run", "orc_joint_step", "orc_potential",
                  "orc_adjoint", "orc_num_threads", "orc_semigroup1_step"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a):
    return a.ctypes.data_as(_f64p) if a is not None else None


def _dims(u: np.ndarray, ndim: Optional[int] = None):
    ndim = u.ndim if ndim is None else ndim
    n = np.array(list(reversed(u.shape[-ndim:])), dtype=np.int64)
    return ndim, n


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def grid_dx(n: Sequence[int], period: Optional[Sequence[float]] = None) -> np.ndarray:
    """dx_a = period_a / n_a, the grid step of each axis."""
    period = [1.0] * len(n) if period is None else period
    return np.array([float(p) / float(k) for p, k in zip(period, n)], dtype=np.float64)


def _ktabs(ktabs, ndim):
    if ktabs is None:
        return None, None, []
    keep = []
    ptrs = (_f64p * ndim)()
    half = np.zeros(ndim, dtype=np.int64)
    for a in range(ndim):
        t = ktabs[a]
        if t is None:
            ptrs[a] = _f64p()
        else:
            t = _c(t)
            keep.append(t)
            ptrs[a] = _f64(t)
            half[a] = (t.shape[0] - 1) // 2
    return ptrs, half, keep


def kinetic(s, dx: float, tau: float, P: float) -> np.ndarray:
    """tau * K*(s dx / tau) for L = v^2/2 - P v, in the oracle's evaluation order."""
    d = np.asarray(s, dtype=np.float64) * dx
    return ((0.5 * d) * d) / tau - P * d


def sweep(u: np.ndarray, axis: int, tau: float, P: float, period: float = 1.0,
          ktab: Optional[np.ndarray] = None):
    """One 1-D min-plus sweep along `axis` (0 = fastest).  Returns (w, argmin)."""
    u = _c(u)
    ndim, n = _dims(u)
    dx = float(period) / float(n[axis])
    w = np.empty_like(u)
    arg = np.empty(u.shape, dtype=np.int32)
    kt = None if ktab is None else _c(ktab)
    half = 0 if kt is None else (kt.shape[0] - 1) // 2
    rc = lib().orc_sweep(ndim, n.ctypes.data_as(_i64p), axis, dx, tau, P, _f64(kt), half,
                         _f64(u), _f64(w), arg.ctypes.data_as(_i32p))
    if rc:
        raise RuntimeError("orc_sweep failed: %d" % rc)
    return w, arg


def step(u: np.ndarray, tau: float, P: Sequence[float], V: Optional[np.ndarray] = None,
         period: Optional[Sequence[float]] = None, ktabs=None, with_argmin: bool = False):
    """One time step (all axis sweeps, then the potential step).  Returns u+
    (and the [ndim, *grid] int32 argmin offsets if asked)."""
    u = _c(u).copy()
    ndim, n = _dims(u)
    dx = grid_dx(n, period)
    Pp = _c(P)
    Vc = None if V is None else _c(V)
    ptrs, half, keep = _ktabs(ktabs, ndim)
    arg = np.empty((ndim,) + u.shape, dtype=np.int32) if with_argmin else None
    rc = lib().orc_step(ndim, n.ctypes.data_as(_i64p), _f64(dx), tau, _f64(Pp), ptrs,
                        None if half is None else half.ctypes.data_as(_i64p), _f64(Vc), _f64(u),
                        None if arg is None else arg.ctypes.data_as(_i32p))
    if rc:
        raise RuntimeError("orc_step failed: %d" % rc)
    return (u, arg) if with_argmin else u


def run(u0: np.ndarray, tau: float, P: Sequence[float], nsteps: int, V: Optional[np.ndarray] = None,
        period: Optional[Sequence[float]] = None, ktabs=None, basis: Optional[np.ndarray] = None,
        tcoef: Optional[np.ndarray] = None, n0: int = 0) -> np.ndarray:
    """nsteps steps from u0 (eq. uN).  Time-dependent V: tcoef [steps, M] with basis [M, *grid]."""
    u = _c(u0).copy()
    ndim, n = _dims(u)
    dx = grid_dx(n, period)
    Pp = _c(P)
    ptrs, half, keep = _ktabs(ktabs, ndim)
    Vc = None if V is None else _c(V)
    B = None if basis is None else _c(basis)
    TC = None if tcoef is None else _c(tcoef)
    M = 0 if B is None else B.shape[0]
    rc = lib().orc_run(ndim, n.ctypes.data_as(_i64p), _f64(dx), tau, _f64(Pp), ptrs,
                       None if half is None else half.ctypes.data_as(_i64p), _f64(Vc), M, _f64(B),
                       _f64(TC), n0, nsteps, _f64(u))
    if rc:
        raise RuntimeError("orc_run failed: %d" % rc)
    return u


def joint_step(u: np.ndarray, tau: float, P: Sequence[float], V: Optional[np.ndarray] = None,
               period: Optional[Sequence[float]] = None) -> np.ndarray:
    """One step by the joint n-D minimum (left side of Remark rk28)."""
    u = _c(u).copy()
    ndim, n = _dims(u)
    dx = grid_dx(n, period)
    Pp = _c(P)
    Vc = None if V is None else _c(V)
    rc = lib().orc_joint_step(ndim, n.ctypes.data_as(_i64p), _f64(dx), tau, _f64(Pp), _f64(Vc), _f64(u))
    if rc:
        raise RuntimeError("orc_joint_step failed: %d" % rc)
    return u


def potential(basis: np.ndarray, coef: np.ndarray) -> np.ndarray:
    """V = sum_m c_m phi_m, summed in m order."""
    B = _c(basis)
    c = _c(coef)
    npts = int(np.prod(B.shape[1:]))
    V = np.empty(B.shape[1:], dtype=np.float64)
    lib().orc_potential(npts, B.shape[0], _f64(B), _f64(c), _f64(V))
    return V


def adjoint(u0: np.ndarray, tau: float, P: Sequence[float], nsteps: int, basis: np.ndarray,
            coef: np.ndarray, grad_uT: np.ndarray, period: Optional[Sequence[float]] = None):
    """Returns (uT, grad_u0, grad_coef) of the N-step map for V = sum c_m phi_m."""
    u0 = _c(u0)
    ndim, n = _dims(u0)
    dx = grid_dx(n, period)
    Pp = _c(P)
    B = _c(basis)
    c = _c(coef)
    g = _c(grad_uT)
    uT = np.empty_like(u0)
    gu = np.empty_like(u0)
    gc = np.empty(B.shape[0], dtype=np.float64)
    rc = lib().orc_adjoint(ndim, n.ctypes.data_as(_i64p), _f64(dx), tau, _f64(Pp), nsteps, _f64(u0),
                           B.shape[0], _f64(B), _f64(c), _f64(g), _f64(uT), _f64(gu), _f64(gc))
    if rc:
        raise RuntimeError("orc_adjoint failed: %d" % rc)
    return uT, gu, gc


def num_threads() -> int:
    return int(lib().orc_num_threads())


def semigroup1_step(u: np.ndarray, tau: float, P: float, V: Optional[np.ndarray] = None, period: float = 1.0,
                    ktab: Optional[np.ndarray] = None, with_argmin: bool = False):
    """One step of the first discrete semigroup (Section 2.2, eq. cost1) on a
    1-D periodic grid with static V: the straight-path action, the time
    integral of V by the trapezoid rule over the crossed grid points of
    hv = fl(tau V) (lo_oracle.c).  Returns u+ (and int32 argmin offsets)."""
    u = _c(u)
    N = u.shape[0]
    hv = None if V is None else _c(tau * _c(V))
    kt = None if ktab is None else _c(ktab)
    half = 0 if kt is None else (kt.shape[0] - 1) // 2
    w = np.empty_like(u)
    arg = np.empty(N, dtype=np.int32) if with_argmin else None
    rc = lib().orc_semigroup1_step(N, float(period) / N, tau, P, _f64(kt), half, _f64(hv), _f64(u), _f64(w),
                                   None if arg is None else arg.ctypes.data_as(_i32p))
    if rc:
        raise RuntimeError("orc_semigroup1_step failed: %d" % rc)
    return (w, arg) if with_argmin else w


def semigroup1_run(u0: np.ndarray, tau: float, P: float, nsteps: int, V: Optional[np.ndarray] = None,
                   period: float = 1.0, ktab: Optional[np.ndarray] = None) -> np.ndarray:
    """nsteps steps of the first discrete semigroup (eq. compo)."""
    u = _c(u0).copy()
    for _ in range(nsteps):
        u = semigroup1_step(u, tau, P, V, period, ktab)
    return u
