"""Python front end of the HIP library: PyTorch supplies device memory and
streams, every step of the scheme runs in the library's kernels.

Arrays are torch float64 CUDA (HIP) tensors shaped like the grid in numpy
order, (n[ndim-1], ..., n[0]); axis 0 of the scheme is the last tensor
dimension (fastest in memory).
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import LoDesc, LoPotential, check, lib


def _stream(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t: torch.Tensor, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t


def make_desc(n: Sequence[int], tau: float, P: Sequence[float], period=None, method: str = "fast",
              window=None, kstar_tabs=None, t0: float = 0.0, graph: bool = True, keep=None,
              autotune: bool = False) -> LoDesc:
    ndim = len(n)
    d = LoDesc()
    d.ndim = ndim
    period = [1.0] * ndim if period is None else list(period)
    for a in range(ndim):
        d.n[a] = int(n[a])
        d.period[a] = float(period[a])
        d.P[a] = float(P[a])
        d.window[a] = 0 if window is None else int(window[a])
        if kstar_tabs is not None and kstar_tabs[a] is not None:
            tab = np.ascontiguousarray(kstar_tabs[a], dtype=np.float64)
            if keep is not None:
                keep.append(tab)
            d.kstar_tab[a] = tab.ctypes.data
            d.kstar_half[a] = (tab.shape[0] - 1) // 2
    d.tau = float(tau)
    d.method = _lib.LO_FAST if method == "fast" else _lib.LO_BRUTE
    d.flags = (0 if graph else _lib.LO_FLAG_NO_GRAPH) | (_lib.LO_FLAG_AUTOTUNE if autotune else 0)
    d.t0 = float(t0)
    return d


class Plan:
    """A plan for one grid, time step, kinetic cost and potential (lo_plan).

    n: grid points per axis (axis 0 first).  V: static potential on the grid
    (CUDA float64 tensor shaped like the grid), or basis (CUDA tensor
    [M, *grid]) with static coef (M,) or time-dependent tcoef (steps, M).
    autotune: the first run advances a copy of its input past the first
    steps and times the fast sweeps' launch shapes from there, keeping the
    fastest per axis (results do not depend on the shape); the choice is kept
    for the process's later plans of the same grid (and in the file named by
    the environment variable LO_TUNE_CACHE, when set).
    """

    def __init__(self, n: Sequence[int], tau: float, P: Sequence[float], period=None,
                 V: Optional[torch.Tensor] = None, basis: Optional[torch.Tensor] = None,
                 coef=None, tcoef=None, method: str = "fast", window=None, kstar_tabs=None,
                 t0: float = 0.0, graph: bool = True, autotune: bool = False):
        self.n = tuple(int(v) for v in n)
        self.ndim = len(self.n)
        self.shape = tuple(reversed(self.n))
        self.npts = int(np.prod(self.n))
        self.tau = float(tau)
        self._keep = []
        desc = make_desc(self.n, tau, P, period, method, window, kstar_tabs, t0, graph, self._keep, autotune)
        pot = LoPotential()
        self.V = None
        self.basis = None
        self.nmodes = 0
        if V is not None:
            self.V = _dev_f64(V, "V", self.shape)
            pot.table = self.V.data_ptr()
        elif basis is not None:
            self.basis = _dev_f64(basis, "basis")
            if tuple(self.basis.shape[1:]) != self.shape:
                raise ValueError("basis must be [M, *grid]")
            self.nmodes = int(self.basis.shape[0])
            pot.nmodes = self.nmodes
            pot.basis = self.basis.data_ptr()
            if tcoef is not None:
                tc = np.ascontiguousarray(tcoef, dtype=np.float64).reshape(-1, self.nmodes)
                self._keep.append(tc)
                pot.tcoef = tc.ctypes.data
                pot.ntcoef = tc.shape[0]
            else:
                c = np.ascontiguousarray(coef, dtype=np.float64).reshape(self.nmodes)
                self._keep.append(c)
                pot.coef = c.ctypes.data
        self._desc = desc
        h = ctypes.c_void_p()
        check("lo_plan", lib().lo_plan(ctypes.byref(desc), ctypes.byref(pot), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lo_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_coef(self, coef) -> None:
        c = np.ascontiguousarray(coef, dtype=np.float64).reshape(self.nmodes)
        check("lo_set_coef", lib().lo_set_coef(self._h, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def step(self, u: torch.Tensor, n: int = 0, argmin: bool = False, stream=None):
        """One step in place on u; returns the int16 argmin offsets [ndim, *grid] if asked."""
        _dev_f64(u, "u", self.shape)
        arg = None
        if argmin:
            arg = torch.empty((self.ndim,) + self.shape, dtype=torch.int16, device=u.device)
        check("lo_step", lib().lo_step(self._h, ctypes.c_void_p(u.data_ptr()), int(n),
                                       ctypes.c_void_p(arg.data_ptr() if arg is not None else 0),
                                       _stream(stream)))
        return arg

    def run(self, u: torch.Tensor, nsteps: int, n0: int = 0, ckpt_every: int = 0, stream=None):
        """nsteps steps in place on u; returns the checkpoints if ckpt_every > 0."""
        _dev_f64(u, "u", self.shape)
        ck = None
        if ckpt_every > 0:
            k = (nsteps + ckpt_every - 1) // ckpt_every
            ck = torch.empty((k,) + self.shape, dtype=torch.float64, device=u.device)
        check("lo_run", lib().lo_run(self._h, ctypes.c_void_p(u.data_ptr()), int(n0), int(nsteps),
                                     int(ckpt_every), ctypes.c_void_p(ck.data_ptr() if ck is not None else 0),
                                     _stream(stream)))
        return ck

    def backward(self, ckpt: torch.Tensor, nsteps: int, ckpt_every: int, grad_uT: torch.Tensor,
                 want_u0: bool = True, want_coef: bool = True, stream=None):
        """Adjoint of the N-step map: returns (grad_u0 tensor or None, grad_coef ndarray or None)."""
        if ckpt is not None and ckpt.numel() > 0:
            _dev_f64(ckpt, "ckpt")
        ckpt_ptr = ckpt.data_ptr() if ckpt is not None and ckpt.numel() > 0 else 0
        _dev_f64(grad_uT, "grad_uT", self.shape)
        gu = torch.empty_like(grad_uT) if want_u0 else None
        gc = np.zeros(max(self.nmodes, 1), dtype=np.float64) if (want_coef and self.nmodes > 0) else None
        check("lo_backward", lib().lo_backward(
            self._h, ctypes.c_void_p(ckpt_ptr), int(nsteps), int(ckpt_every),
            ctypes.c_void_p(grad_uT.data_ptr()), ctypes.c_void_p(gu.data_ptr() if gu is not None else 0),
            gc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if gc is not None else None, _stream(stream)))
        return gu, (gc[: self.nmodes] if gc is not None else None)

    def diag(self):
        w = (ctypes.c_int32 * 3)()
        m = (ctypes.c_int32 * 3)()
        st = lib().lo_last_diag(self._h, m, w)
        if st not in (_lib.LO_OK, _lib.LO_ERR_WINDOW):
            check("lo_last_diag", st)
        return list(w[: self.ndim]), list(m[: self.ndim])

    def time_kernels(self, u: torch.Tensor, nsteps: int, n0: int = 0, stream=None):
        """Mean duration (ms) of each axis' sweep kernel over nsteps steps (HIP events)."""
        _dev_f64(u, "u", self.shape)
        ms = np.zeros(3, dtype=np.float64)
        check("lo_time_kernels", lib().lo_time_kernels(self._h, ctypes.c_void_p(u.data_ptr()), int(n0), int(nsteps),
                                                       ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                       _stream(stream)))
        return ms[: self.ndim]

    def run_decomp(self, u: torch.Tensor, nsteps: int, eta: float = 0.0, window: int = 0, n0: int = 0,
                   stream=None):
        """Comparison path (1-D plans): nsteps steps of the paper's convex /
        concave decomposition algorithm with tolerance eta on offsets
        [-window, window] (0: the plan's whole table).  Returns (pieces,
        breaks) counted over the run."""
        _dev_f64(u, "u", self.shape)
        pieces, breaks = ctypes.c_int64(0), ctypes.c_int64(0)
        check("lo_run_decomp", lib().lo_run_decomp(self._h, ctypes.c_void_p(u.data_ptr()), int(n0), int(nsteps),
                                                   float(eta), int(window), ctypes.byref(pieces),
                                                   ctypes.byref(breaks), _stream(stream)))
        return pieces.value, breaks.value

    def run_record(self, u: torch.Tensor, nsteps: int, n0: int = 0, stream=None) -> torch.Tensor:
        """Run nsteps steps recording every sweep's int16 argmins; returns the
        record ([nsteps, ndim, *grid]) for backward_recorded."""
        _dev_f64(u, "u", self.shape)
        E = torch.empty((max(int(nsteps), 0), self.ndim) + self.shape, dtype=torch.int16, device=u.device)
        check("lo_run_record", lib().lo_run_record(self._h, ctypes.c_void_p(u.data_ptr()), int(n0), int(nsteps),
                                                   ctypes.c_void_p(E.data_ptr() if E.numel() else 0),
                                                   _stream(stream)))
        return E

    def backward_recorded(self, E: torch.Tensor, nsteps: int, grad_uT: torch.Tensor, want_u0: bool = True,
                          want_coef: bool = True, stream=None):
        """Adjoint from a record of run_record: (grad_u0 tensor or None, grad_coef ndarray or None)."""
        if E.dtype != torch.int16 or not E.is_contiguous() or tuple(E.shape) != (int(nsteps), self.ndim) + self.shape:
            raise ValueError("E must be the contiguous int16 record of run_record")
        _dev_f64(grad_uT, "grad_uT", self.shape)
        gu = torch.empty_like(grad_uT) if want_u0 else None
        gc = np.zeros(max(self.nmodes, 1), dtype=np.float64) if (want_coef and self.nmodes > 0) else None
        check("lo_backward_recorded", lib().lo_backward_recorded(
            self._h, ctypes.c_void_p(E.data_ptr() if E.numel() else 0), int(nsteps),
            ctypes.c_void_p(grad_uT.data_ptr()), ctypes.c_void_p(gu.data_ptr() if gu is not None else 0),
            gc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if gc is not None else None, _stream(stream)))
        return gu, (gc[: self.nmodes] if gc is not None else None)

    def run_semigroup1(self, u: torch.Tensor, nsteps: int, window: int = 0, stream=None):
        """nsteps steps of the first discrete semigroup (1-D plans, static V):
        straight-path action with the trapezoid time integral of V, offsets
        within [-window, window] (0: the plan's whole table)."""
        _dev_f64(u, "u", self.shape)
        check("lo_run_semigroup1", lib().lo_run_semigroup1(self._h, ctypes.c_void_p(u.data_ptr()), int(nsteps),
                                                           int(window), _stream(stream)))

    def kinetic_table(self, axis: int, s0: int, count: int) -> np.ndarray:
        out = np.empty(count, dtype=np.float64)
        check("lo_kinetic_table", lib().lo_kinetic_table(self._h, int(axis), int(s0), int(count),
                                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out


def step_noalloc(u: torch.Tensor, n: Sequence[int], tau: float, P: Sequence[float], tau_v=None, step: int = 0,
                 period=None, method: str = "fast", window=None, t0: float = 0.0, argmin: bool = False,
                 stream=None):
    """One step in place on u without a plan and without device allocation
    by the library (lo_step_noalloc): mechanical cost, tau_v = fl(tau V(t_n))
    as a CUDA float64 tensor shaped like the grid, or None.  Returns the int16
    argmins [ndim, *grid] if asked (allocated here, by torch)."""
    shape = tuple(reversed([int(v) for v in n]))
    _dev_f64(u, "u", shape)
    if tau_v is not None:
        _dev_f64(tau_v, "tau_v", shape)
    desc = make_desc(n, tau, P, period, method, window, None, t0)
    arg = None
    if argmin:
        arg = torch.empty((len(n),) + shape, dtype=torch.int16, device=u.device)
    check("lo_step_noalloc", lib().lo_step_noalloc(
        ctypes.byref(desc), ctypes.c_void_p(tau_v.data_ptr() if tau_v is not None else 0),
        ctypes.c_void_p(u.data_ptr()), int(step), ctypes.c_void_p(arg.data_ptr() if arg is not None else 0),
        _stream(stream)))
    return arg


def effective_H(sides: Sequence[int], P: np.ndarray, V_by_side: dict, tau: float, T: float,
                method: str = "fast", autotune: bool = False, stream=None) -> np.ndarray:
    """Batched discrete effective Hamiltonian of square 2-D instances
    (lo_effective_H).  V_by_side: side -> CUDA float64 tensor [side, side].
    autotune: each batch's fast sweeps take the launch shapes the tuner picks
    (results do not depend on them).  Returns [ninst, 3] = (lower bound,
    midpoint, upper bound)."""
    ninst = len(sides)
    descs = (LoDesc * ninst)()
    pots = (LoPotential * ninst)()
    for i, s in enumerate(sides):
        s = int(s)
        descs[i] = make_desc([s, s], tau, [float(P[i][0]), float(P[i][1])], method=method, autotune=autotune)
        V = _dev_f64(V_by_side[s], "V", (s, s))
        pots[i].table = V.data_ptr()
    out = np.zeros((ninst, 3), dtype=np.float64)
    check("lo_effective_H", lib().lo_effective_H(ninst, descs, pots, float(T),
                                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 _stream(stream)))
    return out


class LaxOleinik(torch.autograd.Function):
    """u(T) = T^N u0 for V = sum_m coef_m basis_m, differentiable in u0 and coef.

    forward(u0, coef, plan, nsteps, ckpt_every); gradients come from the
    library's argmin-scatter adjoint: lo_backward recomputing segments of
    ckpt_every steps from FP64 checkpoints, or, with ckpt_every = 0, every
    step's argmins recorded by the forward pass (lo_run_record,
    lo_backward_recorded: no recomputation, 2 ndim bytes a point a step)."""

    @staticmethod
    def forward(ctx, u0: torch.Tensor, coef: torch.Tensor, plan: Plan, nsteps: int, ckpt_every: int):
        plan.set_coef(coef.detach().cpu().numpy())
        u = u0.detach().clone()
        ck = plan.run_record(u, nsteps) if ckpt_every == 0 else plan.run(u, nsteps, 0, ckpt_every)
        ctx.plan = plan
        ctx.nsteps = nsteps
        ctx.ckpt_every = ckpt_every
        ctx.save_for_backward(ck, coef)
        return u

    @staticmethod
    def backward(ctx, grad_uT: torch.Tensor):
        ck, coef = ctx.saved_tensors
        if ctx.ckpt_every == 0:
            gu, gc = ctx.plan.backward_recorded(ck, ctx.nsteps, grad_uT.contiguous(),
                                                want_u0=ctx.needs_input_grad[0], want_coef=ctx.needs_input_grad[1])
        else:
            gu, gc = ctx.plan.backward(ck, ctx.nsteps, ctx.ckpt_every, grad_uT.contiguous(),
                                       want_u0=ctx.needs_input_grad[0], want_coef=ctx.needs_input_grad[1])
        gcoef = None
        if gc is not None:
            gcoef = torch.as_tensor(gc, dtype=coef.dtype, device=coef.device)
        return gu, gcoef, None, None, None
