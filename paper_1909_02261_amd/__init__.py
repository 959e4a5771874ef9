"""TensCol population step on MI355X (gfx950): Python binding of libtcol.

Only argument marshalling lives here; every step of the method runs in the HIP
kernels of libtcol.so (see include/tcol.h).  PyTorch provides device memory and
the stream.  There is no CPU fallback: without the built library the import of
the binding fails.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

from . import _lib
from ._lib import BF16, BKPART, ECP, FP4, FP8, FP32, KCOL, KPART, MCOL, MSCP, TcolError

__all__ = ["Params", "Solver", "TensColLoss", "init_weights", "descent", "mfma_peak", "conflicts_noalloc",
           "KCOL", "ECP", "KPART", "BKPART", "MSCP", "MCOL",
           "FP32", "BF16", "FP8", "FP4", "TcolError"]


@dataclass
class Params:
    """Parameters of one graph (defaults: the paper's parameter table for the GCP)."""
    n: int
    k: int
    D: int
    problem: int = KCOL
    precision: int = FP32
    eta: float = 1e-3
    rho: float = 100.0
    nb_iter: int = 5
    alpha: float = 2.5
    lam: float = 1e-5
    beta: float = 1.2
    mu: float = 1e-6
    nu: float = 0.0
    bonus_diag: int = 1
    stop_on_legal: int = 1
    momentum: float = 0.0
    max_demand: int = 0      # multicolouring (MCOL): the largest number of colours of a vertex

    def c_struct(self) -> _lib.GraphParams:
        return _lib.GraphParams(self.problem, self.precision, self.n, self.k, self.D, self.eta, self.rho,
                                self.nb_iter, self.alpha, self.lam, self.beta, self.mu, self.nu,
                                self.bonus_diag, self.stop_on_legal, self.momentum, self.max_demand)

    @classmethod
    def from_dict(cls, d: dict) -> "Params":
        keys = cls.__dataclass_fields__.keys()
        return cls(**{k: v for k, v in d.items() if k in keys})


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Solver:
    """A libtcol context over G graphs.

    graphs: list of (A, W) with A a CUDA uint8 [n, n] 0/1 adjacency and W a CUDA
    float32 [D, n, k] weight tensor that the solver updates in place.
    """

    def __init__(self, graphs: Sequence, params: Sequence[Params], stream=None, workspace: bool = True):
        torch = _torch()
        lib = _lib.load()
        if len(graphs) != len(params) or not graphs:
            raise ValueError("one Params per graph")
        self.G = len(graphs)
        self.params = list(params)
        self.A = []
        self.W = []
        for (A, W), p in zip(graphs, params):
            if not (A.is_cuda and W.is_cuda):
                raise ValueError("A and W must be device tensors")
            if A.dtype != torch.uint8 or tuple(A.shape) != (p.n, p.n):
                raise ValueError(f"A must be uint8 [{p.n}, {p.n}]")
            if W.dtype != torch.float32 or tuple(W.shape) != (p.D, p.n, p.k) or not W.is_contiguous():
                raise ValueError(f"W must be contiguous float32 [{p.D}, {p.n}, {p.k}]")
            self.A.append(A.contiguous())
            self.W.append(W)
        self._cp = (_lib.GraphParams * self.G)(*[p.c_struct() for p in params])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        size = ctypes.c_size_t(0)
        _lib.check(lib.tcol_workspace_size(self.G, self._cp, ctypes.byref(size)), "tcol_workspace_size")
        self.ws = None
        ws_ptr, ws_bytes = None, 0
        if workspace:
            self.ws = torch.empty(size.value, dtype=torch.uint8, device=self.W[0].device)
            ws_ptr, ws_bytes = ctypes.c_void_p(self.ws.data_ptr()), size.value
        A_arr = (ctypes.c_void_p * self.G)(*[a.data_ptr() for a in self.A])
        W_arr = (ctypes.c_void_p * self.G)(*[w.data_ptr() for w in self.W])
        ctx = ctypes.c_void_p()
        _lib.check(lib.tcol_init(ctypes.byref(ctx), self.G, self._cp, A_arr, W_arr, ws_ptr, ws_bytes,
                                 ctypes.c_void_p(self.stream.cuda_stream)), "tcol_init")
        self._ctx = ctx
        self._lib = lib

    # ------------------------------------------------------------------ API --
    def close(self) -> None:
        if getattr(self, "_ctx", None):
            self._lib.tcol_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def options(self) -> dict:
        o = _lib.Options()
        _lib.check(self._lib.tcol_get_options(self._ctx, ctypes.byref(o)), "tcol_get_options")
        return {f: getattr(o, f) for f, _ in o._fields_}

    def set_options(self, **kw) -> None:
        cur = self.options()
        cur.update(kw)
        o = _lib.Options(**cur)
        _lib.check(self._lib.tcol_set_options(self._ctx, ctypes.byref(o)), "tcol_set_options")

    def step(self, max_steps: int, colors_out: Optional[List] = None):
        """Run up to max_steps iterations; returns (steps_done, legal_d list)."""
        done = ctypes.c_int32(0)
        legal = (ctypes.c_int32 * self.G)()
        outs = None
        if colors_out is not None:
            outs = (ctypes.c_void_p * self.G)(*[None if c is None else c.data_ptr() for c in colors_out])
        _lib.check(self._lib.tcol_step(self._ctx, int(max_steps), ctypes.byref(done), legal, outs), "tcol_step")
        return done.value, list(legal)

    def conflicts(self, g: int = 0):
        """(colours int16 [D, n], main fitness int64 [D], added fitness int64 [D]) of the current W:
        f_color (the cut for partitioning) and f_eq (the colour cost for minimum sum colouring,
        0 for k-COL and plain partitioning)."""
        torch = _torch()
        p = self.params[g]
        dev = self.W[g].device
        c = torch.empty((p.D, p.n), dtype=torch.int16, device=dev)
        fc = torch.empty(p.D, dtype=torch.int64, device=dev)
        fe = torch.empty(p.D, dtype=torch.int64, device=dev)
        _lib.check(self._lib.tcol_conflicts(self._ctx, g, _ptr(c), _ptr(fc), _ptr(fe)), "tcol_conflicts")
        return c, fc, fe

    def loss_grad(self, g: int = 0, want_loss=True, want_gs=True, want_gw=True):
        """(loss float64 [5] = L, sum main fitness, sum added fitness, kappa, varpi; grad_S; grad_W)."""
        torch = _torch()
        p = self.params[g]
        dev = self.W[g].device
        loss = torch.empty(5, dtype=torch.float64, device=dev) if want_loss else None
        gs = torch.empty((p.D, p.n, p.k), dtype=torch.float32, device=dev) if want_gs else None
        gw = torch.empty((p.D, p.n, p.k), dtype=torch.float32, device=dev) if want_gw else None
        _lib.check(self._lib.tcol_loss_grad(self._ctx, g, _ptr(loss), _ptr(gs), _ptr(gw)), "tcol_loss_grad")
        return loss, gs, gw

    def set_demand(self, demand, g: int = 0) -> None:
        """Multicolouring demands c_i (n ints in 1..max_demand) of graph g (an MCOL graph)."""
        import numpy as np
        d = np.ascontiguousarray(np.asarray(demand, dtype=np.int32))
        if d.shape != (self.params[g].n,):
            raise ValueError(f"demand must have {self.params[g].n} entries")
        _lib.check(self._lib.tcol_set_demand(self._ctx, g, d.ctypes.data_as(ctypes.c_void_p)), "tcol_set_demand")

    def selection(self, g: int = 0):
        """int16 [D, n, max(1, max_demand)]: each vertex's selected colours in decreasing weight, -1
        past its demand (the argmax colouring for one colour per vertex)."""
        torch = _torch()
        p = self.params[g]
        cm = max(1, p.max_demand) if p.problem == MCOL else 1
        out = torch.empty((p.D, p.n, cm), dtype=torch.int16, device=self.W[g].device)
        _lib.check(self._lib.tcol_selection(self._ctx, g, _ptr(out)), "tcol_selection")
        return out

    def class_conflicts(self, g: int = 0):
        """S_d^T A S_d of every member (int32 [D, k, k]): edges between colour classes."""
        torch = _torch()
        p = self.params[g]
        C = torch.empty((p.D, p.k, p.k), dtype=torch.int32, device=self.W[g].device)
        _lib.check(self._lib.tcol_class_conflicts(self._ctx, g, _ptr(C)), "tcol_class_conflicts")
        return C

    def mtilde(self, g: int = 0):
        torch = _torch()
        p = self.params[g]
        m = torch.empty((p.n, p.n), dtype=torch.int32, device=self.W[g].device)
        _lib.check(self._lib.tcol_mtilde(self._ctx, g, _ptr(m)), "tcol_mtilde")
        return m

    def get_t(self, g: int = 0) -> int:
        t = ctypes.c_int64(0)
        _lib.check(self._lib.tcol_get_t(self._ctx, g, ctypes.byref(t)), "tcol_get_t")
        return t.value

    def set_t(self, t: int, g: int = 0) -> None:
        _lib.check(self._lib.tcol_set_t(self._ctx, g, int(t)), "tcol_set_t")

    def reset(self) -> None:
        _lib.check(self._lib.tcol_reset(self._ctx), "tcol_reset")

    def set_wait_limit(self, polls: int) -> None:
        """Batch launch (fused = 3): polls of a waiting item before it gives up (0: default)."""
        _lib.check(self._lib.tcol_set_wait_limit(self._ctx, int(polls)), "tcol_set_wait_limit")

    def cancel(self) -> None:
        """Batch launch: make the tcol_step in progress (another thread) give up (TCOL_EABORT)."""
        _lib.check(self._lib.tcol_cancel(self._ctx), "tcol_cancel")

    def counters(self, g: int = 0) -> dict:
        """Iterations of graph g evaluated since init, by the route of the penalty product."""
        out = (ctypes.c_int64 * 3)()
        _lib.check(self._lib.tcol_get_counters(self._ctx, g, out), "tcol_get_counters")
        return {"no_penalty": out[0], "dense": out[1], "sparse": out[2]}

    def profile(self, steps: int, as_only: bool = False) -> dict:
        """Average ms per iteration of each kernel phase (eager launches, HIP events)."""
        ms = (ctypes.c_float * _lib.NPHASES)()
        _lib.check(self._lib.tcol_profile(self._ctx, int(steps), int(as_only), ms), "tcol_profile")
        return dict(zip(_lib.PHASES, [float(x) for x in ms]))

    def autotune(self):
        bm, ntw = ctypes.c_int32(0), ctypes.c_int32(0)
        _lib.check(self._lib.tcol_autotune(self._ctx, ctypes.byref(bm), ctypes.byref(ntw)), "tcol_autotune")
        return bm.value, ntw.value


def mfma_peak(precision: int, iters: int = 4000) -> float:
    """Achievable dense MFMA TFLOP/s of the current device for one operand type
    (tcol_mfma_peak: register operands, every CU, no memory traffic)."""
    lib = _lib.load()
    out = ctypes.c_double(0.0)
    _lib.check(lib.tcol_mfma_peak(int(precision), int(iters), ctypes.byref(out)), "tcol_mfma_peak")
    return out.value


def conflicts_noalloc(A, W, params: Params, colors=None, f_main=None, f_sec=None, stream=None):
    """tcol_conflicts_noalloc: colours and fitness of the population W (float32 [D, n, k]) on the
    graph A (uint8 [n, n]) with no context and no device allocation inside the library.  The
    output tensors (int16 [D, n], int64 [D], int64 [D]) are the caller's; they are created here
    when not given.  Asynchronous on `stream`."""
    torch = _torch()
    p = params
    if A.dtype != torch.uint8 or tuple(A.shape) != (p.n, p.n) or not A.is_contiguous() or not A.is_cuda:
        raise ValueError(f"A must be a contiguous uint8 device tensor [{p.n}, {p.n}]")
    if W.dtype != torch.float32 or tuple(W.shape) != (p.D, p.n, p.k) or not W.is_contiguous() or not W.is_cuda:
        raise ValueError(f"W must be a contiguous float32 device tensor [{p.D}, {p.n}, {p.k}]")
    if colors is None:
        colors = torch.empty((p.D, p.n), dtype=torch.int16, device=W.device)
    if f_main is None:
        f_main = torch.empty(p.D, dtype=torch.int64, device=W.device)
    if f_sec is None:
        f_sec = torch.empty(p.D, dtype=torch.int64, device=W.device)
    lib = _lib.load()
    st = stream if stream is not None else torch.cuda.current_stream()
    cp = p.c_struct()
    _lib.check(lib.tcol_conflicts_noalloc(ctypes.byref(cp), _ptr(A), _ptr(W), _ptr(colors), _ptr(f_main),
                                          _ptr(f_sec), ctypes.c_void_p(st.cuda_stream)), "tcol_conflicts_noalloc")
    return colors, f_main, f_sec


def init_weights(W, seed: int, sigma0: float = 0.01, stream=None) -> None:
    """Fill the contiguous fp32 device tensor W with N(0, sigma0^2) draws (tcol_init_weights)."""
    torch = _torch()
    if W.dtype != torch.float32 or not W.is_contiguous() or not W.is_cuda:
        raise ValueError("W must be a contiguous float32 device tensor")
    lib = _lib.load()
    st = stream if stream is not None else torch.cuda.current_stream()
    _lib.check(lib.tcol_init_weights(_ptr(W), W.numel(), int(seed) & (2**64 - 1), float(sigma0),
                                     ctypes.c_void_p(st.cuda_stream)), "tcol_init_weights")


def descent(A, params: Params, k_first: int, k_min: int = 1, max_steps: int = 10000, attempts: int = 1,
            seed: int = 0, sigma0: float = 0.01, stream=None):
    """Colour-count descent on graph A (uint8 n x n device tensor) with the method's parameters
    `params` (k is overridden).  Returns (result dict, int16 device tensor of the legal colouring
    with result["k_best"] colours, or None when none was found)."""
    torch = _torch()
    if A.dtype != torch.uint8 or not A.is_contiguous() or not A.is_cuda:
        raise ValueError("A must be a contiguous uint8 device tensor")
    lib = _lib.load()
    st = stream if stream is not None else torch.cuda.current_stream()
    colors = torch.zeros(params.n, dtype=torch.int16, device=A.device)
    opt = _lib.DescentOptions(int(k_first), int(k_min), int(max_steps), int(attempts), int(seed) & (2**64 - 1),
                              float(sigma0))
    res = _lib.DescentResult()
    cp = params.c_struct()
    _lib.check(lib.tcol_descent(_ptr(A), ctypes.byref(cp), ctypes.byref(opt), ctypes.byref(res), _ptr(colors),
                                ctypes.c_void_p(st.cuda_stream)), "tcol_descent")
    out = {f: getattr(res, f) for f, _ in _lib.DescentResult._fields_}
    return out, (colors if res.k_best >= 0 else None)


class TensColLoss:
    """torch.autograd.Function whose backward is libtcol's straight-through gradient kernel.

    loss = TensColLoss.apply(W, solver, g) returns the global loss L(t) (a float64
    scalar on the device) of graph g at the solver's current t; W must be the
    weight tensor registered with the solver.  backward returns grad_out * grad_W.
    """

    _fn = None

    @classmethod
    def apply(cls, W, solver: Solver, g: int = 0):
        if cls._fn is None:
            cls._fn = _make_function()
        return cls._fn.apply(W, solver, g)


def _make_function():
    torch = _torch()

    class _TensColLossFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, W, solver, g):
            if W.data_ptr() != solver.W[g].data_ptr():
                raise ValueError("W is not the weight tensor registered with this solver")
            loss, _, gw = solver.loss_grad(g, want_loss=True, want_gs=False, want_gw=True)
            ctx.save_for_backward(gw)
            return loss[0]

        @staticmethod
        def backward(ctx, grad_out):
            (gw,) = ctx.saved_tensors
            return (grad_out.to(gw.dtype) * gw, None, None)

    return _TensColLossFn
