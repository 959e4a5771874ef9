"""FP64 CPU oracle of one TensCol iteration -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library; it is checked against
the paper itself (worked examples, closed forms, brute force, invariances and
finite differences) in tests/test_oracle.py.

`tcol_oracle.c` holds the arithmetic (plain C, FP64, single thread); this module
only marshals numpy arrays to it.  `literal.py` is a second, literal numpy
transcription of the paper's tensor formulas for tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


class OrcParams(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int32), ("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("D", ctypes.c_int32), ("eta", ctypes.c_double), ("rho", ctypes.c_double),
                ("nb_iter", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("lam", ctypes.c_double), ("beta", ctypes.c_double), ("mu", ctypes.c_double),
                ("nu", ctypes.c_double), ("bonus_diag", ctypes.c_int32),
                ("stop_on_legal", ctypes.c_int32), ("momentum", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        src = _build.SRC
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        _lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        _lib.orc_colors.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        _lib.orc_colors.restype = ctypes.c_int
        _lib.orc_class_sizes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        _lib.orc_fcolor.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
        _lib.orc_equity_bounds.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
        _lib.orc_feq.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        _lib.orc_fcut.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
        _lib.orc_fmscp.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
        _lib.orc_fitness.argtypes = [P, P, P, P, P, P, P]
        _lib.orc_mtilde.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
        _lib.orc_class_conflicts.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
        _lib.orc_grad_s.argtypes = [P, i64, P, P, P, P, P]
        _lib.orc_grad_w.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
        _lib.orc_update.argtypes = [P, i64, P, P, P]
        _lib.orc_loss.argtypes = [P, i64, P, P, P, P, P]
        _lib.orc_iteration.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P]
        _lib.orc_iteration.restype = ctypes.c_int
        _lib.orc_run.argtypes = [P, P, P, P, ctypes.c_int, P, P]
        _lib.orc_select.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
        _lib.orc_select.restype = ctypes.c_int
        _lib.orc_fcolor_multi.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
        _lib.orc_mtilde_multi.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        _lib.orc_class_sizes_multi.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        _lib.orc_grad_s_multi.argtypes = [P, i64, P, P, P, P]
        _lib.orc_iteration_multi.argtypes = [P, P, P, P, P, P, P, P, P, P]
        _lib.orc_iteration_multi.restype = ctypes.c_int
        _lib.orc_run.restype = ctypes.c_int
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


@dataclass
class Params:
    problem: int
    n: int
    k: int
    D: int
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

    @classmethod
    def from_dict(cls, d: dict) -> "Params":
        keys = cls.__dataclass_fields__.keys()
        return cls(**{k: v for k, v in d.items() if k in keys})

    def c_struct(self) -> OrcParams:
        return OrcParams(self.problem, self.n, self.k, self.D, self.eta, self.rho, self.nb_iter,
                         self.alpha, self.lam, self.beta, self.mu, self.nu, self.bonus_diag,
                         self.stop_on_legal, self.momentum)


def colors(W: np.ndarray) -> np.ndarray:
    """argmax over the colour axis (lowest index on ties); W [D, n, k]."""
    W = _c(W, np.float64)
    D, n, k = W.shape
    c = np.zeros((D, n), dtype=np.int16)
    rc = lib().orc_colors(D, n, k, _ptr(W), _ptr(c))
    if rc:
        raise FloatingPointError("non-finite weight")
    return c


def class_sizes(c: np.ndarray, k: int) -> np.ndarray:
    c = _c(c, np.int16)
    D, n = c.shape
    V = np.zeros((D, k), dtype=np.int32)
    lib().orc_class_sizes(D, n, k, _ptr(c), _ptr(V))
    return V


def fcolor(A: np.ndarray, c: np.ndarray) -> np.ndarray:
    A = _c(A, np.uint8)
    c = _c(c, np.int16)
    D, n = c.shape
    f = np.zeros(D, dtype=np.int64)
    lib().orc_fcolor(D, n, _ptr(A), _ptr(c), _ptr(f))
    return f


def fcut(A: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Cut edges of each member's partition."""
    A = _c(A, np.uint8)
    c = _c(c, np.int16)
    D, n = c.shape
    f = np.zeros(D, dtype=np.int64)
    lib().orc_fcut(D, n, _ptr(A), _ptr(c), _ptr(f))
    return f


def fmscp(V: np.ndarray) -> np.ndarray:
    """Colour cost sum_l (l + 1) #V_dl of minimum sum colouring."""
    V = _c(V, np.int32)
    D, k = V.shape
    f = np.zeros(D, dtype=np.int64)
    lib().orc_fmscp(D, k, _ptr(V), _ptr(f))
    return f


def fitness(p: "Params", A: np.ndarray, c: np.ndarray):
    """(fmain, fsec, f) of each member for the problem of p."""
    A = _c(A, np.uint8)
    c = _c(c, np.int16)
    V = class_sizes(c, p.k)
    fm = np.zeros(p.D, np.int64); fs = np.zeros(p.D, np.int64); f = np.zeros(p.D, np.int64)
    ps = p.c_struct()
    lib().orc_fitness(ctypes.byref(ps), _ptr(A), _ptr(c), _ptr(V), _ptr(fm), _ptr(fs), _ptr(f))
    return fm, fs, f


def equity_bounds(n: int, k: int):
    c1 = np.zeros(1, np.int32)
    c2 = np.zeros(1, np.int32)
    lib().orc_equity_bounds(n, k, _ptr(c1), _ptr(c2))
    return int(c1[0]), int(c2[0])


def feq(V: np.ndarray, n: int) -> np.ndarray:
    V = _c(V, np.int32)
    D, k = V.shape
    f = np.zeros(D, dtype=np.int64)
    lib().orc_feq(D, n, k, _ptr(V), _ptr(f))
    return f


def mtilde(c: np.ndarray) -> np.ndarray:
    c = _c(c, np.int16)
    D, n = c.shape
    M = np.zeros((n, n), dtype=np.int32)
    lib().orc_mtilde(D, n, _ptr(c), _ptr(M))
    return M


def class_conflicts(A: np.ndarray, c: np.ndarray, k: int) -> np.ndarray:
    """S_d^T A S_d for every member: int32 [D, k, k], entry (l, l') the ordered edges from
    colour class l to class l' of member d."""
    A = _c(A, np.uint8)
    c = _c(c, np.int16)
    D, n = c.shape
    C = np.zeros((D, k, k), dtype=np.int32)
    lib().orc_class_conflicts(D, n, k, _ptr(A), _ptr(c), _ptr(C))
    return C


def grad_s(p: Params, t: int, A, c, Mt, V) -> np.ndarray:
    A = _c(A, np.uint8); c = _c(c, np.int16); Mt = _c(Mt, np.int32); V = _c(V, np.int32)
    g = np.zeros((p.D, p.n, p.k), dtype=np.float64)
    ps = p.c_struct()
    lib().orc_grad_s(ctypes.byref(ps), int(t), _ptr(A), _ptr(c), _ptr(Mt), _ptr(V), _ptr(g))
    return g


def grad_w(W: np.ndarray, gS: np.ndarray) -> np.ndarray:
    W = _c(W, np.float64); gS = _c(gS, np.float64)
    D, n, k = W.shape
    g = np.zeros_like(W)
    lib().orc_grad_w(D, n, k, _ptr(W), _ptr(gS), _ptr(g))
    return g


def update(p: Params, t: int, W: np.ndarray, gW: np.ndarray, vel: Optional[np.ndarray] = None) -> np.ndarray:
    """Step 4 on a copy of W; vel (FP64, updated in place) is the momentum state."""
    W = np.array(W, dtype=np.float64, copy=True)
    gW = _c(gW, np.float64)
    ps = p.c_struct()
    lib().orc_update(ctypes.byref(ps), int(t), _ptr(W), _ptr(gW), _ptr(vel))
    return W


def loss(p: Params, t: int, A, Mt, fc, fe) -> np.ndarray:
    """[L, sum fmain, sum fsec, kappa, varpi]; fc / fe are fmain / fsec of `fitness`."""
    A = _c(A, np.uint8); Mt = _c(Mt, np.int32)
    fc = _c(fc, np.int64); fe = _c(fe, np.int64)
    out = np.zeros(5, dtype=np.float64)
    ps = p.c_struct()
    lib().orc_loss(ctypes.byref(ps), int(t), _ptr(A), _ptr(Mt), _ptr(fc), _ptr(fe), _ptr(out))
    return out


@dataclass
class IterResult:
    status: int                 # 1 = legal member found (no update), 0 = updated
    W: np.ndarray               # weights after the iteration (FP64)
    t: int
    colors: np.ndarray
    f: np.ndarray
    f_color: np.ndarray         # fmain: f_color, or f_cut for partitioning
    f_eq: np.ndarray            # fsec: f_eq, f_mscp or 0
    gS: Optional[np.ndarray]
    gW: Optional[np.ndarray]
    legal_d: int


def iteration(p: Params, t: int, A: np.ndarray, W: np.ndarray, want_grads: bool = True,
              vel: Optional[np.ndarray] = None) -> IterResult:
    """One iteration (steps 1-4) from weights W (any float dtype, upcast to FP64).  With
    momentum, vel (FP64 [D, n, k], updated in place) is the velocity; zeros when omitted."""
    A = _c(A, np.uint8)
    Wd = np.array(W, dtype=np.float64, copy=True)
    D, n, k = Wd.shape
    tt = np.array([t], dtype=np.int64)
    c = np.zeros((D, n), np.int16)
    f = np.zeros(D, np.int64); fc = np.zeros(D, np.int64); fe = np.zeros(D, np.int64)
    gS = np.zeros((D, n, k)) if want_grads else None
    gW = np.zeros((D, n, k)) if want_grads else None
    ld = np.zeros(1, np.int32)
    if p.momentum != 0.0 and vel is None:
        vel = np.zeros((D, n, k))
    if vel is not None:
        assert vel.dtype == np.float64 and vel.flags.c_contiguous and vel.shape == (D, n, k)
    ps = p.c_struct()
    rc = lib().orc_iteration(ctypes.byref(ps), _ptr(tt), _ptr(A), _ptr(Wd), _ptr(vel), _ptr(c), _ptr(f),
                             _ptr(fc), _ptr(fe), _ptr(gS), _ptr(gW), _ptr(ld))
    if rc < 0:
        raise RuntimeError(f"oracle iteration failed: {rc}")
    return IterResult(rc, Wd, int(tt[0]), c, f, fc, fe, gS if rc == 0 else None,
                      gW if rc == 0 else None, int(ld[0]))


def run(p: Params, t: int, A: np.ndarray, W: np.ndarray, max_steps: int):
    """Algorithm loop; returns (W, t, steps_done, legal_d, colours of the legal member or None)."""
    A = _c(A, np.uint8)
    Wd = np.array(W, dtype=np.float64, copy=True)
    tt = np.array([t], dtype=np.int64)
    ld = np.zeros(1, np.int32)
    col = np.zeros(p.n, np.int16)
    ps = p.c_struct()
    done = lib().orc_run(ctypes.byref(ps), _ptr(tt), _ptr(A), _ptr(Wd), int(max_steps), _ptr(ld),
                         _ptr(col))
    if done < 0:
        raise RuntimeError(f"oracle run failed: {done}")
    return Wd, int(tt[0]), done, int(ld[0]), (col if ld[0] >= 0 else None)


# ---- multicolouring (problem 5): vertex i takes demand[i] colours ----

MCOL = 5


def select(W: np.ndarray, demand: Optional[np.ndarray] = None) -> np.ndarray:
    """Step 1 of multicolouring: in each row the demand[i] colours of largest weight (lower
    colour first on ties); multi-hot uint8 [D, n, k]."""
    W = _c(W, np.float64)
    D, n, k = W.shape
    S = np.zeros((D, n, k), dtype=np.uint8)
    dem = None if demand is None else _c(demand, np.int32)
    rc = lib().orc_select(D, n, k, _ptr(W), _ptr(dem), _ptr(S))
    if rc == -5:
        raise FloatingPointError("non-finite weight")
    if rc:
        raise ValueError("demand outside 1..k")
    return S


def fcolor_multi(A: np.ndarray, S: np.ndarray) -> np.ndarray:
    A = _c(A, np.uint8)
    S = _c(S, np.uint8)
    D, n, k = S.shape
    f = np.zeros(D, dtype=np.int64)
    lib().orc_fcolor_multi(D, n, k, _ptr(A), _ptr(S), _ptr(f))
    return f


def mtilde_multi(S: np.ndarray) -> np.ndarray:
    S = _c(S, np.uint8)
    D, n, k = S.shape
    M = np.zeros((n, n), dtype=np.int32)
    lib().orc_mtilde_multi(D, n, k, _ptr(S), _ptr(M))
    return M


def class_sizes_multi(S: np.ndarray) -> np.ndarray:
    S = _c(S, np.uint8)
    D, n, k = S.shape
    V = np.zeros((D, k), dtype=np.int32)
    lib().orc_class_sizes_multi(D, n, k, _ptr(S), _ptr(V))
    return V


def grad_s_multi(p: Params, t: int, A, S, Mt) -> np.ndarray:
    A = _c(A, np.uint8); S = _c(S, np.uint8); Mt = _c(Mt, np.int32)
    g = np.zeros((p.D, p.n, p.k), dtype=np.float64)
    ps = p.c_struct()
    lib().orc_grad_s_multi(ctypes.byref(ps), int(t), _ptr(A), _ptr(S), _ptr(Mt), _ptr(g))
    return g


@dataclass
class MultiIterResult:
    status: int                 # 1 = legal member found (no update), 0 = updated
    W: np.ndarray
    t: int
    S: np.ndarray               # the selection of step 1
    f_color: np.ndarray
    gS: Optional[np.ndarray]
    gW: Optional[np.ndarray]
    legal_d: int


def iteration_multi(p: Params, t: int, A: np.ndarray, W: np.ndarray, demand: Optional[np.ndarray] = None,
                    want_grads: bool = True) -> MultiIterResult:
    """One multicolouring iteration (steps 1-4) from W (upcast to FP64)."""
    A = _c(A, np.uint8)
    Wd = np.array(W, dtype=np.float64, copy=True)
    D, n, k = Wd.shape
    dem = None if demand is None else _c(demand, np.int32)
    tt = np.array([t], dtype=np.int64)
    S = np.zeros((D, n, k), np.uint8)
    f = np.zeros(D, np.int64)
    gS = np.zeros((D, n, k)) if want_grads else None
    gW = np.zeros((D, n, k)) if want_grads else None
    ld = np.zeros(1, np.int32)
    ps = p.c_struct()
    rc = lib().orc_iteration_multi(ctypes.byref(ps), _ptr(tt), _ptr(A), _ptr(dem), _ptr(Wd), _ptr(S), _ptr(f),
                                   _ptr(gS), _ptr(gW), _ptr(ld))
    if rc < 0:
        raise RuntimeError(f"oracle multicolouring iteration failed: {rc}")
    return MultiIterResult(rc, Wd, int(tt[0]), S, f, gS if rc == 0 else None, gW if rc == 0 else None, int(ld[0]))
