"""ctypes declarations of libtcol's C ABI (include/tcol.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtcol.so")

TCOL_OK = 0
STATUS = {0: "TCOL_OK", -1: "TCOL_EINVAL", -2: "TCOL_ESHAPE", -3: "TCOL_EGRAPH", -4: "TCOL_EHIP",
          -5: "TCOL_ENONFINITE", -6: "TCOL_ENOMEM", -7: "TCOL_ESTATE", -8: "TCOL_EABORT"}

KCOL, ECP, KPART, BKPART, MSCP, MCOL = 0, 1, 2, 3, 4, 5
FP32, BF16, FP8, FP4 = 0, 1, 2, 3


class GraphParams(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int32), ("precision", ctypes.c_int32), ("n", ctypes.c_int32),
                ("k", ctypes.c_int32), ("D", ctypes.c_int32), ("eta", ctypes.c_float),
                ("rho", ctypes.c_float), ("nb_iter", ctypes.c_int32), ("alpha", ctypes.c_float),
                ("lambda_", ctypes.c_float), ("beta", ctypes.c_float), ("mu", ctypes.c_float),
                ("nu", ctypes.c_float), ("bonus_diag", ctypes.c_int32), ("stop_on_legal", ctypes.c_int32),
                ("momentum", ctypes.c_float), ("max_demand", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("fused", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("tile_bm", ctypes.c_int32), ("tile_ntw", ctypes.c_int32), ("penalty", ctypes.c_int32)]


class DescentOptions(ctypes.Structure):
    _fields_ = [("k_first", ctypes.c_int32), ("k_min", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("attempts", ctypes.c_int32), ("seed", ctypes.c_uint64), ("sigma0", ctypes.c_double)]


class DescentResult(ctypes.Structure):
    _fields_ = [("k_best", ctypes.c_int32), ("k_tried", ctypes.c_int32), ("attempt_best", ctypes.c_int32),
                ("steps_best", ctypes.c_int32), ("steps_total", ctypes.c_int64)]


class TcolError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({_strerror(status)})")


EXPORTS = ["tcol_status_string", "tcol_workspace_size", "tcol_init", "tcol_set_options",
           "tcol_get_options", "tcol_step", "tcol_conflicts", "tcol_loss_grad", "tcol_mtilde",
           "tcol_get_t", "tcol_set_t", "tcol_reset", "tcol_autotune", "tcol_profile", "tcol_destroy",
           "tcol_init_weights", "tcol_descent", "tcol_mfma_peak", "tcol_get_counters", "tcol_conflicts_noalloc",
           "tcol_class_conflicts", "tcol_set_demand", "tcol_selection", "tcol_set_wait_limit", "tcol_cancel"]
NPHASES = 10
PHASES = ["colors", "class_sizes", "expand", "mtilde", "gemm", "fitness", "update", "advance", "gemm_as_only",
          "gemm_as_store"]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libtcol.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libtcol.so not found at {path}; build it with "
                          f"`python -m paper_1909_02261_amd.build` (hipcc, gfx950)")
    # torch first: libtcol must bind to the HIP runtime that torch's tensors and streams live in
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.tcol_status_string.argtypes = [i32]
    lib.tcol_status_string.restype = ctypes.c_char_p
    lib.tcol_workspace_size.argtypes = [i32, ctypes.POINTER(GraphParams), ctypes.POINTER(ctypes.c_size_t)]
    lib.tcol_init.argtypes = [ctypes.POINTER(P), i32, ctypes.POINTER(GraphParams), ctypes.POINTER(P),
                              ctypes.POINTER(P), P, ctypes.c_size_t, P]
    lib.tcol_set_options.argtypes = [P, ctypes.POINTER(Options)]
    lib.tcol_get_options.argtypes = [P, ctypes.POINTER(Options)]
    lib.tcol_step.argtypes = [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(P)]
    lib.tcol_conflicts.argtypes = [P, i32, P, P, P]
    lib.tcol_loss_grad.argtypes = [P, i32, P, P, P]
    lib.tcol_mtilde.argtypes = [P, i32, P]
    lib.tcol_class_conflicts.argtypes = [P, i32, P]
    lib.tcol_set_demand.argtypes = [P, i32, P]
    lib.tcol_selection.argtypes = [P, i32, P]
    lib.tcol_get_t.argtypes = [P, i32, ctypes.POINTER(i64)]
    lib.tcol_set_t.argtypes = [P, i32, i64]
    lib.tcol_reset.argtypes = [P]
    lib.tcol_set_wait_limit.argtypes = [P, i32]
    lib.tcol_cancel.argtypes = [P]
    lib.tcol_get_counters.argtypes = [P, i32, ctypes.POINTER(i64)]
    lib.tcol_conflicts_noalloc.argtypes = [ctypes.POINTER(GraphParams), P, P, P, P, P, P]
    lib.tcol_autotune.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.tcol_profile.argtypes = [P, i32, i32, ctypes.POINTER(ctypes.c_float)]
    lib.tcol_mfma_peak.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_double)]
    lib.tcol_init_weights.argtypes = [P, i64, ctypes.c_uint64, ctypes.c_double, P]
    lib.tcol_descent.argtypes = [P, ctypes.POINTER(GraphParams), ctypes.POINTER(DescentOptions),
                                 ctypes.POINTER(DescentResult), P, P]
    lib.tcol_destroy.argtypes = [P]
    lib.tcol_destroy.restype = None
    for name in EXPORTS:
        if name not in ("tcol_status_string", "tcol_destroy"):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _strerror(status: int) -> str:
    try:
        return load().tcol_status_string(status).decode()
    except Exception:
        return "?"


def check(status: int, what: str) -> None:
    if status != TCOL_OK:
        raise TcolError(status, what)
