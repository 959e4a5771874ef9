"""Host-side checks of libtcol: the C ABI loads, exports every declared entry point,
and validates arguments before touching the GPU (no compute call here)."""
import ctypes
import os
import re

import pytest

from paper_1909_02261_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tcol.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tcol_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1909_02261_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(_lib.EXPORTS)


def params(**kw):
    d = dict(problem=0, precision=0, n=100, k=10, D=4, eta=1e-3, rho=10.0, nb_iter=5, alpha=2.5,
             lambda_=1e-5, beta=1.2, mu=1e-6, nu=0.0, bonus_diag=1, stop_on_legal=1)
    d.update(kw)
    return _lib.GraphParams(**d)


def ws(lib, *ps):
    arr = (_lib.GraphParams * len(ps))(*ps)
    b = ctypes.c_size_t(0)
    st = lib.tcol_workspace_size(len(ps), arr, ctypes.byref(b))
    return st, b.value


def test_workspace_size_and_validation(lib):
    st, b1 = ws(lib, params())
    assert st == 0 and b1 > 0
    st, b2 = ws(lib, params(n=1000, k=90, D=256, precision=1))
    assert st == 0 and b2 > b1
    # two graphs need at least the sum of their regions
    st, b12 = ws(lib, params(), params(n=1000, k=90, D=256, precision=1))
    assert st == 0 and b12 >= b1 + b2 - 4096
    # FP8 keeps a bf16 copy of S for the penalty pass
    st, b8 = ws(lib, params(n=1000, k=90, D=256, precision=2))
    assert st == 0 and b8 > 0
    assert ws(lib, params(n=0))[0] == -2
    assert ws(lib, params(k=0))[0] == -2
    assert ws(lib, params(D=5000))[0] == -2
    assert ws(lib, params(n=40000))[0] == -2
    assert ws(lib, params(precision=7))[0] == -1
    for prob in (1, 2, 3, 4):                           # ECP, (balanced) k-partitioning, min-sum colouring
        assert ws(lib, params(problem=prob))[0] == 0
    assert ws(lib, params(problem=5))[0] == -1
    assert ws(lib, params(problem=-1))[0] == -1
    assert ws(lib, params(momentum=1.0))[0] == -1       # heavy-ball coefficient in [0, 1)
    assert ws(lib, params(momentum=-0.1))[0] == -1
    st, bm = ws(lib, params(momentum=0.9))              # the velocity lives in the workspace
    assert st == 0 and bm >= b1 + 4 * 4 * 100 * 10
    assert ws(lib, params(alpha=1.0))[0] == -1          # lambda > 0 needs alpha > 1
    assert ws(lib, params(alpha=1.0, lambda_=0.0))[0] == 0
    assert ws(lib, params(beta=0.5))[0] == -1           # mu > 0 needs beta > 1
    assert ws(lib, params(eta=0.0))[0] == -1
    assert ws(lib, params(rho=0.5))[0] == -1
    assert ws(lib, params(nb_iter=0))[0] == -1
    assert ws(lib, params(mu=-1.0))[0] == -1
    assert lib.tcol_workspace_size(0, None, None) == -1


def test_init_rejects_bad_arguments_without_gpu(lib):
    ctx = ctypes.c_void_p()
    p = (_lib.GraphParams * 1)(params())
    assert lib.tcol_init(ctypes.byref(ctx), 1, p, None, None, None, 0, None) == -1
    assert ctx.value is None
    A = (ctypes.c_void_p * 1)(None)
    W = (ctypes.c_void_p * 1)(None)
    assert lib.tcol_init(ctypes.byref(ctx), 1, p, A, W, None, 0, None) == -1
    bad = (_lib.GraphParams * 1)(params(k=0))
    A = (ctypes.c_void_p * 1)(1)
    W = (ctypes.c_void_p * 1)(1)
    assert lib.tcol_init(ctypes.byref(ctx), 1, bad, A, W, None, 0, None) == -2
    # workspace given but too small
    assert lib.tcol_init(ctypes.byref(ctx), 1, p, A, W, ctypes.c_void_p(1), 16, None) == -6
    # every call rejects a NULL context
    assert lib.tcol_step(None, 1, None, None, None) == -1
    assert lib.tcol_conflicts(None, 0, None, None, None) == -1
    assert lib.tcol_loss_grad(None, 0, None, None, None) == -1
    assert lib.tcol_mtilde(None, 0, None) == -1
    assert lib.tcol_set_t(None, 0, 0) == -1
    assert lib.tcol_reset(None) == -1
    assert lib.tcol_cancel(None) == -1
    assert lib.tcol_set_wait_limit(None, 0) == -1
    lib.tcol_destroy(None)
    # the colour-count descent is for colouring problems only (checked before any device work)
    dopt = _lib.DescentOptions(10, 1, 100, 1, 0, 0.01)
    dres = _lib.DescentResult()
    for prob in (2, 3, 4):
        bp = params(problem=prob)
        assert lib.tcol_descent(ctypes.c_void_p(1), ctypes.byref(bp), ctypes.byref(dopt), ctypes.byref(dres),
                                None, None) == -1


def test_status_strings(lib):
    for code in range(-8, 1):
        assert lib.tcol_status_string(code)
    assert b"non-finite" in lib.tcol_status_string(-5)


def test_binding_fails_loudly_without_library(tmp_path):
    import importlib
    old = _lib._lib
    try:
        _lib._lib = None
        with pytest.raises(ImportError):
            _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._lib = old


def test_mfma_peak_rejects_bad_arguments_without_gpu(lib):
    """tcol_mfma_peak validates its arguments before any HIP call."""
    out = ctypes.c_double(0.0)
    assert lib.tcol_mfma_peak(3, 10, None) == -1       # TCOL_EINVAL
    assert lib.tcol_mfma_peak(3, 0, ctypes.byref(out)) == -1
    assert lib.tcol_mfma_peak(4, 10, ctypes.byref(out)) == -1
    assert lib.tcol_mfma_peak(-1, 10, ctypes.byref(out)) == -1


def test_noalloc_rejects_what_its_scratch_cannot_hold(lib):
    """tcol_conflicts_noalloc checks its arguments and the size its fixed scratch array holds
    before touching any device (the pointers below are never dereferenced)."""
    dummy = ctypes.c_void_p(16)
    big = params(n=8000, k=500, D=64)
    assert lib.tcol_conflicts_noalloc(ctypes.byref(big), dummy, dummy, None, None, None, None) == -6
    small = params()
    assert lib.tcol_conflicts_noalloc(ctypes.byref(small), None, dummy, None, None, None, None) == -1
    assert lib.tcol_conflicts_noalloc(None, dummy, dummy, None, None, None, None) == -1
    bad = params(k=0)
    assert lib.tcol_conflicts_noalloc(ctypes.byref(bad), dummy, dummy, None, None, None, None) == -2


def test_multicolouring_parameters(lib):
    """Multicolouring (problem 5) needs 1 <= max_demand <= min(8, k) and no momentum; other
    problems take max_demand 0 or 1."""
    assert ws(lib, params(problem=5, max_demand=3))[0] == 0
    assert ws(lib, params(problem=5, max_demand=1))[0] == 0
    assert ws(lib, params(problem=5, max_demand=0))[0] == -1
    assert ws(lib, params(problem=5, max_demand=9, k=20))[0] == -1
    assert ws(lib, params(problem=5, max_demand=4, k=3))[0] == -1
    assert ws(lib, params(problem=5, max_demand=2, momentum=0.5))[0] == -1
    assert ws(lib, params(problem=0, max_demand=2))[0] == -1
    assert ws(lib, params(problem=6))[0] == -1
    # the selection slots make the workspace grow with max_demand
    assert ws(lib, params(problem=5, max_demand=4))[1] > ws(lib, params(problem=5, max_demand=1))[1]
