"""The allocation-free entry point tcol_conflicts_noalloc, called through the C ABI, against
tcol_conflicts of a context built on the same graph and weights: colours, main and added
fitness bit-exact, on consecutive calls whose second input is smaller than the first (the
shared scratch array keeps the first call's contents), for k-colouring, the ECP and
k-partitioning (whose cut needs the edge count the call takes from the scratch)."""
import ctypes

import numpy as np
import pytest

import tcolgen
from tcolgen import BF16, ECP, FP4, FP8, FP32, KCOL, KPART, GraphCase

from gpu_util import host, make_solver

pytestmark = pytest.mark.gpu


def noalloc(case, A_t, W_t):
    """One call of tcol_conflicts_noalloc through ctypes on the current stream."""
    torch = __import__("torch")
    import paper_1909_02261_amd as pk
    from paper_1909_02261_amd import _lib
    lib = _lib.load()
    p = pk.Params.from_dict(case.params()).c_struct()
    c = torch.full((case.D, case.n), -7, dtype=torch.int16, device="cuda")
    fm = torch.full((case.D,), -7, dtype=torch.int64, device="cuda")
    fs = torch.full((case.D,), -7, dtype=torch.int64, device="cuda")
    st = lib.tcol_conflicts_noalloc(ctypes.byref(p), ctypes.c_void_p(A_t.data_ptr()), ctypes.c_void_p(W_t.data_ptr()),
                                    ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(fm.data_ptr()),
                                    ctypes.c_void_p(fs.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    torch.cuda.synchronize()
    return host(c), host(fm), host(fs)


def with_context(case, A, W):
    s, _ = make_solver([case], As=[A], Ws=[W])
    c, fm, fs = (host(x) for x in s.conflicts(0))
    s.close()
    return c, fm, fs


PAIRS = [
    (GraphCase("big_kcol", KCOL, 1000, 28, 40, FP4, "gnp", 0.5, graph_seed=13),
     GraphCase("small_kcol", KCOL, 300, 30, 12, BF16, "gnp", 0.4, graph_seed=14)),
    (GraphCase("big_ecp", ECP, 777, 61, 9, FP8, "gnp", 0.5, graph_seed=15, mu=0.0, nu=1e-5),
     GraphCase("small_ecp", ECP, 150, 11, 6, FP32, "gnp", 0.5, graph_seed=8, mu=0.0, nu=1e-5)),
    (GraphCase("big_kpart", KPART, 600, 5, 16, FP4, "gnp", 0.3, graph_seed=16),
     GraphCase("small_kpart", KPART, 77, 4, 3, FP4, "gnp", 0.6, graph_seed=17)),
]


@pytest.mark.parametrize("pair", PAIRS, ids=[p[0].problem for p in PAIRS])
def test_noalloc_matches_context_on_two_calls(pair):
    torch = __import__("torch")
    for case in pair:                       # the second call's input is the smaller one
        A = case.adjacency()
        W = case.weights()
        # a few exact ties and colours of large index, so the argmax convention is exercised
        W[0, :5, :] = 0.0
        W[-1, 3, case.k - 1] = 1.0
        A_t = torch.from_numpy(A).cuda()
        W_t = torch.from_numpy(W).cuda()
        got = noalloc(case, A_t, W_t)
        want = with_context(case, A, W)
        for g, w, what in zip(got, want, ("colours", "main fitness", "added fitness")):
            assert np.array_equal(g, w), (case.name, what)


def test_noalloc_c5_size():
    """The largest size the scratch holds: the n = 4000, k = 280, D = 32 workload."""
    torch = __import__("torch")
    case = tcolgen.case_c5(FP4)
    A = case.adjacency()
    W = case.weights()
    got = noalloc(case, torch.from_numpy(A).cuda(), torch.from_numpy(W).cuda())
    want = with_context(case, A, W)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
