"""GPU tests of the device initial weights and the colour-count descent driver, through the C ABI.

The descent (solve k-COL for decreasing k, Sections 1 and 3) is checked against an
oracle driver that repeats the same schedule with the FP64 oracle iteration on the
same initial weights, and on Mycielski graphs, whose chromatic number is known by
construction.
"""
import numpy as np
import pytest

import oracle
import tcolgen
from tcolgen import ECP, FP32, KCOL, GraphCase

from gpu_util import orc_params

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy()


def _pk():
    import paper_1909_02261_amd as pk
    return pk


@pytest.mark.parametrize("D,n,k,seed", [(3, 17, 5, 7), (2, 33, 11, 12345678901), (1, 1, 1, 0)])
def test_init_weights_matches_generator(D, n, k, seed):
    """Device Philox4x32-10 + Box-Muller against the host generator: the same draws, so the
    values agree to the last fp32 bit except where the FP64 libm results round differently."""
    torch = __import__("torch")
    pk = _pk()
    W = torch.empty(D * n * k, dtype=torch.float32, device="cuda")
    pk.init_weights(W, seed, 0.01)
    got = host(W)
    ref = tcolgen.weights0(D, n, k, seed).reshape(-1)
    ulp = np.spacing(np.abs(ref).astype(np.float32))
    assert np.all(np.abs(got - ref) <= ulp)
    assert np.mean(got == ref) >= 0.999


def _oracle_descent(case_params, A, k_first, k_min, max_steps, seed, sigma0=0.01):
    """The descent schedule with the FP64 oracle: one attempt per k from the same weights."""
    best, steps_best, col_best, tried = -1, 0, None, 0
    for k in range(k_first, k_min - 1, -1):
        d = dict(case_params, k=k, stop_on_legal=1)
        p = orc_params(d)
        W0 = tcolgen.weights0(d["D"], d["n"], k, seed + 1000003 * k, sigma0)
        tried += 1
        _, _, done, legal_d, col = oracle.run(p, 0, A, W0, max_steps)
        if legal_d < 0:
            break
        best, steps_best, col_best = k, done + 1, col
    return best, steps_best, col_best, tried


@pytest.mark.parametrize("graph_seed", [41, 42])
def test_descent_matches_oracle_driver(graph_seed):
    torch = __import__("torch")
    pk = _pk()
    n, D = 40, 4
    A = tcolgen.gnp(n, 0.3, graph_seed)
    k_first = tcolgen.greedy_colour_count(A) + 1
    case = GraphCase("desc", KCOL, n, k_first, D, FP32, "gnp", 0.3, graph_seed=graph_seed, rho=10.0, lam=1e-3,
                     mu=1e-4)
    prm = case.params()
    res, col = pk.descent(torch.from_numpy(A).cuda(), pk.Params.from_dict(prm), k_first, 1, max_steps=300,
                          attempts=1, seed=11)
    best, steps_best, col_ref, tried = _oracle_descent(prm, A, k_first, 1, 300, 11)
    print(f"gpu {res} oracle k_best {best} steps {steps_best} tried {tried}")
    assert res["k_best"] == best and res["k_tried"] == tried
    assert res["steps_best"] == steps_best
    assert col is not None
    c = host(col).astype(np.int16)
    assert np.array_equal(c, col_ref)
    assert int(oracle.fcolor(A, c[None, :])[0]) == 0 and c.max() < best


@pytest.mark.parametrize("m", [4, 5])
def test_descent_reaches_chromatic_number_of_mycielski(m):
    """Mycielski M_m has chromatic number m: the descent must stop exactly there (m - 1
    colours admit no legal colouring), with a legal m-colouring."""
    torch = __import__("torch")
    pk = _pk()
    A = tcolgen.mycielski(m)
    n = A.shape[0]
    prm = pk.Params(n=n, k=m + 2, D=8, precision=FP32, rho=10.0, lam=1e-3, mu=1e-4)
    res, col = pk.descent(torch.from_numpy(A).cuda(), prm, m + 2, 2, max_steps=2000, attempts=2, seed=5)
    print(f"M{m}: {res}")
    assert res["k_best"] == m and res["k_tried"] == 4
    c = host(col)
    assert int(oracle.fcolor(A, c[None, :].astype(np.int16))[0]) == 0 and c.max() < m


def test_descent_ecp_planted():
    """ECP descent on a planted equitable 6-partite graph: the colouring returned is legal and
    equitable for k_best colours, and k_best is at most the planted 6."""
    torch = __import__("torch")
    pk = _pk()
    P = tcolgen.planted(60, 6, 19, density=0.4)
    prm = pk.Params(n=60, k=8, D=8, problem=ECP, precision=FP32, rho=10.0, lam=1e-3, mu=0.0, nu=1e-3)
    res, col = pk.descent(torch.from_numpy(P.A).cuda(), prm, 8, 6, max_steps=3000, attempts=2, seed=9)
    print(f"ECP planted: {res}")
    assert res["k_best"] == 6
    c = host(col).astype(np.int16)
    assert int(oracle.fcolor(P.A, c[None, :])[0]) == 0
    V = oracle.class_sizes(c[None, :], 6)
    assert int(oracle.feq(V, 60)[0]) == 0


def test_descent_rejects_bad_options():
    torch = __import__("torch")
    pk = _pk()
    A = torch.from_numpy(tcolgen.mycielski(3)).cuda()
    prm = pk.Params(n=5, k=3, D=2)
    for kw in (dict(k_first=3, k_min=4), dict(k_first=0), dict(k_first=3, max_steps=0), dict(k_first=3, attempts=0),
               dict(k_first=3, sigma0=0.0)):
        with pytest.raises(pk.TcolError) as ei:
            pk.descent(A, prm, **kw)
        assert ei.value.status == -1
