"""CPU checks of the helpers the GPU tests build their reference steps with: bf16 rounding
against torch's round-to-nearest-even conversion, the class products against one-hot matrix
products, and the penalty operand against the oracle's own gradient (which the oracle pins
tie to the paper)."""
import numpy as np
import pytest

import oracle
import tcolgen
from tcolgen import FP32, KCOL, KPART, GraphCase

from gpu_util import bf16_rne, class_product, operand_values, orc_params


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-20, 20, 20000),
                        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, -0.0,
                                  3.3895314e38], np.float32)]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(bf16_rne(x), want)


def test_class_product_is_the_one_hot_product():
    rng = np.random.default_rng(1)
    n, k, D = 37, 6, 3
    X = rng.standard_normal((n, n))
    c = rng.integers(0, k, size=(D, n)).astype(np.int16)
    c[1] = 0                                           # a member with a single class
    got = class_product(X, c, k)
    for d in range(D):
        S = np.zeros((n, k))
        S[np.arange(n), c[d]] = 1.0
        assert np.allclose(got[d], X @ S, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("problem,bonus_diag", [(KCOL, 1), (KCOL, 0), (KPART, 1)])
def test_operand_times_s_is_the_oracle_penalty_term(problem, bonus_diag):
    """sgn P . S equals the oracle's gradient minus its gradient with lambda = mu = 0."""
    case = GraphCase("pen", problem, 40, 5, 4, FP32, "gnp", 0.5, graph_seed=3, lam=1e-2, mu=3e-3,
                     bonus_diag=bonus_diag)
    A = case.adjacency()
    p = orc_params(case.params())
    p0 = orc_params(dict(case.params(), lam=0.0, mu=0.0))
    c = oracle.colors(case.weights().astype(np.float64))
    Mt = oracle.mtilde(c)
    V = oracle.class_sizes(c, case.k)
    t = 7
    diff = oracle.grad_s(p, t, A, c, Mt, V) - oracle.grad_s(p0, t, A, c, Mt, V)
    sgn = -1.0 if problem == KPART else 1.0
    got = sgn * class_product(operand_values(p, t, A, Mt, "fp64"), c, case.k)
    assert np.allclose(got, diff, rtol=1e-12, atol=1e-15)
    # the fp32 and bf16 forms stay within their unit roundoff of the FP64 values
    P64 = operand_values(p, t, A, Mt, "fp64")
    for form, u in (("fp32", 2.0 ** -23), ("bf16", 2.0 ** -8 + 2.0 ** -23)):
        P = operand_values(p, t, A, Mt, form)
        assert np.all(np.abs(P - P64) <= u * np.abs(P64) + 1e-300)
