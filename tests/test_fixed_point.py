"""The sparse penalty rows sum the FP32 values of the penalty operand in 64-bit fixed
point: every value times 2^sc, with sc = 62 - (E1 + bits(n)) where |P| < 2^E1 (the
largest exponent of the table t * 2 alpha lambda x^(alpha-1), -t * 2 beta mu x^(beta-1),
x = 0..D, rounded to FP32 as the kernels form it) and n < 2^bits(n).  This checks, over
the paper's parameter grid (Section 5: alpha, beta, lambda, mu) and the sizes the
library accepts, the two properties the kernels rely on: no row sum can overflow, and
the table is exactly representable (integer sums are then the exact sums of the FP32
terms, in any order) whenever its exponents span at most 38 - bits(n); otherwise each
term is rounded at 2^-sc, far below the final FP32 rounding of a row.  It restates
the scale rule on the host; the GPU parity tests check the kernels' sums."""
import itertools

import numpy as np


def table(alpha, beta, lam, mu, D, partition, t):
    x = np.arange(D + 1, dtype=np.float64)
    if partition:
        x = D - x
    with np.errstate(divide="ignore"):
        pen = np.where(x > 0, 2.0 * alpha * lam * x ** (alpha - 1.0), 0.0).astype(np.float32)
        bon = np.where(x > 0, 2.0 * beta * mu * x ** (beta - 1.0), 0.0).astype(np.float32)
    tf = np.float32(t)
    return np.concatenate([-(tf * bon), tf * pen]).astype(np.float32)


def test_fixed_point_scale_over_the_parameter_grid():
    worst_rel = 0.0
    n_exact = n_total = 0
    for alpha, beta, lam, mu, D, n, t, part in itertools.product(
            (1.5, 2.0, 2.5), (1.2, 1.5, 2.0), (1e-4, 1e-5, 1e-6), (1e-5, 1e-6, 1e-7),
            (8, 32, 200, 1024), (125, 4000, 32768), (1, 100, 100000), (False, True)):
        v = table(alpha, beta, lam, mu, D, part, t)
        nz = v[v != 0]
        _, e = np.frexp(nz)
        E1, E2 = int(e.max()), int(n).bit_length()
        sc = 62 - (E1 + E2)
        q = nz.astype(np.float64) * 2.0 ** sc
        # no overflow: a row adds at most n terms of at most max|q|
        assert n * (np.abs(q).max() + 0.5) < 2.0 ** 63
        exact = bool(np.all(q == np.round(q)))
        span = int(e.max() - e.min())
        if span <= 38 - E2:
            assert exact, (alpha, beta, lam, mu, D, n, t, part)
        n_exact += exact
        n_total += 1
        # rounding of a row (n terms, each within 2^-(sc+1)) relative to max|P|
        worst_rel = max(worst_rel, n * 2.0 ** (-sc - 1) / float(np.abs(nz).max()))
    assert worst_rel < 2.0 ** -30
    # at the benchmark's n = 4000 every setting of the grid is exact
    print(f"{n_exact}/{n_total} settings exact; worst row rounding {worst_rel:.1e} of max|P|")


def test_fixed_point_exact_at_n4000():
    for alpha, beta, lam, mu, D, t, part in itertools.product(
            (1.5, 2.0, 2.5), (1.2, 1.5, 2.0), (1e-4, 1e-5, 1e-6), (1e-5, 1e-6, 1e-7),
            (8, 32, 200, 1024), (1, 100, 100000), (False, True)):
        v = table(alpha, beta, lam, mu, D, part, t)
        nz = v[v != 0]
        _, e = np.frexp(nz)
        sc = 62 - (int(e.max()) + int(4000).bit_length())
        q = nz.astype(np.float64) * 2.0 ** sc
        assert np.all(q == np.round(q))
