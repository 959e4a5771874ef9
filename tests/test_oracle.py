"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each test checks it against a
value the paper prints, a closed form, a second formulation (the literal
tensor transcription, brute force over edges or colourings), an invariance
the paper states, or finite differences.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import literal
import tcolgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def onehot(c, k):
    c = np.asarray(c)
    D, n = c.shape
    S = np.zeros((D, n, k))
    for d in range(D):
        S[d, np.arange(n), c[d]] = 1.0
    return S


def adj_from_edges(n, edges):
    A = np.zeros((n, n), np.uint8)
    for i, j in edges:
        A[i, j] = A[j, i] = 1
    return A


def rand_params(problem, n, k, D, **kw):
    d = dict(problem=problem, n=n, k=k, D=D, eta=1e-3, rho=10.0, nb_iter=5, alpha=2.5,
             lam=1e-2, beta=1.2, mu=3e-3, nu=0.05, bonus_diag=1, stop_on_legal=1)
    d.update(kw)
    return oracle.Params(**d)


def colour_weights(c, k, rng, scale=1.0):
    """Weights whose argmax is the colouring c (other entries strictly smaller)."""
    c = np.asarray(c)
    D, n = c.shape
    W = rng.uniform(-1.0, 0.0, size=(D, n, k))
    for d in range(D):
        W[d, np.arange(n), c[d]] = 1.0 + rng.uniform(0, 1, size=n)
    return W * scale


# ---------------------------------------------------------------- step 1 -----

def test_argmax_ties_lowest_and_nonfinite():
    W = np.zeros((2, 3, 4))
    W[0, 0] = [1, 3, 3, 2]      # tie between colours 1 and 2 -> 1
    W[0, 1] = [5, 5, 5, 5]      # all equal -> 0
    W[0, 2] = [-1, -2, -1, 0.5]
    W[1, 0] = [0, 0, 0, 1e-30]
    W[1, 1] = [-0.0, 0.0, -1, -1]  # -0 == +0 -> 0
    W[1, 2] = [2, 1, 2, 1]
    c = oracle.colors(W)
    assert c.tolist() == [[1, 0, 3], [3, 0, 0]]
    W[1, 2, 3] = np.nan
    with pytest.raises(FloatingPointError):
        oracle.colors(W)
    W[1, 2, 3] = np.inf
    with pytest.raises(FloatingPointError):
        oracle.colors(W)


def test_argmax_matches_literal_one_hot():
    rng = np.random.default_rng(5)
    W = rng.standard_normal((3, 17, 6))
    c = oracle.colors(W)
    S = literal.one_hot_argmax(W)
    assert np.array_equal(onehot(c, 6), S)


# ---------------------------------------------------------------- step 2 -----

@pytest.mark.parametrize("n,k,seed", [(4, 3, 0), (5, 3, 1), (6, 2, 2), (6, 3, 3)])
def test_fcolor_exhaustive_all_colourings(n, k, seed):
    """Every one of the k^n colourings: the oracle's edge count equals the paper's
    1/2 sum(A o S S') (literal) and a brute force written here over the edge list."""
    A = tcolgen.gnp(n, 0.6, seed)
    cols = np.array(list(itertools.product(range(k), repeat=n)), dtype=np.int16)
    f = oracle.fcolor(A, cols)
    f_lit = literal.fitness_color(A.astype(float), onehot(cols, k))
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if A[i, j]]
    f_bf = np.array([sum(1 for i, j in edges if c[i] == c[j]) for c in cols])
    assert np.array_equal(f, f_bf)
    assert np.array_equal(f, f_lit.astype(np.int64))
    # a legal colouring exists iff min f == 0; chromatic number by exhaustion
    assert (f.min() == 0) == any(all(c[i] != c[j] for i, j in edges) for c in cols)


def test_fcolor_complete_graph_one_colour():
    for n in (1, 2, 7, 12):
        A = np.ones((n, n), np.uint8) - np.eye(n, dtype=np.uint8)
        c = np.zeros((1, n), np.int16)
        assert oracle.fcolor(A, c)[0] == n * (n - 1) // 2


def test_fitness_zero_on_planted_colouring():
    P = tcolgen.planted(200, 9, seed=11)
    c = P.classes[None, :]
    assert oracle.fcolor(P.A, c)[0] == 0
    V = oracle.class_sizes(c, 9)
    assert oracle.feq(V, 200)[0] == 0
    # and a perturbed colouring has conflicts
    c2 = c.copy()
    i = int(np.nonzero(P.A[0])[0][0])
    c2[0, i] = c2[0, 0]
    assert oracle.fcolor(P.A, c2)[0] >= 1


def test_feq_closed_forms():
    # n=10, k=3, all vertices in one class: c1=3, c2=4 -> (10-4) + 2*3 = 12
    assert oracle.equity_bounds(10, 3) == (3, 4)
    V = np.array([[10, 0, 0]], np.int32)
    assert oracle.feq(V, 10)[0] == 12
    # k divides n: c1 = c2 = n/k
    assert oracle.equity_bounds(12, 3) == (4, 4)
    assert oracle.feq(np.array([[12, 0, 0]], np.int32), 12)[0] == 8 + 4 + 4
    assert oracle.feq(np.array([[4, 4, 4]], np.int32), 12)[0] == 0
    # general: equals sum_l max(0, c1 - V) + max(0, V - c2) for integer V
    rng = np.random.default_rng(3)
    for _ in range(50):
        n = int(rng.integers(1, 60)); k = int(rng.integers(1, 12))
        c = rng.integers(0, k, size=(4, n)).astype(np.int16)
        V = oracle.class_sizes(c, k)
        c1, c2 = n // k, -(-n // k)
        want = (np.maximum(0, c1 - V) + np.maximum(0, V - c2)).sum(axis=1)
        assert np.array_equal(oracle.feq(V, n), want)
        assert np.array_equal(oracle.feq(V, n), literal.equity_fitness(onehot(c, k)).astype(np.int64))
        # zero iff class sizes differ by at most one
        eqt = (V.max(axis=1) - V.min(axis=1)) <= 1
        assert np.array_equal(oracle.feq(V, n) == 0, eqt)


# ---------------------------------------------------------------- step 3 -----

def test_kappa_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "kappa_worked_example.json")))
    A = adj_from_edges(g["n"], g["edges"])
    for case in g["cases"]:
        c = np.array(case["colors"], np.int16)
        assert oracle.fcolor(A, c).tolist() == case["conflicts_per_member"]
        Mt = oracle.mtilde(c)
        p = oracle.Params(problem=0, n=g["n"], k=g["k"], D=c.shape[0], alpha=g["alpha"], lam=1.0,
                          beta=1.5, mu=0.0)
        out = oracle.loss(p, 1, A, Mt, oracle.fcolor(A, c), np.zeros(c.shape[0], np.int64))
        assert out[3] == case["kappa"]
        assert literal.kappa(A.astype(float), onehot(c, g["k"]), g["alpha"]) == case["kappa"]


def test_mtilde_properties():
    rng = np.random.default_rng(7)
    D, n, k = 6, 40, 5
    c = rng.integers(0, k, size=(D, n)).astype(np.int16)
    Mt = oracle.mtilde(c)
    assert np.array_equal(Mt, Mt.T)
    assert np.all(np.diag(Mt) == D)
    V = oracle.class_sizes(c, k)
    assert Mt.sum() == int((V.astype(np.int64) ** 2).sum())
    assert np.array_equal(Mt, literal.group_concentration(onehot(c, k)).astype(np.int32))
    # D = 1: Mt is the association matrix of the single member
    M1 = oracle.mtilde(c[:1])
    assert np.array_equal(M1, (c[0][:, None] == c[0][None, :]).astype(np.int32))


def test_kappa_varpi_single_member_identities():
    """D=1: kappa = 2 f_color; varpi = sum_l V_l^2 - 2 f_color (diagonal included), n less without."""
    rng = np.random.default_rng(1)
    for trial in range(10):
        n, k = int(rng.integers(5, 40)), int(rng.integers(2, 7))
        A = tcolgen.gnp(n, 0.4, 100 + trial)
        c = rng.integers(0, k, size=(1, n)).astype(np.int16)
        f = oracle.fcolor(A, c)
        V = oracle.class_sizes(c, k)
        Mt = oracle.mtilde(c)
        for diag in (1, 0):
            p = oracle.Params(problem=0, n=n, k=k, D=1, alpha=2.5, beta=1.2, lam=1, mu=1,
                              bonus_diag=diag)
            out = oracle.loss(p, 0, A, Mt, f, np.zeros(1, np.int64))
            assert out[3] == pytest.approx(2 * f[0], abs=1e-12)
            want = float((V.astype(float) ** 2).sum() - 2 * f[0] - (0 if diag else n))
            assert out[4] == pytest.approx(want, abs=1e-12)


def test_identical_copies_scale():
    """D identical members: Mt = D M, kappa = D^alpha 2f, varpi = D^beta (sum V^2 - 2f)."""
    rng = np.random.default_rng(2)
    n, k, D = 30, 4, 5
    A = tcolgen.gnp(n, 0.5, 9)
    c1 = rng.integers(0, k, size=(1, n)).astype(np.int16)
    c = np.repeat(c1, D, axis=0)
    Mt = oracle.mtilde(c)
    assert np.array_equal(Mt, D * oracle.mtilde(c1))
    f = oracle.fcolor(A, c)
    V = oracle.class_sizes(c1, k)
    p = oracle.Params(problem=0, n=n, k=k, D=D, alpha=2.5, beta=1.2)
    out = oracle.loss(p, 0, A, Mt, f, np.zeros(D, np.int64))
    assert out[3] == pytest.approx(D ** 2.5 * 2 * f[0], rel=1e-13)
    assert out[4] == pytest.approx(D ** 1.2 * ((V.astype(float) ** 2).sum() - 2 * f[0]), rel=1e-13)


def test_gamma_matrix_term():
    """At t = 0 the gradient is A.S: entry (d,i,l) counts the neighbours of i coloured l
    (the TabuCol gamma matrix); sum_i gS[d,i,c_d(i)] = 2 f_color(S_d)."""
    rng = np.random.default_rng(4)
    D, n, k = 3, 35, 6
    A = tcolgen.gnp(n, 0.3, 21)
    c = rng.integers(0, k, size=(D, n)).astype(np.int16)
    V = oracle.class_sizes(c, k)
    p = rand_params(1, n, k, D)
    gS = oracle.grad_s(p, 0, A, c, oracle.mtilde(c), V)
    gamma = np.zeros((D, n, k))
    for d in range(D):
        for i in range(n):
            for j in np.nonzero(A[i])[0]:
                gamma[d, i, c[d, j]] += 1
    assert np.array_equal(gS, gamma)
    f = oracle.fcolor(A, c)
    for d in range(D):
        assert gS[d, np.arange(n), c[d]].sum() == 2 * f[d]


@pytest.mark.parametrize("problem,diag", [(0, 1), (1, 1), (0, 0), (1, 0), (2, 1), (3, 1), (3, 0), (4, 1)])
def test_grad_s_matches_literal(problem, diag):
    rng = np.random.default_rng(10 + problem + 2 * diag)
    D, n, k = 4, 23, 5
    A = tcolgen.gnp(n, 0.5, 31)
    c = rng.integers(0, k, size=(D, n)).astype(np.int16)
    p = rand_params(problem, n, k, D, bonus_diag=diag)
    t = 7
    gS = oracle.grad_s(p, t, A, c, oracle.mtilde(c), oracle.class_sizes(c, k))
    lit = literal.grad_s(A.astype(float), onehot(c, k), t, p.alpha, p.lam, p.beta, p.mu, p.nu,
                         problem, diag)
    np.testing.assert_allclose(gS, lit, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("problem,diag", [(0, 1), (1, 1), (0, 0), (2, 1), (3, 1), (3, 0), (4, 1)])
def test_grad_s_finite_differences(problem, diag):
    """Central differences (h = 1e-3) of the paper's loss, as a polynomial in S, at the hard S."""
    rng = np.random.default_rng(20 + problem)
    D, n, k = 3, 14, 4
    A = tcolgen.gnp(n, 0.5, 41)
    c = rng.integers(0, k, size=(D, n)).astype(np.int16)
    p = rand_params(problem, n, k, D, bonus_diag=diag)
    t = 5
    gS = oracle.grad_s(p, t, A, c, oracle.mtilde(c), oracle.class_sizes(c, k))
    S = onehot(c, k)
    Af = A.astype(float)
    h = 1e-3

    def L(Sx):
        return literal.global_loss(Af, Sx, t, p.alpha, p.lam, p.beta, p.mu, p.nu, problem, diag)

    for (d, i, l) in tcolgen.fd_entries(32, D, n, k, seed=3):
        Sp = S.copy(); Sp[d, i, l] += h
        Sm = S.copy(); Sm[d, i, l] -= h
        fd = (L(Sp) - L(Sm)) / (2 * h)
        assert fd == pytest.approx(gS[d, i, l], rel=1e-4, abs=1e-6), (d, i, l)


# ---------------------------------------------------------------- step 4 -----

def test_grad_w_finite_differences_of_surrogate():
    """The straight-through gradient is the exact gradient of Phi(w) = sum_l G_l softmax(w)_l
    with G frozen; check by central differences, plus zero row sums and the constant-G case."""
    rng = np.random.default_rng(8)
    D, n, k = 2, 5, 7
    W = rng.standard_normal((D, n, k)) * 0.7
    G = rng.standard_normal((D, n, k)) * 3
    gW = oracle.grad_w(W, G)
    np.testing.assert_allclose(gW, literal.grad_w(W, G), rtol=1e-12, atol=1e-14)
    assert np.abs(gW.sum(axis=2)).max() < 1e-13
    h = 1e-3
    for d in range(D):
        for i in range(n):
            for j in range(k):
                def phi(w):
                    e = np.exp(w - w.max())
                    return float((G[d, i] * e / e.sum()).sum())
                wp = W[d, i].copy(); wp[j] += h
                wm = W[d, i].copy(); wm[j] -= h
                fd = (phi(wp) - phi(wm)) / (2 * h)
                assert fd == pytest.approx(gW[d, i, j], rel=1e-4, abs=1e-7)
    Gc = np.broadcast_to(rng.standard_normal((D, n, 1)), (D, n, k)).copy()
    assert np.abs(oracle.grad_w(W, Gc)).max() < 1e-14


def test_grad_w_large_weights_stable():
    W = np.array([[[1000.0, 999.0, -1000.0]]])
    G = np.array([[[1.0, 2.0, 3.0]]])
    gW = oracle.grad_w(W, G)
    assert np.all(np.isfinite(gW))
    np.testing.assert_allclose(gW, literal.grad_w(W, G), rtol=1e-12, atol=1e-300)


def test_update_and_smoothing_schedule():
    p = oracle.Params(problem=0, n=2, k=3, D=1, eta=0.1, rho=4.0, nb_iter=5)
    W = np.arange(6, dtype=float).reshape(1, 2, 3)
    gW = np.ones_like(W)
    assert np.allclose(oracle.update(p, 0, W, gW), W - 0.1)
    assert np.allclose(oracle.update(p, 3, W, gW), W - 0.1)
    assert np.allclose(oracle.update(p, 4, W, gW), (W - 0.1) / 4.0)   # (t+1) mod 5 == 0
    assert np.allclose(oracle.update(p, 9, W, gW), (W - 0.1) / 4.0)


def test_loss_matches_literal():
    rng = np.random.default_rng(12)
    for problem in (0, 1, 2, 3, 4):
        D, n, k = 4, 20, 4
        A = tcolgen.gnp(n, 0.5, 51)
        c = rng.integers(0, k, size=(D, n)).astype(np.int16)
        p = rand_params(problem, n, k, D)
        Mt = oracle.mtilde(c)
        fc, fe, _ = oracle.fitness(p, A, c)
        out = oracle.loss(p, 6, A, Mt, fc, fe)
        lit = literal.global_loss(A.astype(float), onehot(c, k), 6, p.alpha, p.lam, p.beta, p.mu,
                                  p.nu, problem)
        assert out[0] == pytest.approx(lit, rel=1e-12)


# ---------------------------------------------------------------- invariances --

def test_invariances():
    """Colour permutation within a member, population order and vertex relabelling
    leave fitness and the group concentration matrix unchanged (permuted accordingly)."""
    rng = np.random.default_rng(13)
    D, n, k = 4, 25, 5
    A = tcolgen.gnp(n, 0.5, 61)
    c = rng.integers(0, k, size=(D, n)).astype(np.int16)
    p = rand_params(1, n, k, D)
    t = 3
    f = oracle.fcolor(A, c)
    Mt = oracle.mtilde(c)
    gS = oracle.grad_s(p, t, A, c, Mt, oracle.class_sizes(c, k))
    # colours of member 1 permuted
    perm = rng.permutation(k)
    c2 = c.copy(); c2[1] = perm[c[1]]
    assert np.array_equal(oracle.fcolor(A, c2), f)
    assert np.array_equal(oracle.mtilde(c2), Mt)
    gS2 = oracle.grad_s(p, t, A, c2, oracle.mtilde(c2), oracle.class_sizes(c2, k))
    np.testing.assert_allclose(gS2[1][:, perm], gS[1], rtol=1e-13, atol=1e-13)
    # population order
    q = rng.permutation(D)
    assert np.array_equal(oracle.fcolor(A, c[q]), f[q])
    assert np.array_equal(oracle.mtilde(c[q]), Mt)
    # vertex relabelling P A P^T
    v = rng.permutation(n)
    Ap = A[np.ix_(v, v)]
    cp = c[:, v]
    assert np.array_equal(oracle.fcolor(Ap, cp), f)
    assert np.array_equal(oracle.mtilde(cp), Mt[np.ix_(v, v)])
    gSp = oracle.grad_s(p, t, Ap, cp, oracle.mtilde(cp), oracle.class_sizes(cp, k))
    np.testing.assert_allclose(gSp, gS[:, v, :], rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- iteration ----

def test_iteration_composes_steps_and_matches_literal():
    rng = np.random.default_rng(14)
    for problem in (0, 1, 2, 3, 4):
        D, n, k = 3, 18, 4
        A = tcolgen.gnp(n, 0.5, 71)
        W = rng.standard_normal((D, n, k)) * 0.01
        p = rand_params(problem, n, k, D)
        for t in (0, 4):      # t=4: (t+1) mod 5 == 0, smoothing applies
            r = oracle.iteration(p, t, A, W)
            assert r.status == 0 and r.t == t + 1
            S = literal.one_hot_argmax(W)
            gS = literal.grad_s(A.astype(float), S, t, p.alpha, p.lam, p.beta, p.mu, p.nu, problem)
            gW = literal.grad_w(W, gS)
            W1 = W - p.eta * gW
            if (t + 1) % p.nb_iter == 0:
                W1 = W1 / p.rho
            np.testing.assert_allclose(r.gS, gS, rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(r.gW, gW, rtol=1e-10, atol=1e-15)
            np.testing.assert_allclose(r.W, W1, rtol=1e-13, atol=1e-17)


def test_planted_population_stops_before_update():
    P = tcolgen.planted(120, 6, seed=5)
    rng = np.random.default_rng(15)
    D, n, k = 4, 120, 6
    c = rng.integers(0, k, size=(D, n)).astype(np.int16)
    c[2] = P.classes       # member 2 holds the hidden legal colouring
    c[3] = P.classes
    W = colour_weights(c, k, rng, scale=0.01)
    p = rand_params(1, n, k, D)
    r = oracle.iteration(p, 3, P.A, W)
    assert r.status == 1 and r.legal_d == 2 and r.t == 3
    np.testing.assert_array_equal(r.W, W)
    Wf, t, done, ld, col = oracle.run(p, 3, P.A, W, 10)
    assert done == 0 and ld == 2 and np.array_equal(col, P.classes)


def test_run_matches_repeated_iterations():
    rng = np.random.default_rng(16)
    D, n, k = 3, 20, 5
    A = tcolgen.gnp(n, 0.5, 81)
    W = rng.standard_normal((D, n, k)) * 0.01
    p = rand_params(0, n, k, D, stop_on_legal=0)
    Wr, t, done, ld, _ = oracle.run(p, 0, A, W, 12)
    Wi, ti = W, 0
    for _ in range(12):
        r = oracle.iteration(p, ti, A, Wi, want_grads=False)
        Wi, ti = r.W, r.t
    assert done == 12 and t == 12 and ti == 12
    np.testing.assert_array_equal(Wr, Wi)


def test_mycielski_toy_reaches_legal():
    """The paper's toy setting (D=1, lambda=mu=0, eta=1e-3, nb_iter=5, rho=200, seed 0) on a
    synthetic Mycielski graph with chi=5 finds a legal 5-colouring."""
    A = tcolgen.mycielski(5)
    n = A.shape[0]
    W = tcolgen.weights0(1, n, 5, seed=0)
    p = oracle.Params(problem=0, n=n, k=5, D=1, eta=1e-3, rho=200.0, nb_iter=5, lam=0.0, mu=0.0)
    Wf, t, done, ld, col = oracle.run(p, 0, A, W, 20000)
    assert ld == 0
    assert oracle.fcolor(A, col[None, :])[0] == 0


# ------------------------------------------------- other problems (Section 6) --

@pytest.mark.parametrize("n,k,seed", [(5, 2, 0), (6, 3, 1), (6, 2, 2)])
def test_cut_exhaustive_all_partitions(n, k, seed):
    """f_cut by brute force over edges for every k-partition of small graphs, against the
    literal 1/2 sum(A o (J - M)) and |E| - f_color."""
    A = tcolgen.gnp(n, 0.6, 200 + seed)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if A[i, j]]
    cols = np.array(list(itertools.product(range(k), repeat=n)), dtype=np.int16)
    got = oracle.fcut(A, cols)
    want = np.array([sum(1 for i, j in edges if c[i] != c[j]) for c in cols], dtype=np.int64)
    assert np.array_equal(got, want)
    assert np.array_equal(got, len(edges) - oracle.fcolor(A, cols))
    lit = literal.fitness_cut(A.astype(float), onehot(cols, k))
    assert np.array_equal(got, lit.astype(np.int64))


def test_partition_single_member_identities():
    """D = 1, partitioning: D - mt is 1 across groups and 0 inside, so kappa = 2 f_cut and
    varpi counts the ordered non-adjacent pairs split across groups."""
    rng = np.random.default_rng(31)
    for trial in range(8):
        n, k = int(rng.integers(5, 30)), int(rng.integers(2, 6))
        A = tcolgen.gnp(n, 0.4, 300 + trial)
        c = rng.integers(0, k, size=(1, n)).astype(np.int16)
        p = oracle.Params(problem=2, n=n, k=k, D=1, alpha=2.5, beta=1.2, lam=1, mu=1)
        fm, fs, f = oracle.fitness(p, A, c)
        out = oracle.loss(p, 0, A, oracle.mtilde(c), fm, fs)
        split = sum(1 for i in range(n) for j in range(n) if i != j and not A[i, j] and c[0, i] != c[0, j])
        assert out[3] == pytest.approx(2 * fm[0], abs=1e-12)
        assert out[4] == pytest.approx(split, abs=1e-12)
        assert fs[0] == 0 and f[0] == fm[0]


def test_balanced_partition_fitness_adds_equity():
    rng = np.random.default_rng(32)
    n, k, D = 23, 4, 5
    A = tcolgen.gnp(n, 0.5, 33)
    c = rng.integers(0, k, size=(D, n)).astype(np.int16)
    p = oracle.Params(problem=3, n=n, k=k, D=D)
    fm, fs, f = oracle.fitness(p, A, c)
    assert np.array_equal(fm, oracle.fcut(A, c))
    assert np.array_equal(fs, literal.equity_fitness(onehot(c, k)).astype(np.int64))
    assert np.array_equal(f, fm + fs)


def test_mscp_fitness_closed_forms():
    """f_mscp = sum_i (c(i) + 1): n with every vertex in colour 0, and sum_l (l + 1) #V_l."""
    n, k = 17, 5
    A = tcolgen.gnp(n, 0.5, 34)
    p = oracle.Params(problem=4, n=n, k=k, D=2)
    c = np.zeros((2, n), np.int16)
    c[1] = np.arange(n) % k
    fm, fs, f = oracle.fitness(p, A, c)
    assert fs[0] == n
    assert fs[1] == sum((i % k) + 1 for i in range(n))
    assert np.array_equal(fm, oracle.fcolor(A, c)) and np.array_equal(f, fm + fs)
    assert np.array_equal(fs, literal.fitness_mscp(onehot(c, k)).astype(np.int64))


def test_partition_invariances():
    """Relabelling the groups of a member leaves the cut and D - Mt unchanged, and permutes
    the gradient's group axis."""
    rng = np.random.default_rng(35)
    D, n, k = 3, 21, 4
    A = tcolgen.gnp(n, 0.5, 36)
    c = rng.integers(0, k, size=(D, n)).astype(np.int16)
    p = rand_params(3, n, k, D)
    gS = oracle.grad_s(p, 4, A, c, oracle.mtilde(c), oracle.class_sizes(c, k))
    perm = rng.permutation(k)
    c2 = c.copy(); c2[0] = perm[c[0]]
    assert np.array_equal(oracle.fcut(A, c2), oracle.fcut(A, c))
    gS2 = oracle.grad_s(p, 4, A, c2, oracle.mtilde(c2), oracle.class_sizes(c2, k))
    np.testing.assert_allclose(gS2[0][:, perm], gS[0], rtol=1e-13, atol=1e-13)


# ------------------------------------------------------- momentum (Section 7) --

@pytest.mark.parametrize("gamma", [0.5, 0.9])
def test_momentum_matches_torch_sgd(gamma):
    """Heavy-ball steps: the oracle's iterations with momentum gamma equal torch.optim.SGD
    (momentum=gamma, dampening 0) fed the oracle's straight-through gradient each step
    (smoothing off: nb_iter beyond the run)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(40)
    D, n, k = 3, 16, 4
    A = tcolgen.gnp(n, 0.5, 41)
    W0 = rng.standard_normal((D, n, k)) * 0.05
    p = rand_params(1, n, k, D, eta=0.05, nb_iter=1000, stop_on_legal=0, momentum=gamma)
    vel = np.zeros((D, n, k))
    Wo, t = W0.copy(), 0
    Wt = torch.tensor(W0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.SGD([Wt], lr=p.eta, momentum=gamma, dampening=0.0)
    for step in range(6):
        W_np = Wt.detach().numpy()
        c = oracle.colors(W_np)
        gS = oracle.grad_s(p, step, A, c, oracle.mtilde(c), oracle.class_sizes(c, k))
        opt.zero_grad()
        Wt.grad = torch.tensor(oracle.grad_w(W_np, gS))
        opt.step()
        r = oracle.iteration(p, t, A, Wo, vel=vel)
        Wo, t = r.W, r.t
        np.testing.assert_allclose(Wo, Wt.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_momentum_zero_is_plain_and_row_sums_kept():
    """gamma = 0 is the plain step; with momentum the velocity rows sum to zero like gW, so
    the weight row sums stay put between smoothings."""
    rng = np.random.default_rng(42)
    D, n, k = 2, 12, 5
    A = tcolgen.gnp(n, 0.5, 43)
    W = rng.standard_normal((D, n, k)) * 0.05
    p0 = rand_params(0, n, k, D, stop_on_legal=0, nb_iter=1000)
    pm = rand_params(0, n, k, D, stop_on_legal=0, nb_iter=1000, momentum=0.0)
    np.testing.assert_array_equal(oracle.iteration(p0, 2, A, W).W, oracle.iteration(pm, 2, A, W).W)
    pg = rand_params(0, n, k, D, stop_on_legal=0, nb_iter=1000, momentum=0.8, eta=0.1)
    vel = np.zeros((D, n, k))
    Wi, t = W.copy(), 0
    for _ in range(5):
        r = oracle.iteration(pg, t, A, Wi, vel=vel)
        Wi, t = r.W, r.t
    assert np.abs(vel.sum(axis=2)).max() < 1e-12
    np.testing.assert_allclose(Wi.sum(axis=2), W.sum(axis=2), atol=1e-12)


def test_class_conflicts_pins():
    """S_d^T A S_d: trace = 2 f_color (itself pinned by exhaustive enumeration), symmetric,
    entries summing to 2 |E|, equal to the literal matrix product, and on a complete bipartite
    graph coloured by its sides every edge between the two classes."""
    rng = np.random.default_rng(11)
    for n, k, D, p in ((9, 3, 4, 0.5), (30, 5, 3, 0.3), (1, 2, 2, 0.5)):
        A = tcolgen.gnp(n, p, seed=n)
        c = rng.integers(0, k, size=(D, n)).astype(np.int16)
        C = oracle.class_conflicts(A, c, k)
        assert C.shape == (D, k, k)
        assert np.array_equal(np.trace(C, axis1=1, axis2=2), 2 * oracle.fcolor(A, c))
        assert np.array_equal(C, np.transpose(C, (0, 2, 1)))
        assert np.all(C.sum(axis=(1, 2)) == A.sum())
        assert np.array_equal(C, np.rint(literal.class_conflicts(A.astype(float), onehot(c, k))).astype(np.int32))
    # a bipartite graph coloured by its sides: every edge runs between classes 0 and 1
    n = 10
    A = np.zeros((n, n), np.uint8)
    for i in range(5):
        for j in range(5, 10):
            A[i, j] = A[j, i] = 1
    c = np.array([[0] * 5 + [1] * 5], np.int16)
    C = oracle.class_conflicts(A, c, 3)[0]
    assert C[0, 1] == C[1, 0] == 25 and C.sum() == 50


# ------------------------------------------------------------ multicolouring -----

def rand_demand(n, k, rng, cmax=3):
    return rng.integers(1, min(cmax, k) + 1, size=n).astype(np.int32)


def test_select_matches_literal_top_c():
    """Step 1 of multicolouring against a stable sort of the negated weights; integer weights
    make ties common, and ties go to the lower colour."""
    rng = np.random.default_rng(51)
    D, n, k = 3, 40, 7
    W = rng.integers(-2, 3, size=(D, n, k)).astype(np.float64)
    dem = rand_demand(n, k, rng, cmax=5)
    S = oracle.select(W, dem)
    assert np.array_equal(S, literal.top_c(W, dem).astype(np.uint8))
    assert np.array_equal(S.sum(axis=2), np.broadcast_to(dem, (D, n)))
    with pytest.raises(ValueError):
        oracle.select(W, np.full(n, k + 1, np.int32))
    W[1, 2, 3] = np.nan
    with pytest.raises(FloatingPointError):
        oracle.select(W, dem)


def test_multi_with_unit_demand_is_k_colouring():
    """With every c_i = 1 the selection is the argmax and every quantity, and a whole
    iteration, is the k-colouring one (problem 0, whose pins are above)."""
    rng = np.random.default_rng(52)
    D, n, k = 4, 30, 6
    A = tcolgen.gnp(n, 0.5, 52)
    W = rng.normal(size=(D, n, k))
    one = np.ones(n, np.int32)
    S = oracle.select(W, one)
    c = oracle.colors(W)
    assert np.array_equal(S, onehot(c, k).astype(np.uint8))
    assert np.array_equal(oracle.fcolor_multi(A, S), oracle.fcolor(A, c))
    Mt = oracle.mtilde_multi(S)
    assert np.array_equal(Mt, oracle.mtilde(c))
    p0 = rand_params(0, n, k, D, stop_on_legal=0)
    p5 = rand_params(5, n, k, D, stop_on_legal=0, nu=0.0)
    # the same sums, grouped differently (the multi form adds a_ij and the penalty per pair first)
    np.testing.assert_allclose(oracle.grad_s_multi(p5, 9, A, S, Mt),
                               oracle.grad_s(p0, 9, A, c, Mt, oracle.class_sizes(c, k)), rtol=1e-13, atol=1e-13)
    for t in (0, 4):
        r5 = oracle.iteration_multi(p5, t, A, W, one)
        r0 = oracle.iteration(p0, t, A, W)
        assert r5.status == r0.status == 0
        np.testing.assert_allclose(r5.W, r0.W, rtol=1e-13, atol=1e-16)


def _subset_members(n, k, demand):
    """Every assignment of demand[i] different colours to each vertex, as multi-hot members."""
    choices = [list(itertools.combinations(range(k), int(c))) for c in demand]
    out = []
    for combo in itertools.product(*choices):
        S = np.zeros((n, k), np.uint8)
        for i, cols in enumerate(combo):
            S[i, list(cols)] = 1
        out.append(S)
    return np.stack(out)


@pytest.mark.parametrize("name,n,edges,demand,k_no,k_yes", [
    # the 5-cycle needs 5 colours when every vertex takes 2 (its 2-fold chromatic number)
    ("C5 x2", 5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)], [2, 2, 2, 2, 2], 4, 5),
    # a triangle whose vertices take 1, 2 and 3 colours needs 6
    ("K3 1,2,3", 3, [(0, 1), (1, 2), (0, 2)], [1, 2, 3], 5, 6),
])
def test_multicolouring_exhaustive(name, n, edges, demand, k_no, k_yes):
    """f_color of multicolourings against facts about the graphs: enumerating every assignment,
    no legal one exists with k_no colours and one does with k_yes; and on each assignment the
    value is the number of (edge, shared colour) pairs, counted with Python sets."""
    A = adj_from_edges(n, edges)
    for k, want_legal in ((k_no, False), (k_yes, True)):
        S = _subset_members(n, k, demand)
        f = oracle.fcolor_multi(A, S)
        assert (f.min() == 0) == want_legal, (name, k)
        for d in range(0, len(S), max(1, len(S) // 50)):
            sets = [set(np.nonzero(S[d, i])[0]) for i in range(n)]
            assert f[d] == sum(len(sets[i] & sets[j]) for i, j in edges)


def test_mtilde_multi_properties():
    rng = np.random.default_rng(53)
    D, n, k = 5, 25, 6
    W = rng.normal(size=(D, n, k))
    dem = rand_demand(n, k, rng)
    S = oracle.select(W, dem)
    Mt = oracle.mtilde_multi(S)
    assert np.array_equal(Mt, Mt.T)
    assert np.array_equal(np.diag(Mt), D * dem)
    V = oracle.class_sizes_multi(S)
    assert np.array_equal(V, S.sum(axis=1))
    assert Mt.sum() == int((V.astype(np.int64) ** 2).sum())
    assert np.array_equal(Mt, np.rint(literal.group_concentration(S.astype(float))).astype(np.int32))


@pytest.mark.parametrize("diag", [1, 0])
def test_grad_s_multi_literal_and_finite_differences(diag):
    """The gradient with multi-hot S against the literal tensor form, and against central
    differences (h = 1e-3) of the paper's loss as a polynomial in S at the selected S."""
    rng = np.random.default_rng(54 + diag)
    D, n, k = 3, 14, 5
    A = tcolgen.gnp(n, 0.5, 54)
    W = rng.normal(size=(D, n, k))
    dem = rand_demand(n, k, rng)
    S = oracle.select(W, dem)
    p = rand_params(5, n, k, D, bonus_diag=diag, nu=0.0)
    t = 6
    gS = oracle.grad_s_multi(p, t, A, S, oracle.mtilde_multi(S))
    Sf = S.astype(float)
    Af = A.astype(float)
    lit = literal.grad_s(Af, Sf, t, p.alpha, p.lam, p.beta, p.mu, p.nu, 5, diag)
    np.testing.assert_allclose(gS, lit, rtol=1e-12, atol=1e-12)
    h = 1e-3

    def L(Sx):
        return literal.global_loss(Af, Sx, t, p.alpha, p.lam, p.beta, p.mu, p.nu, 5, diag)

    for (d, i, l) in tcolgen.fd_entries(32, D, n, k, seed=5):
        Sp = Sf.copy(); Sp[d, i, l] += h
        Sm = Sf.copy(); Sm[d, i, l] -= h
        fd = (L(Sp) - L(Sm)) / (2 * h)
        assert fd == pytest.approx(gS[d, i, l], rel=1e-4, abs=1e-6), (d, i, l)


def test_loss_multi_matches_literal():
    rng = np.random.default_rng(56)
    D, n, k = 4, 20, 6
    A = tcolgen.gnp(n, 0.4, 56)
    W = rng.normal(size=(D, n, k))
    dem = rand_demand(n, k, rng)
    S = oracle.select(W, dem)
    p = rand_params(5, n, k, D, nu=0.0)
    Mt = oracle.mtilde_multi(S)
    f = oracle.fcolor_multi(A, S)
    out = oracle.loss(p, 7, A, Mt, f, np.zeros(D, np.int64))
    lit = literal.global_loss(A.astype(float), S.astype(float), 7, p.alpha, p.lam, p.beta, p.mu, p.nu, 5, 1)
    assert out[0] == pytest.approx(lit, rel=1e-12)
    assert out[1] == pytest.approx(literal.fitness_color(A.astype(float), S.astype(float)).sum())


def test_iteration_multi_composes_literal_steps():
    """One iteration: literal selection, gradient, straight-through backward, update and
    smoothing give the oracle's W; a member holding a legal multicolouring stops it."""
    rng = np.random.default_rng(57)
    D, n, k = 3, 18, 6
    A = tcolgen.gnp(n, 0.3, 57)
    W = rng.normal(size=(D, n, k))
    dem = rand_demand(n, k, rng)
    p = rand_params(5, n, k, D, nu=0.0, stop_on_legal=0)
    for t in (3, 4):          # t = 4 smooths (nb_iter 5)
        r = oracle.iteration_multi(p, t, A, W, dem)
        S = literal.top_c(W, dem)
        gS = literal.grad_s(A.astype(float), S, t, p.alpha, p.lam, p.beta, p.mu, p.nu, 5, 1)
        Wn = W - p.eta * literal.grad_w(W, gS)
        if (t + 1) % p.nb_iter == 0:
            Wn = Wn / p.rho
        np.testing.assert_allclose(r.W, Wn, rtol=1e-12, atol=1e-15)
        assert r.t == t + 1
    # a legal member: the triangle with demands 1, 2, 3 and 6 colours, member 1 coloured legally
    A3 = adj_from_edges(3, [(0, 1), (1, 2), (0, 2)])
    dem3 = np.array([1, 2, 3], np.int32)
    W3 = rng.normal(size=(2, 3, 6)) * 0.01
    W3[1, 0, 0] = W3[1, 1, [1, 2]] = W3[1, 2, [3, 4, 5]] = 1.0
    p3 = rand_params(5, 3, 6, 2, nu=0.0)
    r = oracle.iteration_multi(p3, 2, A3, W3, dem3)
    assert r.status == 1 and r.legal_d == 1 and r.f_color[1] == 0
