"""GPU parity of libtcol (through its C ABI) against the FP64 oracle.

Bar: colours, conflict counts, equity fitness, the group concentration matrix
and the stop decision bit-exact; FP32 loss, gradient and updated weights within
1e-5 norm-wise (max |diff| <= 1e-5 max |ref| per tensor; the loss against
sum|f_color| + nu t sum|f_eq| + lambda t |kappa| + mu t |varpi|).  In the bf16,
fp8 and fp4 operand modes the dense penalty pass rounds its operand to bf16:
those results are checked at the same 1e-5 against the oracle's values taken
with that operand rounded as the library declares it, and against the exact FP64
oracle within the bound the rounding implies (unit roundoff 2^-8 per operand
entry plus FP32 accumulation); both errors are printed.
"""
import numpy as np
import pytest

import oracle
import tcolgen
from tcolgen import BF16, ECP, FP4, FP8, FP32, KCOL, GraphCase

from gpu_util import (check_loss_grad, expected_route, grad_s_bound, host, make_solver, normwise, orc_params,
                      penalty_terms, reference_step, run_resynced, step_route)

pytestmark = pytest.mark.gpu

TOL = 1e-5


def small_cases():
    out = []
    for prec in (FP32, BF16, FP8, FP4):
        out.append(GraphCase(f"ragged77_kcol_p{prec}", KCOL, 77, 7, 5, prec, "gnp", 0.4, graph_seed=7,
                             rho=10.0, lam=1e-2, mu=3e-3))
        out.append(GraphCase(f"ragged150_ecp_p{prec}", ECP, 150, 11, 6, prec, "gnp", 0.5, graph_seed=8,
                             rho=10.0, lam=1e-2, mu=3e-3, nu=0.05))
    out.append(GraphCase("multi_tile300", KCOL, 300, 30, 12, FP32, "gnp", 0.5, graph_seed=9, lam=1e-3, mu=1e-4))
    out.append(tcolgen.case_c1())
    return out


def ids(cases):
    return [c.name for c in cases]


@pytest.mark.parametrize("case", small_cases(), ids=ids(small_cases()))
def test_conflicts_bit_exact(case):
    s, (A,) = make_solver([case])
    W = host(s.W[0])
    c, fc, fe = s.conflicts(0)
    c_ref = oracle.colors(W)
    assert np.array_equal(host(c), c_ref)
    assert np.array_equal(host(fc), oracle.fcolor(A, c_ref))
    fe_ref = oracle.feq(oracle.class_sizes(c_ref, case.k), case.n) if case.problem == ECP else np.zeros(case.D)
    assert np.array_equal(host(fe), fe_ref)
    s.close()


SHAPES = [(64, 2), (64, 4), (128, 4), (128, 6), (128, 8), (64, 9), (128, 9), (256, 4), (256, 6)]


@pytest.mark.parametrize("prec", [FP32, BF16, FP8, FP4])
def test_conflicts_every_tile_shape(prec):
    """f_color through the contraction's gather is exact for every instantiated tile shape, on a
    graph whose size spans several row tiles with a ragged tail and whose D*k is not a multiple
    of any column tile."""
    case = GraphCase("shapes", KCOL, 1000, 28, 40, prec, "gnp", 0.5, graph_seed=13, stop_on_legal=0)
    A = case.adjacency()
    W = case.weights()
    ref = oracle.fcolor(A, oracle.colors(W))
    s, _ = make_solver([case], As=[A], Ws=[W])
    bad = []
    for bm, ntw in SHAPES:
        s.set_options(tile_bm=bm, tile_ntw=ntw)
        for rep in range(4):    # a stage-buffer race shows up only now and then
            _, fc, _ = s.conflicts(0)
            got = host(fc)
            if not np.array_equal(got, ref):
                bad.append(((bm, ntw), rep, np.nonzero(got != ref)[0].tolist()[:8]))
    s.close()
    assert not bad, bad


@pytest.mark.parametrize("case", small_cases(), ids=ids(small_cases()))
def test_mtilde_bit_exact(case):
    s, (A,) = make_solver([case])
    M = host(s.mtilde(0))
    assert np.array_equal(M, oracle.mtilde(oracle.colors(host(s.W[0]))))
    s.close()


@pytest.mark.parametrize("case", small_cases(), ids=ids(small_cases()))
@pytest.mark.parametrize("t", [0, 3, 57])
def test_loss_and_gradients(case, t):
    s, (A,) = make_solver([case])
    s.set_t(t)
    check_loss_grad(case, s, A, t)
    s.close()


PATHS = {"plain": dict(fused=0), "fast_dense": dict(fused=1, penalty=1), "fast_sparse": dict(fused=1, penalty=2),
         "epi_dense": dict(fused=2, penalty=1), "epi_sparse": dict(fused=2, penalty=2)}


@pytest.mark.parametrize("path", list(PATHS))
def test_c1_resynced_200_steps(path):
    wr, wx, _ = run_resynced(tcolgen.case_c1(), 200, check_every=10, **PATHS[path])
    print(f"C1 {path} worst W error {wr:.2e} (FP64 {wx:.2e})")


@pytest.mark.parametrize("path", [p for p in PATHS if p != "plain"])
@pytest.mark.parametrize("prec", [FP32, BF16, FP8, FP4])
def test_fused_large_k_resynced(path, prec):
    """Many colours against few members (the shape where the penalty operand is sparse),
    ECP so every loss term is active, a ragged n and several tiles."""
    case = GraphCase(f"ecp_n600_k120_D8_p{prec}", ECP, 600, 120, 8, prec, "gnp", 0.5, graph_seed=31, rho=10.0,
                     lam=2e-2, mu=5e-3, nu=0.05)
    wr, wx, _ = run_resynced(case, 8, t0=3, **PATHS[path])
    print(f"{case.name} {path}: worst W error against the route's operand {wr:.2e}, against FP64 {wx:.2e}")


@pytest.mark.parametrize("path", [p for p in PATHS if p != "plain"])
def test_degenerate_population(path):
    """Every vertex in one colour in every member: Mt is all D, the penalty operand is dense,
    the sparse kernel lists every vertex of a row and counts by comparison, and the
    per-iteration choice takes the dense pass."""
    n, k, D = 300, 100, 8
    case = GraphCase("degenerate", KCOL, n, k, D, FP32, "gnp", 0.5, graph_seed=33, lam=1e-2, mu=1e-3)
    W = case.weights()
    W[:, :, 0] += 1.0
    wr, wx, _ = run_resynced(case, 3, t0=2, W=W, **PATHS[path])
    print(f"degenerate worst W error {wr:.2e} (FP64 {wx:.2e})")


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("prec", [BF16, FP8, FP4])
def test_small_resynced_low_precision(prec, path):
    case = GraphCase("kcol90", KCOL, 90, 9, 6, prec, "gnp", 0.5, graph_seed=12, rho=10.0, lam=1e-2, mu=3e-3)
    wr, wx, _ = run_resynced(case, 30, **PATHS[path])
    print(f"prec {prec} {path}: worst W error against the route's operand {wr:.2e}, against FP64 {wx:.2e}")


@pytest.mark.parametrize("path", list(PATHS))
def test_c2_resynced_steps(path):
    wr, wx, _ = run_resynced(tcolgen.case_c2(FP32), 12, check_every=4, **PATHS[path])
    print(f"C2 {path} worst W error {wr:.2e} (FP64 {wx:.2e})")


def test_c2_trajectory_2000_steps():
    """C2 (k-COL, G(500, .5), k = 50, D = 64, FP32) for its configured 2000 iterations on the
    default schedule (fast path, hipGraph replay of 8-step runs, per-iteration penalty
    choice), with the stop rule on.  Every 100 iterations the GPU's own W_t starts one
    resynced step: W_{t+1} against the oracle within 1e-5 norm-wise, the route the
    documented one, colours and conflicts after it exact.  A legal member found on the way
    stops the run: then the returned member and colouring must be the oracle's for the W
    the GPU stopped at."""
    case = tcolgen.case_c2(FP32)
    assert case.stop_on_legal == 1
    s, (A,) = make_solver([case])
    p = orc_params(case.params())
    t = 0
    worst = 0.0
    checks = 0
    col = __import__("torch").zeros(case.n, dtype=__import__("torch").int16, device="cuda")
    while t < 2000:
        done, legal = s.step(99, colors_out=[col])
        t += done
        assert s.get_t() == t
        W0 = host(s.W[0])
        if legal[0] >= 0:
            ref = oracle.iteration(p, t, A, W0, want_grads=False)
            assert ref.status == 1 and ref.legal_d == legal[0]
            assert oracle.fcolor(A, host(col)[None, :])[0] == 0
            print(f"C2: legal {case.k}-colouring by member {legal[0]} at t = {t}")
            break
        before = s.counters()
        done, legal = s.step(1, colors_out=[col])
        route = step_route(s, before)
        ref, W_route, bound = reference_step(p, t, A, W0, route, FP32)
        assert route == expected_route(case, {}, t, ref.colors)
        if ref.status == 1:
            assert done == 0 and legal == [ref.legal_d]
            assert np.array_equal(host(col), ref.colors[ref.legal_d])
            print(f"C2: legal {case.k}-colouring by member {legal[0]} at t = {t} (checked step)")
            break
        assert done == 1
        W1 = host(s.W[0])
        e = normwise(W1, W_route)
        worst = max(worst, e)
        assert e <= TOL, (t, e)
        assert np.abs(W1 - ref.W).max() <= bound + TOL * np.abs(ref.W).max()
        c, fc, _ = s.conflicts(0)
        c_ref = oracle.colors(W1)
        assert np.array_equal(host(c), c_ref)
        assert np.array_equal(host(fc), oracle.fcolor(A, c_ref))
        t += 1
        checks += 1
    s.close()
    print(f"C2 trajectory: {checks} resynced checkpoints up to t = {t}, worst W error {worst:.2e}")
    assert checks >= 1


def test_fast_multistep_run_matches_oracle_trajectory():
    """A single tcol_step call of 12 iterations on the fast schedule (hipGraph replay of runs
    of 4, where the class-size launch of each iteration ends the previous one), with the
    per-iteration penalty choice switching between the dense pass and the sparse rows
    (smoothing by 100 every second iteration), FP32: the weights, t and the number of
    updates against the oracle iterated from the same W0, and the number of iterations on
    each route against the documented choice on the oracle's colours."""
    case = GraphCase("multistep", KCOL, 400, 40, 4, FP32, "gnp", 0.5, graph_seed=62, rho=100.0, nb_iter=2,
                     lam=1e-2, mu=3e-3, stop_on_legal=0)
    W = case.weights()
    W[0, :200, 0] += 0.05
    opts = dict(fused=1, penalty=3, use_graph=1, unroll=4)
    s, (A,) = make_solver([case], Ws=[W], **opts)
    p = orc_params(case.params())
    before = s.counters()
    done, _ = s.step(12)
    after = s.counters()
    assert done == 12 and s.get_t() == 12
    Wr = W.astype(np.float64)
    want = {"none": 0, "dense": 0, "sparse": 0}
    for t in range(12):
        r = oracle.iteration(p, t, A, Wr, want_grads=False)
        want[expected_route(case, opts, t, r.colors)] += 1
        Wr = r.W
    got = {"none": after["no_penalty"] - before["no_penalty"], "dense": after["dense"] - before["dense"],
           "sparse": after["sparse"] - before["sparse"]}
    e = normwise(host(s.W[0]), Wr)
    print(f"12-step run: W error {e:.2e}, routes {got} (expected {want})")
    assert got == want
    assert want["dense"] > 0 and want["sparse"] > 0
    assert e <= TOL
    s.close()


def test_nonfinite_restart_on_the_sparse_route():
    """A stop for a non-finite weight, then a restart, on the fast schedule with sparse rows and
    the per-iteration choice (penalty 3).  Every row is saturated (one weight 1e4, the rest 0:
    the softmax is exactly one-hot, the gradient exactly 0, and with rho = 1 the weights never
    change), the learning rate is 3e38, and one row is uniform: its first update overflows.
    (1) A NaN placed in W between two tcol_step calls stops the next call before any update.
    (2) The overflowing row stops a captured 8-iteration run at the start of its second
    iteration, where the class-size launch ends the first one.  After each stop the caller
    restores finite weights and calls tcol_reset; then resynced steps follow the oracle with
    the documented penalty route, colours and conflicts exact."""
    import paper_1909_02261_amd as pk
    n, k, D = 400, 40, 4
    case = GraphCase("restart", KCOL, n, k, D, FP32, "gnp", 0.3, graph_seed=71, eta=3e38, rho=1.0,
                     lam=1e-2, mu=3e-3, stop_on_legal=0)
    A = case.adjacency()
    rng = np.random.default_rng(5)
    cols = rng.integers(0, k, size=(D, n))
    # member 1 colours every neighbour of vertex 11 with colour 0, so that row's gradient at a
    # uniform softmax is about deg(11) / k >> 1 and the update overflows
    cols[1, np.nonzero(A[11])[0]] = 0
    Wf = np.zeros((D, n, k), np.float32)
    Wf[np.arange(D)[:, None], np.arange(n)[None, :], cols] = 1e4
    opts = dict(fused=1, penalty=3, use_graph=1, unroll=8)
    s, _ = make_solver([case], As=[A], Ws=[Wf], **opts)
    p = orc_params(case.params())
    torch = __import__("torch")
    saved = s.W[0].clone()

    def resume_and_check(t0, steps):
        s.W[0].copy_(saved)
        s.set_t(t0)
        s.reset()
        t = t0
        for _ in range(steps):
            W0 = host(s.W[0])
            before = s.counters()
            done, _ = s.step(1)
            route = step_route(s, before)
            ref, W_route, _ = reference_step(p, t, A, W0, route, FP32)
            assert route == expected_route(case, opts, t, ref.colors) == "sparse", route
            assert done == 1 and normwise(host(s.W[0]), W_route) <= TOL
            c, fc, _ = s.conflicts(0)
            assert np.array_equal(host(c), ref.colors)
            assert np.array_equal(host(fc), oracle.fcolor(A, ref.colors))
            t += 1

    resume_and_check(1, 3)
    # (1) NaN between calls
    s.W[0][2, 7, 3] = float("nan")
    with pytest.raises(pk.TcolError) as ei:
        s.step(4)
    assert ei.value.status == -5
    resume_and_check(5, 3)
    # (2) an update that overflows inside a captured run
    s.W[0][1, 11, :] = 0.0
    with pytest.raises(pk.TcolError) as ei:
        s.step(8)
    assert ei.value.status == -5
    assert not torch.isfinite(s.W[0][1, 11]).all()
    resume_and_check(9, 4)
    s.close()


def test_planted_stops_at_step0():
    case = tcolgen.case_c3(FP8)
    P = tcolgen.planted(case.n, case.k, case.graph_seed)
    W = case.weights()
    W[5, np.arange(case.n), P.classes] += 1.0     # member 5 holds the hidden legal colouring
    for prec, fused in ((FP8, 1), (BF16, 2), (FP32, 0), (FP8, 0), (FP8, 2), (FP4, 1), (FP4, 2)):
        case.precision = prec
        s, _ = make_solver([case], As=[P.A], Ws=[W], fused=fused)
        c, fc, fe = s.conflicts(0)
        assert int(host(fc)[5]) == 0
        c_ref = oracle.colors(W)
        assert np.array_equal(host(fc), oracle.fcolor(P.A, c_ref)), (prec, fused, s.options())
        col = __import__("torch").zeros(case.n, dtype=__import__("torch").int16, device="cuda")
        done, legal = s.step(10, colors_out=[col])
        assert done == 0 and legal == [5]
        assert np.array_equal(host(col), P.classes)
        assert np.array_equal(host(s.W[0]), W)
        s.close()


def test_edge_cases():
    torch = __import__("torch")
    # k = 1: every edge conflicts; D = 1
    case = GraphCase("k1", KCOL, 40, 1, 1, FP32, "gnp", 0.3, graph_seed=3)
    s, (A,) = make_solver([case])
    c, fc, fe = s.conflicts(0)
    assert int(host(fc)[0]) == int(A.sum() // 2)
    s.close()
    # n = 1, empty graph: legal at once
    case = GraphCase("n1", KCOL, 1, 3, 2, BF16, "gnp", 0.5)
    s, _ = make_solver([case])
    assert s.step(5) == (0, [0])
    s.close()
    # complete graph with k = n (legal colourings exist); one member coloured legally
    n = 20
    A = (np.ones((n, n)) - np.eye(n)).astype(np.uint8)
    W = np.zeros((3, n, n), np.float32)
    W[1, np.arange(n), np.arange(n)] = 1.0
    W[0, :, 0] = 1.0
    case = GraphCase("Kn", KCOL, n, n, 3, FP8, "gnp", 1.0)
    s, _ = make_solver([case], As=[A], Ws=[W])
    c, fc, fe = s.conflicts(0)
    assert host(fc).tolist() == [n * (n - 1) // 2, 0, n * (n - 1) // 2]   # member 2: all-zero W ties -> colour 0
    s.close()


def test_nonfinite_and_bad_graph():
    import paper_1909_02261_amd as pk
    torch = __import__("torch")
    case = GraphCase("nan", KCOL, 50, 5, 4, FP32, "gnp", 0.5, graph_seed=4)
    W = case.weights()
    W[2, 7, 3] = np.nan
    s, _ = make_solver([case], Ws=[W])
    with pytest.raises(pk.TcolError) as ei:
        s.step(3)
    assert ei.value.status == -5
    s.close()
    A = case.adjacency()
    A[0, 1] = 1
    A[1, 0] = 0
    with pytest.raises(pk.TcolError) as ei:
        make_solver([case], As=[A])
    assert ei.value.status == -3


def test_graph_replay_matches_eager_and_is_deterministic():
    case = GraphCase("det", KCOL, 200, 20, 8, BF16, "gnp", 0.5, graph_seed=5, rho=10.0, lam=1e-3, mu=1e-4,
                     stop_on_legal=0)
    for fused, pen in ((0, 0), (1, 1), (1, 2), (2, 1), (2, 2)):
        outs = []
        for use_graph, unroll in ((0, 1), (1, 4), (1, 8)):
            s, _ = make_solver([case], use_graph=use_graph, unroll=unroll, fused=fused, penalty=pen)
            done, _ = s.step(23)
            assert done == 23 and s.get_t() == 23
            outs.append(host(s.W[0]).copy())
            s.close()
        assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_checkpoint_resume():
    torch = __import__("torch")
    case = GraphCase("ckpt", ECP, 120, 10, 6, FP32, "gnp", 0.5, graph_seed=6, rho=10.0, nu=1e-3, mu=0.0,
                     lam=1e-3, stop_on_legal=0)
    s, _ = make_solver([case])
    s.step(20)
    W_full = host(s.W[0]).copy()
    s.close()
    s, _ = make_solver([case])
    s.step(10)
    W_mid = s.W[0].clone()
    t_mid = s.get_t()
    s.close()
    s2, _ = make_solver([case], Ws=[host(W_mid)])
    s2.set_t(t_mid)
    s2.step(10)
    assert np.array_equal(host(s2.W[0]), W_full)
    s2.close()


def test_batch_of_uneven_graphs_matches_separate_contexts():
    cases = [GraphCase("b0", KCOL, 130, 12, 4, BF16, "gnp", 0.5, graph_seed=21, lam=1e-3, mu=1e-4, stop_on_legal=0),
             GraphCase("b1", ECP, 257, 19, 3, BF16, "gnp", 0.1, graph_seed=22, mu=0.0, nu=1e-3, stop_on_legal=0),
             GraphCase("b2", KCOL, 64, 30, 7, BF16, "gnp", 0.9, graph_seed=23, alpha=1.5, stop_on_legal=0)]
    for fused in (0, 1, 2):
        sb, _ = make_solver(cases, fused=fused)
        o = sb.options()
        sb.step(9)
        batch_W = [host(w).copy() for w in sb.W]
        batch_f = [host(sb.conflicts(g)[1]) for g in range(3)]
        sb.close()
        for g, c in enumerate(cases):
            # same tile shape as the batch: the per-element arithmetic is then identical
            s1, _ = make_solver([c], fused=fused, tile_bm=o["tile_bm"], tile_ntw=o["tile_ntw"])
            s1.step(9)
            assert np.array_equal(host(s1.W[0]), batch_W[g])
            assert np.array_equal(host(s1.conflicts(0)[1]), batch_f[g])
            s1.close()


def test_autograd_backward_matches_step_and_finite_differences():
    torch = __import__("torch")
    import paper_1909_02261_amd as pk
    case = tcolgen.case_c2(FP32)
    case.nb_iter = 1000   # no smoothing in the compared step
    s, (A,) = make_solver([case])
    s.set_t(4)
    W = s.W[0]
    W.requires_grad_(True)
    L = pk.TensColLoss.apply(W, s, 0)
    L.backward()
    grad = W.grad.detach().clone()
    W.requires_grad_(False)
    W.grad = None
    # oracle gradient
    p = orc_params(case.params())
    Wh = host(W).astype(np.float64)
    c = oracle.colors(Wh)
    gS_ref = oracle.grad_s(p, 4, A, c, oracle.mtilde(c), oracle.class_sizes(c, case.k))
    gW_ref = oracle.grad_w(Wh, gS_ref)
    assert normwise(host(grad), gW_ref) <= TOL
    # central differences (h = 1e-3, FP64) of the surrogate sum_l G_l softmax(w)_l with G frozen
    _, gs, _ = s.loss_grad(0)
    G = host(gs).astype(np.float64)
    h = 1e-3
    for (d, i, j) in tcolgen.fd_entries(32, case.D, case.n, case.k, seed=2):
        w = Wh[d, i].copy()

        def phi(x):
            e = np.exp(x - x.max())
            return float((G[d, i] * e / e.sum()).sum())
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        fd = (phi(wp) - phi(wm)) / (2 * h)
        assert abs(fd - float(host(grad)[d, i, j])) <= 1e-4 * max(1e-3, abs(fd)) + 1e-6
    # W - eta * grad equals the library's own update step
    W_exp = host(W) - np.float32(case.eta) * host(grad)
    s.step(1)
    assert normwise(host(s.W[0]), W_exp) <= 1e-6
    s.close()


@pytest.mark.parametrize("mk", [lambda: tcolgen.case_c4(BF16), lambda: tcolgen.case_c3(FP8), lambda: tcolgen.case_c3(BF16),
                                lambda: tcolgen.case_c3(FP4)],
                         ids=["C4_ecp_bf16", "C3_fp8", "C3_bf16", "C3_fp4"])
def test_full_size_conflicts_and_equity_exact(mk):
    case = mk()
    s, (A,) = make_solver([case])
    for it in range(3):
        c, fc, fe = s.conflicts(0)
        W = host(s.W[0])
        c_ref = oracle.colors(W)
        assert np.array_equal(host(c), c_ref)
        assert np.array_equal(host(fc), oracle.fcolor(A, c_ref))
        if case.problem == ECP:
            assert np.array_equal(host(fe), oracle.feq(oracle.class_sizes(c_ref, case.k), case.n))
        s.step(7)
    s.close()


@pytest.mark.parametrize("prec", [FP8, FP4], ids=["fp8", "fp4"])
def test_c5_full_size(prec):
    case = tcolgen.case_c5(prec)
    s, (A,) = make_solver([case])
    s.set_t(100)
    c, fc, fe = s.conflicts(0)
    W = host(s.W[0])
    c_ref = oracle.colors(W)
    assert np.array_equal(host(c), c_ref)
    assert np.array_equal(host(fc), oracle.fcolor(A, c_ref))
    assert np.array_equal(host(s.mtilde(0)), oracle.mtilde(c_ref))
    check_loss_grad(case, s, A, 100)
    s.close()


@pytest.mark.parametrize("penalty", ["dense", "sparse"])
@pytest.mark.parametrize("prec", [FP8, FP4], ids=["fp8", "fp4"])
def test_c5_full_size_step(prec, penalty):
    """One fast-path step at the benchmark's size (n = 4000, k = 280, D = 32) in fp8 (the
    configuration's own A.S operands) and fp4, with the penalty active and each route forced,
    against the oracle's iteration from the same weights: the sparse rows sum FP32 values
    exactly, the dense pass rounds its operand to bf16."""
    case = tcolgen.case_c5(prec)
    case.stop_on_legal = 0
    opts = dict(fused=1, penalty={"dense": 1, "sparse": 2}[penalty])
    s, (A,) = make_solver([case], **opts)
    t = 40
    s.set_t(t)
    W0 = host(s.W[0])
    before = s.counters()
    done, _ = s.step(1)
    route = step_route(s, before)
    assert done == 1 and route == penalty
    p = orc_params(case.params())
    ref, W_route, bound = reference_step(p, t, A, W0, route, prec)
    W1 = host(s.W[0])
    e_r, e_x = normwise(W1, W_route), normwise(W1, ref.W)
    print(f"C5 {prec} {penalty}: W error against the route's operand {e_r:.2e}, against FP64 {e_x:.2e} "
          f"(bound {bound / np.abs(ref.W).max():.2e})")
    assert e_r <= TOL
    assert np.abs(W1 - ref.W).max() <= bound + TOL * np.abs(ref.W).max()
    c, fc, _ = s.conflicts(0)
    c_ref = oracle.colors(W1)
    assert np.array_equal(host(c), c_ref)
    assert np.array_equal(host(fc), oracle.fcolor(A, c_ref))
    s.close()


def test_c4_full_size_step_loss_and_autotuned_tile():
    """C4 (ECP, G(1000, .5), k = 90, D = 256, bf16 operands, hipGraph-captured fast step): one
    resynced step at full size against the oracle (W' at 1e-5 against the bf16-operand
    reference, within the rounding bound of FP64), loss and gradients at full size, then the
    autotuner: its choice keeps W and t, the integer results with its tile equal those of
    the default tile, and one more resynced step with it holds the same bar.  A second
    autotune call on a context of the same signature takes the cached choice."""
    case = tcolgen.case_c4(BF16)
    case.stop_on_legal = 0
    s, (A,) = make_solver([case])
    p = orc_params(case.params())
    t = 40
    s.set_t(t)

    def resynced_step(t, opts):
        W0 = host(s.W[0])
        before = s.counters()
        done, _ = s.step(1)
        route = step_route(s, before)
        ref, W_route, bound = reference_step(p, t, A, W0, route, BF16)
        assert done == 1 and route == expected_route(case, opts, t, ref.colors)
        W1 = host(s.W[0])
        e_r, e_x = normwise(W1, W_route), normwise(W1, ref.W)
        print(f"C4 step t={t}: W error against the bf16-operand reference {e_r:.2e}, against FP64 {e_x:.2e}")
        assert e_r <= TOL
        assert np.abs(W1 - ref.W).max() <= bound + TOL * np.abs(ref.W).max()
        return W1

    resynced_step(t, {})
    t += 1
    check_loss_grad(case, s, A, t)
    c0, f0, e0 = (host(x) for x in s.conflicts(0))
    W_before = host(s.W[0]).copy()
    default = s.options()
    bm, ntw = s.autotune()
    tuned = s.options()
    print(f"C4 autotune: default {default}, tuned {tuned}")
    assert (tuned["tile_bm"], tuned["tile_ntw"]) == (bm, ntw)
    assert np.array_equal(host(s.W[0]), W_before) and s.get_t() == t
    c1, f1, e1 = (host(x) for x in s.conflicts(0))
    assert np.array_equal(c0, c1) and np.array_equal(f0, f1) and np.array_equal(e0, e1)
    resynced_step(t, tuned)
    s.close()
    s2, _ = make_solver([case])
    assert s2.autotune() == (bm, ntw)
    assert s2.options() == tuned
    s2.close()


@pytest.mark.parametrize("prec", [FP4, FP8])
def test_penalty_pass_every_tile_shape(prec):
    """The dense penalty pass (bf16 P against S; in fp4 mode S comes from the fp4 operand and
    is widened in registers) for every tile shape: gradient with respect to S against the
    oracle on a graph with a ragged n over several row tiles and D k not a multiple of any
    column tile."""
    case = GraphCase("penshapes", KCOL, 1000, 28, 40, prec, "gnp", 0.5, graph_seed=14, lam=1e-2, mu=3e-3,
                     rho=10.0, stop_on_legal=0)
    A = case.adjacency()
    W = case.weights()
    p = orc_params(case.params())
    t = 9
    c = oracle.colors(W.astype(np.float64))
    Mt = oracle.mtilde(c)
    gS_ref = oracle.grad_s(p, t, A, c, Mt, oracle.class_sizes(c, case.k))
    corr, B = penalty_terms(p, t, A, c, Mt, "bf16")
    gS_op = gS_ref + corr
    bS = grad_s_bound(p, "bf16", B, float(np.abs(gS_ref).max()), 1024)
    s, _ = make_solver([case], As=[A], Ws=[W])
    s.set_t(t)
    worst = {}
    for bm, ntw in SHAPES:
        s.set_options(tile_bm=bm, tile_ntw=ntw)
        _, gs, _ = s.loss_grad(0, want_loss=False, want_gw=False)
        gs = host(gs)
        worst[(bm, ntw)] = (normwise(gs, gS_op), normwise(gs, gS_ref))
        assert np.abs(gs - gS_ref).max() <= bS + TOL * np.abs(gS_ref).max(), (bm, ntw)
    s.close()
    print(f"precision {prec}: gradS error per shape (bf16-operand reference, FP64) {worst}")
    assert max(v[0] for v in worst.values()) <= TOL, worst


@pytest.mark.parametrize("prec", [FP32, FP8, FP4])
def test_auto_penalty_small_classes(prec):
    """Per-iteration penalty choice without the size floor (penalty 3) on rows that stay
    sparse (n = 600, k = 60, D = 4: about 40 class-mates per row against n = 600), so
    every iteration takes the sparse rows, which are FP32 in every operand mode."""
    case = GraphCase("auto_sparse", KCOL, 600, 60, 4, prec, "gnp", 0.3, graph_seed=61, rho=10.0,
                     lam=1e-2, mu=3e-3, stop_on_legal=0)
    wr, wx, routes = run_resynced(case, 8, t0=2, fused=1, penalty=3)
    assert set(routes) == {"sparse"}
    print(f"auto penalty, prec {prec}: worst W error vs FP64 {wx:.2e}")


def test_auto_penalty_size_floor():
    """Below the size floor (n = 600) the automatic choice keeps the dense pass even though
    the classes are small: its steps equal those of penalty 1 bit for bit, while penalty 3
    (no floor) takes the sparse FP32 rows, which differ from the bf16 dense operand."""
    case = GraphCase("floor", KCOL, 600, 60, 4, BF16, "gnp", 0.3, graph_seed=61, rho=10.0,
                     lam=1e-2, mu=3e-3, stop_on_legal=0)
    out = {}
    for pen in (0, 1, 3):
        s, _ = make_solver([case], fused=1, penalty=pen)
        s.set_t(2)
        done, _ = s.step(4)
        assert done == 4
        out[pen] = host(s.W[0]).copy()
        s.close()
    assert np.array_equal(out[0], out[1])
    assert not np.array_equal(out[3], out[1])


@pytest.mark.parametrize("path", ["fast_auto", "epi_auto"])
@pytest.mark.parametrize("prec", [FP32, FP8])
def test_auto_penalty_switches(prec, path):
    """Per-iteration penalty choice (penalty 3, no size floor) along a trajectory whose smoothing (rho = 100 every second
    iteration) drives the population in and out of large classes, so iterations take the
    dense pass and the sparse rows in turn (each step's route is the documented one for the
    oracle's colours); FP8 also checks that the bf16 copy of S the dense pass reads is
    written in exactly the iterations that need it."""
    case = GraphCase("auto_switch", KCOL, 400, 40, 4, prec, "gnp", 0.5, graph_seed=62, rho=100.0,
                     nb_iter=2, lam=1e-2, mu=3e-3, stop_on_legal=0)
    W = case.weights()
    W[0, :200, 0] += 0.05       # member 0 starts with a class of 200 vertices
    fused = 1 if path == "fast_auto" else 2
    wr, wx, routes = run_resynced(case, 12, W=W, fused=fused, penalty=3)
    assert "dense" in routes and "sparse" in routes, routes
    print(f"auto switching {path}, prec {prec}: routes {routes}; worst W error against the route's operand "
          f"{wr:.2e}, against FP64 {wx:.2e}")


@pytest.mark.parametrize("prec", [BF16, FP4], ids=["bf16", "fp4"])
@pytest.mark.parametrize("penalty", [0, 3])
def test_c5b_batch_steps_every_graph(penalty, prec):
    """The uneven batch (16 graphs, n from 250 to 2000, p cycling .1/.5/.9, each with its
    greedy colour count as k, D = 16) in one context: one launch sequence steps all of them.
    With penalty 0 every graph is below the sparse rows' size floor and takes the bf16
    dense pass; with penalty 3 the penalty is taken per graph and iteration (sparse rows
    or the dense pass).  Three resynced steps from t = 10, each compared with the oracle
    graph by graph (each graph's own route), colours and conflict counts exact after each."""
    cases = tcolgen.cases_c5b(prec)
    for c in cases:
        c.stop_on_legal = 0
    opts = dict(penalty=penalty)
    s, As = make_solver(cases, **opts)
    t = 10
    s.set_t(t)
    for g in range(1, len(cases)):
        s.set_t(t, g)
    worst_r = worst_x = 0.0
    for _ in range(3):
        W0 = [host(w).copy() for w in s.W]
        before = [s.counters(g) for g in range(len(cases))]
        done, _ = s.step(1)
        assert done == 1
        for g, c in enumerate(cases):
            route = step_route(s, before[g], g)
            p = orc_params(c.params())
            ref, W_route, bound = reference_step(p, t, As[g], W0[g], route, prec)
            assert route == expected_route(c, opts, t, ref.colors), (c.name, route)
            W1 = host(s.W[g])
            e_r, e_x = normwise(W1, W_route), normwise(W1, ref.W)
            worst_r, worst_x = max(worst_r, e_r), max(worst_x, e_x)
            assert e_r <= TOL, (c.name, route, e_r)
            assert np.abs(W1 - ref.W).max() <= bound + TOL * np.abs(ref.W).max(), (c.name, e_x)
            col, fc, _ = s.conflicts(g)
            c_ref = oracle.colors(W1)
            assert np.array_equal(host(col), c_ref)
            assert np.array_equal(host(fc), oracle.fcolor(As[g], c_ref))
        t += 1
    print(f"C5b {prec} penalty {penalty}: worst W error over 16 graphs against the route's operand {worst_r:.2e}, "
          f"against FP64 {worst_x:.2e}")
    s.close()


@pytest.mark.parametrize("case", [GraphCase("cc_ragged", KCOL, 77, 7, 5, FP4, "gnp", 0.4, graph_seed=7),
                                  GraphCase("cc_k90", ECP, 300, 90, 6, BF16, "gnp", 0.5, graph_seed=9, mu=0.0, nu=1e-5),
                                  GraphCase("cc_kpart", tcolgen.KPART, 150, 5, 4, FP8, "gnp", 0.3, graph_seed=10),
                                  GraphCase("cc_fp32_k130", KCOL, 500, 130, 3, FP32, "gnp", 0.5, graph_seed=11)],
                         ids=lambda c: c.name)
def test_class_conflicts_exact(case):
    """S_d^T A S_d on MFMA (one-hot S^T against the contraction's A.S) equals the oracle's edge
    count between colour classes, for ragged n, k not a multiple of the 16 x 16 tiles and every
    operand precision; its trace is twice the conflict count tcol_conflicts reports (for
    partitioning: the same matrix of the groups)."""
    s, (A,) = make_solver([case])
    C = host(s.class_conflicts(0))
    c_ref = oracle.colors(host(s.W[0]))
    assert np.array_equal(C, oracle.class_conflicts(A, c_ref, case.k))
    _, fc, _ = s.conflicts(0)
    trace = np.trace(C, axis1=1, axis2=2)
    if case.problem == tcolgen.KPART:
        assert np.array_equal(host(fc), A.sum() // 2 - trace // 2)
    else:
        assert np.array_equal(host(fc), trace // 2)
    s.close()


def test_class_conflicts_c5():
    """The class-conflict matrices at n = 4000, k = 280, D = 32 (fp4 A.S), bit-exact."""
    case = tcolgen.case_c5(FP4)
    s, (A,) = make_solver([case])
    s.set_t(30)
    s.step(3)
    C = host(s.class_conflicts(0))
    assert np.array_equal(C, oracle.class_conflicts(A, oracle.colors(host(s.W[0])), case.k))
    s.close()


@pytest.mark.parametrize("prec,published", [(FP4, 10100.0), (FP8, 5000.0), (BF16, 2500.0), (FP32, 157.3)],
                         ids=["fp4", "fp8", "bf16", "fp32"])
def test_mfma_peak_measurement_is_plausible(prec, published):
    """The MFMA throughput measurement runs and lands between a quarter of and slightly
    above the published dense peak of its operand type (TFLOP/s)."""
    import paper_1909_02261_amd as pk
    v = max(pk.mfma_peak(prec, 1000) for _ in range(2))
    print(f"measured {v:.1f} TFLOP/s against {published}")
    assert 0.25 * published < v < 1.1 * published
