"""GPU parity of multicolouring (Section 6: vertex i takes its c_i colours of largest weight)
through the C ABI against the FP64 oracle: the selection, the conflict count over shared
colours and the group concentration bit-exact; loss, gradients and resynced steps within 1e-5
norm-wise (the bf16-operand modes against the oracle with the operand rounded as declared,
and against exact FP64 within the bound that rounding implies); the stop on a legal member;
argument errors."""
import numpy as np
import pytest

import oracle
import tcolgen
from tcolgen import BF16, FP4, FP8, FP32

from gpu_util import grad_s_bound, host, loss_scale, normwise, operand_values, orc_params

pytestmark = pytest.mark.gpu

TOL = 1e-5
MCOL = 5


def mparams(n, k, D, prec, cmax, **kw):
    d = dict(problem=MCOL, precision=prec, n=n, k=k, D=D, eta=1e-3, rho=10.0, nb_iter=5, alpha=2.5, lam=1e-2,
             beta=1.2, mu=3e-3, nu=0.0, bonus_diag=1, stop_on_legal=0, momentum=0.0, max_demand=cmax)
    d.update(kw)
    return d


def make(d, A, W, demand, **opts):
    torch = __import__("torch")
    import paper_1909_02261_amd as pk
    s = pk.Solver([(torch.from_numpy(A).cuda(), torch.from_numpy(np.ascontiguousarray(W, np.float32)).cuda())],
                  [pk.Params.from_dict(d)])
    if demand is not None:
        s.set_demand(demand)
    if opts:
        s.set_options(**opts)
    return s


def oparams(d):
    return orc_params(d)


def case(n, k, D, prec, cmax, seed, p=0.4, ties=False, **kw):
    rng = np.random.default_rng(seed)
    A = tcolgen.gnp(n, p, seed)
    if ties:
        W = rng.integers(-2, 3, size=(D, n, k)).astype(np.float32) * np.float32(0.01)
    else:
        W = tcolgen.weights0(D, n, k, seed)
    demand = rng.integers(1, cmax + 1, size=n).astype(np.int32)
    return mparams(n, k, D, prec, cmax, **kw), A, W, demand


def sel_host(S):
    """multi-hot [D, n, k] -> the selection layout [D, n, cmax] cannot be compared directly (order
    within a vertex is by weight); compare as sets via the multi-hot form."""
    return S


def multi_hot(sel, k):
    D, n, cm = sel.shape
    S = np.zeros((D, n, k), np.uint8)
    for s in range(cm):
        d_idx, i_idx = np.nonzero(sel[:, :, s] >= 0)
        S[d_idx, i_idx, sel[d_idx, i_idx, s]] = 1
    return S


def penalty_correction(p, t, A, S, Mt, form):
    """sgn (P_form - P_fp64) . S_d for multi-hot S (matrix products), and max (|P| . S)."""
    P64 = operand_values(p, t, A, Mt, "fp64")
    dP = operand_values(p, t, A, Mt, form) - P64
    Sf = S.astype(np.float64)
    corr = np.stack([dP @ Sf[d] for d in range(S.shape[0])])
    B = float(max((np.abs(P64) @ Sf[d]).max() for d in range(S.shape[0]))) if np.any(P64) else 0.0
    return corr, B


@pytest.mark.parametrize("prec", [FP32, BF16, FP4])
def test_selection_fitness_mtilde_exact(prec):
    d, A, W, dem = case(77, 9, 5, prec, 3, seed=1, ties=True)
    s = make(d, A, W, dem)
    sel = host(s.selection(0))
    S_ref = oracle.select(W.astype(np.float64), dem)
    assert np.array_equal(multi_hot(sel, d["k"]), S_ref)
    # order within a vertex: decreasing weight, lower colour first on ties
    for s_i in range(1, sel.shape[2]):
        a, b = sel[:, :, s_i - 1], sel[:, :, s_i]
        ok = b < 0
        wa = np.take_along_axis(W, np.maximum(a, 0)[..., None].astype(np.int64), axis=2)[..., 0]
        wb = np.take_along_axis(W, np.maximum(b, 0)[..., None].astype(np.int64), axis=2)[..., 0]
        assert np.all(ok | (wa > wb) | ((wa == wb) & (a < b)))
    c, fc, fe = s.conflicts(0)
    assert np.array_equal(host(fc), oracle.fcolor_multi(A, S_ref))
    assert np.all(host(fe) == 0)
    assert np.array_equal(host(c), sel[:, :, 0])
    assert np.array_equal(host(s.mtilde(0)), oracle.mtilde_multi(S_ref))
    s.close()


@pytest.mark.parametrize("prec", [FP32, BF16, FP8, FP4])
@pytest.mark.parametrize("t", [0, 6])
def test_loss_and_gradients(prec, t):
    d, A, W, dem = case(150, 12, 6, prec, 4, seed=2, p=0.5)
    s = make(d, A, W, dem)
    s.set_t(t)
    loss, gs, gw = s.loss_grad(0)
    p = oparams(d)
    Wd = W.astype(np.float64)
    S = oracle.select(Wd, dem)
    Mt = oracle.mtilde_multi(S)
    gS_ref = oracle.grad_s_multi(p, t, A, S, Mt)
    gW_ref = oracle.grad_w(Wd, gS_ref)
    f = oracle.fcolor_multi(A, S)
    L_ref = oracle.loss(p, t, A, Mt, f, np.zeros_like(f))
    loss = host(loss)
    assert loss[1] == L_ref[1] and loss[2] == 0
    tol_kv = d["n"] ** 2 * 2.0 ** -52
    assert abs(loss[3] - L_ref[3]) <= tol_kv * max(1.0, abs(L_ref[3]))
    assert abs(loss[4] - L_ref[4]) <= tol_kv * max(1.0, abs(L_ref[4]))
    assert abs(loss[0] - L_ref[0]) <= TOL * loss_scale(p, t, L_ref)
    form = "fp32" if prec == FP32 else "bf16"
    corr, B = penalty_correction(p, t, A, S, Mt, form)
    gS_op = gS_ref + corr
    gs, gw = host(gs), host(gw)
    eS, eW = normwise(gs, gS_op), normwise(gw, oracle.grad_w(Wd, gS_op))
    bS = grad_s_bound(p, form, B, float(np.abs(gS_ref).max()), 256)
    print(f"MCOL prec {prec} t={t}: against the {form}-operand reference gradS {eS:.2e} gradW {eW:.2e}; against "
          f"FP64 {normwise(gs, gS_ref):.2e} {normwise(gw, gW_ref):.2e} (bound on |dgS| {bS:.2e})")
    assert eS <= TOL and eW <= TOL
    assert np.abs(gs - gS_ref).max() <= bS + TOL * np.abs(gS_ref).max()
    s.close()


@pytest.mark.parametrize("prec,n,k,D,cmax", [(FP32, 120, 15, 6, 3), (FP4, 300, 24, 8, 4), (BF16, 1000, 60, 16, 4)],
                         ids=["fp32_n120", "fp4_n300", "bf16_n1000"])
def test_resynced_steps(prec, n, k, D, cmax):
    """Steps one at a time from the weights the oracle also starts from (the schedule is the
    plain one whatever the options ask): W' within 1e-5 of the route's reference and within the
    rounding bound of FP64; selection and conflicts after each step exact."""
    d, A, W, dem = case(n, k, D, prec, cmax, seed=3, p=0.5)
    s = make(d, A, W, dem, fused=1, penalty=0)
    assert s.options()["fused"] == 0
    p = oparams(d)
    form = "fp32" if prec == FP32 else "bf16"
    t0 = 3
    s.set_t(t0)
    worst = 0.0
    for t in range(t0, t0 + 8):
        W0 = host(s.W[0]).astype(np.float64)
        r = oracle.iteration_multi(p, t, A, W0, dem)
        done, _ = s.step(1)
        assert r.status == 0 and done == 1
        Mt = oracle.mtilde_multi(r.S)
        corr, B = penalty_correction(p, t, A, r.S, Mt, form)
        W_op = oracle.update(p, t, W0, oracle.grad_w(W0, r.gS + corr))
        W1 = host(s.W[0])
        e = normwise(W1, W_op)
        worst = max(worst, e)
        assert e <= TOL, (t, e)
        bound = 2 * p.eta * grad_s_bound(p, form, B, float(np.abs(r.gS).max()), -(-n // 256) * 256)
        if (t + 1) % p.nb_iter == 0:
            bound /= p.rho
        assert np.abs(W1 - r.W).max() <= bound + TOL * np.abs(r.W).max()
        S1 = oracle.select(W1.astype(np.float64), dem)
        assert np.array_equal(multi_hot(host(s.selection(0)), k), S1)
        assert np.array_equal(host(s.conflicts(0)[1]), oracle.fcolor_multi(A, S1))
    print(f"MCOL {prec} n={n}: worst W error against the route's operand {worst:.2e}")
    s.close()


def test_stops_on_a_legal_multicolouring():
    """The 5-cycle with demand 2 and k = 5 (its 2-fold chromatic number): member 1 holds the legal
    2-fold colouring {0,1} {2,3} {4,0} {1,2} {3,4}; the first iteration stops with it, in slot
    order of decreasing weight, and W is unchanged."""
    torch = __import__("torch")
    n, k, D = 5, 5, 3
    A = np.zeros((n, n), np.uint8)
    for i in range(n):
        A[i, (i + 1) % n] = A[(i + 1) % n, i] = 1
    legal = [(0, 1), (2, 3), (4, 0), (1, 2), (3, 4)]
    W = tcolgen.weights0(D, n, k, 9)
    for i, (a, b) in enumerate(legal):
        W[1, i, a] = 2.0
        W[1, i, b] = 1.0
    dem = np.full(n, 2, np.int32)
    for prec in (FP32, FP4):
        d = mparams(n, k, D, prec, 2, stop_on_legal=1)
        s = make(d, A, W, dem)
        col = torch.full((n * 2,), -9, dtype=torch.int16, device="cuda")
        done, legal_d = s.step(5, colors_out=[col])
        assert done == 0 and legal_d == [1]
        assert host(col).reshape(n, 2).tolist() == [list(x) for x in legal]
        assert np.array_equal(host(s.W[0]), W)
        s.close()


def test_errors():
    import paper_1909_02261_amd as pk
    d, A, W, dem = case(40, 6, 3, FP32, 3, seed=4)
    with pytest.raises(pk.TcolError) as ei:
        make(dict(d, momentum=0.5), A, W, None)
    assert ei.value.status == -1
    s = make(d, A, W, None)
    with pytest.raises(pk.TcolError):
        s.set_demand(np.full(40, 4, np.int32))         # above max_demand
    with pytest.raises(pk.TcolError):
        s.set_demand(np.zeros(40, np.int32))
    with pytest.raises(pk.TcolError):
        s.class_conflicts(0)
    # before set_demand every vertex takes one colour: the k-colouring argmax
    sel = host(s.selection(0))
    assert np.array_equal(sel[:, :, 0], oracle.colors(W.astype(np.float64)))
    assert np.all(sel[:, :, 1:] == -1)
    s.close()
    torch = __import__("torch")
    with pytest.raises(pk.TcolError):
        pk.conflicts_noalloc(torch.from_numpy(A).cuda(), torch.from_numpy(W).cuda(), pk.Params.from_dict(d))
