"""Helpers for the GPU parity tests: build solver inputs from seeded cases and compare with the oracle."""
from __future__ import annotations

import numpy as np

import oracle
import tcolgen


def torch_mod():
    import torch
    return torch


def lib_params(case_params: dict):
    import paper_1909_02261_amd as pk
    return pk.Params.from_dict(case_params)


def orc_params(case_params: dict) -> oracle.Params:
    """Oracle parameters with the real-valued ones rounded to fp32, as the C ABI carries them."""
    d = dict(case_params)
    for key in ("eta", "rho", "alpha", "lam", "beta", "mu", "nu", "momentum"):
        d[key] = float(np.float32(d[key]))
    return oracle.Params.from_dict(d)


def make_solver(cases, As=None, Ws=None, **opts):
    """cases: list of GraphCase; returns (solver, A list (np), W tensors)."""
    torch = torch_mod()
    import paper_1909_02261_amd as pk
    graphs, params, Anp = [], [], []
    for idx, c in enumerate(cases):
        A = c.adjacency() if As is None else As[idx]
        W = c.weights() if Ws is None else Ws[idx]
        Anp.append(A)
        graphs.append((torch.from_numpy(np.ascontiguousarray(A)).cuda(),
                       torch.from_numpy(np.ascontiguousarray(W, dtype=np.float32)).cuda()))
        params.append(pk.Params.from_dict(c.params()))
    s = pk.Solver(graphs, params)
    if opts:
        s.set_options(**opts)
    return s, Anp


def normwise(got, ref) -> float:
    """max |got - ref| / max |ref| (0 when both vanish)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max() if ref.size else 0.0
    num = np.abs(got - ref).max() if ref.size else 0.0
    if den == 0.0:
        return float(num)
    return float(num / den)


def loss_scale(p: oracle.Params, t: int, ref) -> float:
    """Tolerance scale of the loss: sum|f_color| + nu t sum|f_eq| + lambda t |kappa| + mu t |varpi|."""
    return abs(ref[1]) + p.nu * t * abs(ref[2]) + p.lam * t * abs(ref[3]) + p.mu * t * abs(ref[4]) + 1e-300


# ---------------------------------------------------------------------------------------
# the penalty operand in the precision each route computes it, for reference steps
# ---------------------------------------------------------------------------------------

U_BF16 = 2.0 ** -8      # unit roundoff of bf16 (8 significant bits, round to nearest even)
U_FP32 = 2.0 ** -24


def bf16_rne(x32: np.ndarray) -> np.ndarray:
    """float32 values rounded to bf16 (nearest, ties to even), returned as float32."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def _is_partition(p) -> bool:
    return p.problem in (tcolgen.KPART, tcolgen.BKPART)


def operand_values(p, t: int, A: np.ndarray, Mt: np.ndarray, form: str) -> np.ndarray:
    """The penalty operand P of eq. (17) (the matrix the contraction multiplies by S, before the
    sign of partitioning), n x n, as FP64 values of the given form:
      "fp64"  t (a 2 alpha lambda x^(alpha-1) - (1 - a) [j != i or bonus_diag] 2 beta mu x^(beta-1));
      "fp32"  the same built in single precision as the library declares it (tables of the two
              coefficients rounded to fp32, times t in fp32);
      "bf16"  the fp32 form rounded to bf16, the operand of the dense pass in the bf16, fp8 and
              fp4 modes;
    x = Mt, or D - Mt for partitioning."""
    n = A.shape[0]
    x = (p.D - Mt) if _is_partition(p) else Mt
    x = x.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        pen = np.where(x > 0, 2.0 * p.alpha * p.lam * np.power(x, p.alpha - 1.0), 0.0)
        bon = np.where(x > 0, 2.0 * p.beta * p.mu * np.power(x, p.beta - 1.0), 0.0)
    edge = A.astype(bool)
    keep = ~edge
    if not p.bonus_diag:
        keep = keep & ~np.eye(n, dtype=bool)
    if form == "fp64":
        return np.where(edge, t * pen, np.where(keep, -t * bon, 0.0))
    t32 = np.float32(t)
    v = np.where(edge, t32 * pen.astype(np.float32), np.where(keep, -(t32 * bon.astype(np.float32)), 0.0))
    v = v.astype(np.float32)
    if form == "bf16":
        v = bf16_rne(v)
    elif form != "fp32":
        raise ValueError(form)
    return v.astype(np.float64)


def class_product(X: np.ndarray, c: np.ndarray, k: int) -> np.ndarray:
    """X . S_d for every member (S_d the one-hot matrix of colours c[d]): [D, n, k]."""
    D = c.shape[0]
    n = X.shape[0]
    out = np.zeros((D, n, k))
    for d in range(D):
        order = np.argsort(c[d], kind="stable")
        counts = np.bincount(c[d], minlength=k)
        starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
        nz = np.nonzero(counts)[0]
        out[d][:, nz] = np.add.reduceat(X[:, order], starts[nz], axis=1)
    return out


def route_form(route: str, precision: int) -> str:
    """Precision of the penalty operand on a route: the dense pass rounds it to bf16 unless every
    operand is fp32; the sparse rows sum its fp32 values exactly."""
    return "bf16" if route == "dense" and precision != tcolgen.FP32 else "fp32"


def penalty_terms(p, t, A, c, Mt, form: str):
    """(sgn (P_form - P_fp64) . S, max over (d, i, l) of (|P_fp64| . S)): the change the route's
    operand precision makes to the oracle's gradient with respect to S, and the magnitude
    that bounds it."""
    P64 = operand_values(p, t, A, Mt, "fp64")
    sgn = -1.0 if _is_partition(p) else 1.0
    dP = operand_values(p, t, A, Mt, form) - P64 if form != "fp64" else np.zeros_like(P64)
    corr = sgn * class_product(dP, c, p.k) if np.any(dP) else np.zeros((p.D, p.n, p.k))
    B = float(class_product(np.abs(P64), c, p.k).max()) if np.any(P64) else 0.0
    return corr, B


def grad_s_bound(p, form: str, B: float, gs_max: float, n_pad: int) -> float:
    """Bound on max |gS_gpu - gS_fp64| from the arithmetic: the operand rounding (unit roundoff
    of its form) on every penalty term, plus FP32 accumulation over n_pad terms of partial sums
    no larger than max |A.S| + max (|P| . S) <= max |gS| + 2 max (|P| . S)."""
    u = U_BF16 if form == "bf16" else U_FP32
    return u * B + n_pad * U_FP32 * (gs_max + 2.0 * B)


def reference_step(p, t: int, A: np.ndarray, W0: np.ndarray, route: str, precision: int):
    """The FP64 oracle's iteration from W0, and beside it the same iteration with the penalty
    operand in the precision the GPU route computes it (route: "dense", "sparse" or "none").
    Returns (oracle result, W' of the route's arithmetic, bound on max |W'_gpu - W'_fp64| from
    the operand rounding and FP32 accumulation: |dgW| <= 2 max |dgS| since the softmax weights
    sum to one, times eta, over rho when the step smooths)."""
    ref = oracle.iteration(p, t, A, W0, want_grads=True)
    if ref.status != 0 or route == "none":
        return ref, ref.W, 0.0
    form = route_form(route, precision)
    c = ref.colors
    Mt = oracle.mtilde(c)
    corr, B = penalty_terms(p, t, A, c, Mt, form)
    gS = ref.gS + corr
    W_route = oracle.update(p, t, np.asarray(W0, np.float64), oracle.grad_w(np.asarray(W0, np.float64), gS))
    n_pad = -(-p.n // 256) * 256
    bound = 2.0 * p.eta * grad_s_bound(p, form, B, float(np.abs(ref.gS).max()), n_pad)
    if p.nb_iter > 0 and (t + 1) % p.nb_iter == 0:
        bound /= p.rho
    return ref, W_route, bound


def step_route(solver, before: dict, g: int = 0) -> str:
    """Route the last evaluated iteration of graph g took, from the counters (before: the counters
    read before that iteration)."""
    after = solver.counters(g)
    diff = {key: after[key] - before[key] for key in before}
    assert sum(diff.values()) == 1, diff
    return {"no_penalty": "none", "dense": "dense", "sparse": "sparse"}[[key for key, v in diff.items() if v][0]]


def expected_route(case, opts: dict, t: int, c: np.ndarray) -> str:
    """Route the library documents for the penalty product of graph `case` at iteration t with
    colours c (include/tcol.h, tcol_options.penalty): none while lambda t = mu t = 0; the plain
    schedule and penalty 1 the dense pass; penalty 2 the sparse rows; penalty 0 and 3 the sparse
    rows for graphs that prefer them (partitioning, or 4 D <= k; with penalty 0 only from
    n = 2048 for partitioning and n = 2750 for colouring) in the iterations whose rows average at
    most n class-mates (sum_d sum_l #V_dl^2 <= n^2; partitioning always), else dense."""
    t32 = np.float32(t)
    if np.float32(case.lam) * t32 == 0 and np.float32(case.mu) * t32 == 0:
        return "none"
    pen = opts.get("penalty", 0)
    if opts.get("fused", 1) == 0 or pen == 1:
        return "dense"
    if pen == 2:
        return "sparse"
    part = case.problem in (tcolgen.KPART, tcolgen.BKPART)
    if part:
        pref = pen == 3 or case.n >= 2048
    else:
        pref = 4 * case.D <= case.k and (pen == 3 or case.n >= 2750)
    if not pref:
        return "dense"
    if part:
        return "sparse"
    V = oracle.class_sizes(c, case.k).astype(np.int64)
    return "dense" if int((V * V).sum()) > case.n * case.n else "sparse"


def run_resynced(case, steps, check_every=1, t0=0, W=None, check_routes=True, **opts):
    """Step the GPU one iteration at a time; before each step the oracle starts from the same
    weights.  Each W' is compared with the oracle's iteration taken with the penalty operand in
    the precision of the route the GPU took (1e-5 norm-wise, the FP32 bar), and with the exact
    FP64 iteration within the bound that precision implies; the stop decision is exact, and
    every `check_every` steps the colours and fitness after the step are bit-exact.  With
    check_routes the route taken must be the documented one (expected_route).
    Returns (worst error against the route's reference, worst error against FP64, routes)."""
    s, (A,) = make_solver([case], Ws=None if W is None else [W], **opts)
    p = orc_params(case.params())
    t = t0
    if t0:
        s.set_t(t0)
    worst_r = worst_x = 0.0
    routes = []
    for it in range(steps):
        W0 = host(s.W[0])
        before = s.counters()
        done, legal = s.step(1)
        route = step_route(s, before)
        routes.append(route)
        ref, W_route, bound = reference_step(p, t, A, W0, route, case.precision)
        if check_routes:
            assert route == expected_route(case, opts, t, ref.colors), (it, route)
        if ref.status == 1:
            assert done == 0 and legal[0] == ref.legal_d
            assert np.array_equal(host(s.W[0]), W0)
            break
        assert done == 1 and legal[0] == -1
        W1 = host(s.W[0])
        e_r = normwise(W1, W_route)
        e_x = normwise(W1, ref.W)
        worst_r, worst_x = max(worst_r, e_r), max(worst_x, e_x)
        assert e_r <= 1e-5, (it, route, e_r)
        assert np.abs(W1 - ref.W).max() <= bound + 1e-5 * np.abs(ref.W).max(), (it, route, e_x, bound)
        if it % check_every == 0:
            c, fm, fs = s.conflicts(0)
            c_ref = oracle.colors(W1)
            fm_ref, fs_ref, _ = oracle.fitness(p, A, c_ref)
            assert np.array_equal(host(c), c_ref)
            assert np.array_equal(host(fm), fm_ref) and np.array_equal(host(fs), fs_ref)
        t += 1
        assert s.get_t() == t
    s.close()
    return worst_r, worst_x, routes


def host(t):
    return t.detach().cpu().numpy()


def check_loss_grad(case, s, A, t, g=0):
    """loss_grad of graph g at t against the oracle: integer parts exact, kappa / varpi within
    the FP64 summation bound n^2 2^-52, the loss to 1e-5 of its scale; gS and gW at 1e-5 against the oracle with the
    penalty operand in the dense pass's precision (this call always takes the dense pass),
    and against the exact FP64 oracle within the bound that precision implies.  Returns
    the errors against FP64."""
    loss, gs, gw = s.loss_grad(g)
    W = host(s.W[g]).astype(np.float64)
    p = orc_params(case.params())
    c = oracle.colors(W)
    V = oracle.class_sizes(c, case.k)
    Mt = oracle.mtilde(c)
    gS_ref = oracle.grad_s(p, t, A, c, Mt, V)
    gW_ref = oracle.grad_w(W, gS_ref)
    fm, fs, _ = oracle.fitness(p, A, c)
    L_ref = oracle.loss(p, t, A, Mt, fm, fs)
    loss = host(loss)
    form = route_form("dense", case.precision)
    corr, B = penalty_terms(p, t, A, c, Mt, form)
    gS_op = gS_ref + corr
    gW_op = oracle.grad_w(W, gS_op)
    gs, gw = host(gs), host(gw)
    eS, eW = normwise(gs, gS_ref), normwise(gw, gW_ref)
    eS_op, eW_op = normwise(gs, gS_op), normwise(gw, gW_op)
    eL = abs(loss[0] - L_ref[0]) / loss_scale(p, t, L_ref)
    n_pad = -(-case.n // 256) * 256
    bS = grad_s_bound(p, form, B, float(np.abs(gS_ref).max()), n_pad)
    print(f"{case.name} t={t} ({form} operand): against FP64 gradS {eS:.2e} gradW {eW:.2e} "
          f"(bound on |dgS| {bS:.2e}); against the {form}-operand reference {eS_op:.2e} {eW_op:.2e}; "
          f"loss {eL:.2e}")
    assert loss[1] == L_ref[1] and loss[2] == L_ref[2]
    # kappa and varpi: n^2 positive FP64 terms summed in two different orders, each sum within
    # n^2 2^-53 of its terms' total
    tol_kv = case.n * case.n * 2.0 ** -52
    print(f"kappa {abs(loss[3] - L_ref[3]) / max(1.0, abs(L_ref[3])):.2e} varpi "
          f"{abs(loss[4] - L_ref[4]) / max(1.0, abs(L_ref[4])):.2e} (bound {tol_kv:.2e})")
    assert abs(loss[3] - L_ref[3]) <= tol_kv * max(1.0, abs(L_ref[3]))
    assert abs(loss[4] - L_ref[4]) <= tol_kv * max(1.0, abs(L_ref[4]))
    assert eL <= 1e-5
    assert eS_op <= 1e-5 and eW_op <= 1e-5, (eS_op, eW_op)
    assert np.abs(gs - gS_ref).max() <= bS + 1e-5 * np.abs(gS_ref).max()
    # the softmax weights sum to one, so |dgW| <= 2 max |dgS|
    assert np.abs(gw - gW_ref).max() <= 2 * bS + 1e-5 * np.abs(gW_ref).max()
    return eS, eW, eL
