"""GPU parity, through the C ABI, of the other problems of Section 6 and the momentum
optimiser variant of Section 7, against the FP64 oracle.

k-partitioning (plain and balanced) replaces the association matrix M by J - M: the
fitness is the cut, the fitness term of the gradient is -A.S and the group concentration
enters the penalty and bonus as D - Mt.  Minimum sum colouring replaces the equity term
by the colour cost z_l = l + 1.  Heavy-ball momentum carries a velocity across steps, so
it is compared over an unsynchronised trajectory.  Integer results (colours, fitness,
stop decision) are bit-exact; FP32 tensors within 1e-5 norm-wise, as for colouring
(in the low-precision modes against the oracle with the dense pass's bf16 operand, and
against the exact FP64 oracle within the bound of that rounding).
"""
import numpy as np
import pytest

import oracle
import tcolgen
from tcolgen import BF16, BKPART, FP4, FP8, FP32, KCOL, KPART, MSCP, GraphCase

from gpu_util import check_loss_grad, host, make_solver, normwise, orc_params, run_resynced

pytestmark = pytest.mark.gpu

TOL = 1e-5
PROBLEMS = {"kpart": KPART, "bkpart": BKPART, "mscp": MSCP}
PATHS = {"plain": dict(fused=0), "fast_dense": dict(fused=1, penalty=1), "fast_sparse": dict(fused=1, penalty=2),
         "epi_dense": dict(fused=2, penalty=1), "epi_sparse": dict(fused=2, penalty=2)}


def case_for(problem, prec, n=131, k=9, D=6, seed=51, **kw):
    d = dict(rho=10.0, lam=1e-2, mu=3e-3, nu=0.05 if problem in (BKPART, MSCP) else 0.0)
    d.update(kw)
    return GraphCase(f"prob{problem}_n{n}_k{k}_D{D}_p{prec}", problem, n, k, D, prec, "gnp", 0.45,
                     graph_seed=seed, **d)


def fitness_ref(case, A, c):
    p = orc_params(case.params())
    return oracle.fitness(p, A, c)


@pytest.mark.parametrize("prec", [FP32, BF16, FP8, FP4])
@pytest.mark.parametrize("name", list(PROBLEMS))
def test_fitness_bit_exact(name, prec):
    case = case_for(PROBLEMS[name], prec)
    s, (A,) = make_solver([case])
    c, fm, fs = s.conflicts(0)
    c_ref = oracle.colors(host(s.W[0]))
    fm_ref, fs_ref, _ = fitness_ref(case, A, c_ref)
    assert np.array_equal(host(c), c_ref)
    assert np.array_equal(host(fm), fm_ref)
    assert np.array_equal(host(fs), fs_ref)
    s.close()


@pytest.mark.parametrize("t", [0, 4, 31])
@pytest.mark.parametrize("prec", [FP32, FP4])
@pytest.mark.parametrize("name", list(PROBLEMS))
def test_loss_and_gradients(name, prec, t):
    case = case_for(PROBLEMS[name], prec)
    s, (A,) = make_solver([case])
    s.set_t(t)
    check_loss_grad(case, s, A, t)
    s.close()


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("name", list(PROBLEMS))
def test_resynced_steps_every_path(name, path):
    """Ragged n over several tiles; D k = 80 columns, so the epilogue path holds whole members."""
    case = case_for(PROBLEMS[name], FP32, n=300, k=10, D=8, seed=52, stop_on_legal=0)
    wr, wx, _ = run_resynced(case, 8, **PATHS[path])
    print(f"{case.name} {path}: worst W error {wr:.2e} (FP64 {wx:.2e})")


@pytest.mark.parametrize("prec", [BF16, FP8, FP4])
@pytest.mark.parametrize("name", list(PROBLEMS))
def test_resynced_low_precision(name, prec):
    case = case_for(PROBLEMS[name], prec, stop_on_legal=0)
    for pen, what in ((2, "FP32 sparse penalty rows"), (1, "bf16 dense penalty operand")):
        wr, wx, _ = run_resynced(case, 5, fused=1, penalty=pen)
        print(f"{case.name} {what}: worst W error against the route's operand {wr:.2e}, against FP64 {wx:.2e}")


def test_partition_stop_on_zero_cut():
    """k disjoint cliques: the partition into the cliques cuts no edge, so a member holding
    it is legal and the run stops before its update, as Algorithm 1 does for colourings."""
    k, size, D = 5, 12, 4
    n = k * size
    A = np.zeros((n, n), np.uint8)
    for q in range(k):
        A[q * size:(q + 1) * size, q * size:(q + 1) * size] = 1
    np.fill_diagonal(A, 0)
    rng = np.random.default_rng(3)
    c = rng.integers(0, k, size=(D, n)).astype(np.int16)
    c[1] = np.arange(n) // size
    c[3] = (np.arange(n) // size + 2) % k
    W = rng.uniform(-1.0, 0.0, size=(D, n, k))
    for d in range(D):
        W[d, np.arange(n), c[d]] = 1.0
    W = (W * 0.01).astype(np.float32)
    for problem in (KPART, BKPART):
        case = GraphCase("cliques", problem, n, k, D, FP32, "gnp", 0.5, rho=10.0, lam=1e-2, mu=3e-3,
                         nu=0.05 if problem == BKPART else 0.0)
        s, _ = make_solver([case], As=[A], Ws=[W])
        col = __import__("torch").zeros(n, dtype=__import__("torch").int16, device="cuda")
        done, legal = s.step(10, colors_out=[col])
        ref = oracle.iteration(orc_params(case.params()), 0, A, W)
        assert ref.status == 1 and ref.legal_d == 1
        assert done == 0 and legal == [1]
        assert np.array_equal(host(col), c[1])
        np.testing.assert_array_equal(host(s.W[0]), W)
        s.close()


@pytest.mark.parametrize("gamma", [0.5, 0.9])
@pytest.mark.parametrize("path", ["plain", "fast_dense", "fast_sparse", "epi_dense"])
@pytest.mark.parametrize("problem", [KCOL, BKPART])
def test_momentum_trajectory(problem, path, gamma):
    """Heavy-ball steps from the same weights: the GPU trajectory (velocity kept on the device)
    follows the oracle's over 8 steps, colours and fitness exact at each step.  The epilogue
    schedule is not used with momentum; asking for it runs the fast one."""
    case = case_for(problem, FP32, n=120, k=8, D=5, seed=53, stop_on_legal=0, momentum=gamma, eta=0.05,
                    nu=0.05 if problem == BKPART else 0.0)
    s, (A,) = make_solver([case], **PATHS[path])
    p = orc_params(case.params())
    W = host(s.W[0]).astype(np.float64)
    vel = np.zeros_like(W)
    worst = 0.0
    for t in range(8):
        r = oracle.iteration(p, t, A, W, want_grads=False, vel=vel)
        W = r.W
        done, _ = s.step(1)
        assert done == 1
        e = normwise(host(s.W[0]), W)
        worst = max(worst, e)
        assert e <= TOL, (t, e)
        c, fm, fs = s.conflicts(0)
        c_ref = oracle.colors(W)
        assert np.array_equal(host(c), c_ref)
        fm_ref, fs_ref, _ = oracle.fitness(p, A, c_ref)
        assert np.array_equal(host(fm), fm_ref) and np.array_equal(host(fs), fs_ref)
    print(f"momentum {gamma} {path}: worst W error {worst:.2e}")
    # a resume from a checkpoint (set_t) restarts the velocity
    s.set_t(0)
    W0 = host(s.W[0]).astype(np.float64)
    r = oracle.iteration(p, 0, A, W0, want_grads=False, vel=np.zeros_like(W0))
    s.step(1)
    assert normwise(host(s.W[0]), r.W) <= TOL
    s.close()


@pytest.mark.parametrize("k", [300, 576])
@pytest.mark.parametrize("added,gamma", [(0, 0.0), (1, 0.0), (0, 0.9), (1, 0.9)],
                         ids=["plain", "added", "momentum", "added_momentum"])
def test_fast_path_many_colours(added, gamma, k):
    """k from 289 to 576 on the fast schedule: the row update holds 24 or 36 colours per
    lane, with and without the added fitness term (colour cost) and the velocity.  The
    trajectory follows the oracle over 4 steps, colours and fitness exact at each step."""
    case = case_for(MSCP if added else KCOL, FP32, n=333, k=k, D=4, seed=57, stop_on_legal=0, momentum=gamma,
                    eta=0.05)
    s, (A,) = make_solver([case], fused=1)
    p = orc_params(case.params())
    W = host(s.W[0]).astype(np.float64)
    vel = np.zeros_like(W)
    worst = 0.0
    for t in range(4):
        r = oracle.iteration(p, t, A, W, want_grads=False, vel=vel)
        W = r.W
        done, _ = s.step(1)
        assert done == 1
        e = normwise(host(s.W[0]), W)
        worst = max(worst, e)
        assert e <= TOL, (t, e)
        c, fm, fs = s.conflicts(0)
        c_ref = oracle.colors(W)
        assert np.array_equal(host(c), c_ref)
        fm_ref, fs_ref, _ = oracle.fitness(p, A, c_ref)
        assert np.array_equal(host(fm), fm_ref) and np.array_equal(host(fs), fs_ref)
    print(f"k={k} added={added} momentum={gamma}: worst W error {worst:.2e}")
    s.close()
