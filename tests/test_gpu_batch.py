"""The batch launch (tcol_options.fused = 3): one kernel launch per run of iterations over every
graph of a context, whose blocks take items from a device queue (class sizes and expansion,
group concentration tiles, contraction tiles, fitness, row-update groups), each item waiting for
its graph's earlier phases (Algorithm 1 per graph)."""
import threading
import time

import numpy as np
import pytest

import oracle
import tcolgen
from gpu_util import expected_route, host, make_solver, normwise, orc_params, reference_step, step_route
from tcolgen import BF16, FP4, FP8, FP32

pytestmark = pytest.mark.gpu

TOL = 1e-5
EABORT = -8


def batch_cases(prec, count=16):
    cases = tcolgen.cases_c5b(prec, count)
    for c in cases:
        c.stop_on_legal = 0
    return cases


@pytest.mark.parametrize("prec", [BF16, FP4], ids=["bf16", "fp4"])
def test_batch_launch_steps_every_graph(prec):
    """The uneven batch (16 graphs, n from 250 to 2000, p cycling .1/.5/.9, k their greedy colour
    counts, D = 16) in the batch launch: three resynced iterations from t = 10, each graph's W'
    against the oracle with the penalty operand of its route (the dense pass: every graph is
    below the sparse rows' size floor) at 1e-5 and against exact FP64 within that operand's
    rounding bound; colours and conflict counts exact after each."""
    cases = batch_cases(prec)
    opts = dict(fused=3)
    s, As = make_solver(cases, **opts)
    assert s.options()["fused"] == 3, "the batch launch is not the schedule that runs"
    t = 10
    for g in range(len(cases)):
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
            assert route == expected_route(c, opts, t, ref.colors) == "dense", (c.name, route)
            W1 = host(s.W[g])
            e_r, e_x = normwise(W1, W_route), normwise(W1, ref.W)
            worst_r, worst_x = max(worst_r, e_r), max(worst_x, e_x)
            assert e_r <= TOL, (c.name, e_r)
            assert np.abs(W1 - ref.W).max() <= bound + TOL * np.abs(ref.W).max(), (c.name, e_x)
            col, fc, _ = s.conflicts(g)
            c_ref = oracle.colors(W1)
            assert np.array_equal(host(col), c_ref)
            assert np.array_equal(host(fc), oracle.fcolor(As[g], c_ref))
        t += 1
    print(f"batch launch {prec}: worst W error against the route's operand {worst_r:.2e}, against FP64 {worst_x:.2e}")
    s.close()


def _run(cases, steps, **opts):
    s, _ = make_solver(cases, **opts)
    for g in range(len(cases)):
        s.set_t(20, g)
    done, legal = s.step(steps)
    W = [host(w) for w in s.W]
    t = [s.get_t(g) for g in range(len(cases))]
    cols = [host(s.conflicts(g)[0]) for g in range(len(cases))]
    s.close()
    return done, legal, W, t, cols


@pytest.mark.parametrize("prec,use_graph", [(BF16, 1), (FP4, 1), (FP8, 0), (FP32, 1)],
                         ids=["bf16", "fp4", "fp8_eager", "fp32"])
def test_batch_launch_equals_fast_schedule(prec, use_graph):
    """Twelve iterations of five uneven graphs in runs of four (so the counter advance between
    runs and the one inside a run are both exercised): the batch launch runs the same block
    bodies as the fast schedule with the same contraction tile, so W, t and the colours are
    bit-identical to the fast schedule's."""
    cases = batch_cases(prec, 5)
    a = _run(cases, 12, fused=3, use_graph=use_graph, unroll=4)
    b = _run(cases, 12, fused=1, use_graph=use_graph, unroll=4, tile_bm=64, tile_ntw=4)
    assert a[0] == b[0] == 12 and a[1] == b[1]
    for g in range(len(cases)):
        assert np.array_equal(a[2][g], b[2][g]), cases[g].name
        assert a[3][g] == b[3][g] == 32
        assert np.array_equal(a[4][g], b[4][g])


def test_batch_launch_wait_limit_aborts_and_recovers():
    """Waits bounded from the host: with a limit of one poll some item gives up, the run reports
    TCOL_EABORT after every block has exited, and the context then runs normally again (the
    same result as a fresh context from the same W and t)."""
    import paper_1909_02261_amd as pk
    cases = batch_cases(BF16, 4)
    s, _ = make_solver(cases, fused=3)
    W0 = [w.clone() for w in s.W]
    s.set_wait_limit(1)
    with pytest.raises(pk.TcolError) as ei:
        s.step(8)
    assert ei.value.status == EABORT
    s.set_wait_limit(0)
    for g in range(len(cases)):
        s.W[g].copy_(W0[g])
        s.set_t(0, g)
    s.reset()
    done, _ = s.step(6)
    assert done == 6
    got = [host(w) for w in s.W]
    fc_got = [host(s.conflicts(g)[1]) for g in range(len(cases))]
    s.close()
    s2, _ = make_solver(cases, fused=3)
    s2.step(6)
    want = [host(w) for w in s2.W]
    fc_want = [host(s2.conflicts(g)[1]) for g in range(len(cases))]
    s2.close()
    for g in range(len(cases)):
        assert np.array_equal(got[g], want[g])
        assert np.array_equal(fc_got[g], fc_want[g])


def test_batch_launch_cancel_from_host():
    """tcol_cancel from another host thread while a long call runs: the call returns
    TCOL_EABORT well before its iterations would have finished, and the next call runs normally."""
    import paper_1909_02261_amd as pk
    cases = batch_cases(BF16, 16)
    s, _ = make_solver(cases, fused=3)
    s.step(2)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(40)
    per_step = (time.perf_counter() - t0) / 40
    steps = int(4.0 / per_step) + 1          # about four seconds of iterations
    timer = threading.Timer(0.3, s.cancel)
    timer.start()
    t0 = time.perf_counter()
    with pytest.raises(pk.TcolError) as ei:
        s.step(steps)
    elapsed = time.perf_counter() - t0
    timer.join()
    assert ei.value.status == EABORT
    print(f"cancelled after {elapsed:.2f} s of a call of {steps} iterations ({per_step * 1e3:.3f} ms each)")
    assert elapsed < 0.75 * steps * per_step
    s.reset()
    done, _ = s.step(3)
    assert done == 3
    s.close()


def test_batch_launch_falls_back_when_a_graph_takes_sparse_rows():
    """fused = 3 needs the dense penalty pass for every graph: a graph on the sparse rows
    (penalty 2) makes the context run the fast schedule instead."""
    cases = batch_cases(BF16, 3)
    s, _ = make_solver(cases, fused=3, penalty=2)
    assert s.options()["fused"] == 1
    s.set_options(fused=3, penalty=1)
    assert s.options()["fused"] == 3
    s.close()
