"""Throughput of the TensCol population step on one MI355X.

One step = one iteration of the method (argmax colouring, fitness through A.S,
group concentration and penalty operand, the contraction for the loss
gradient, softmax straight-through update and smoothing) over the whole
population, on synthetic inputs already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5] [--precision fp8]

Prints one JSON line: population-iterations/s (D * steps / s), the roofline of
the dominant kernel (the MFMA contraction), and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

import tcolgen

PEAK = {"fp4": 10.1e15, "fp8": 5.0e15, "bf16": 2.5e15, "fp32": 157.3e12}
GEMM_SRC = os.path.join(ROOT, "paper_1909_02261_amd", "csrc", "tcol_gemm.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_gemm_c5_hbm_traffic.txt")
# penalty product: per-iteration choice (auto; the dense pass below a floor on n), dense MFMA
# pass, sparse rows, per-iteration choice at any size
PENALTY_MODES = {"auto": 0, "dense": 1, "sparse": 2, "auto-any-n": 3}
PENALTY_NAMES = {v: k for k, v in PENALTY_MODES.items()}
# step schedules (tcol_options.fused)
PATHS = {"separate": 0, "fast": 1, "epilogue": 2, "batch": 3}
PATH_NAMES = {v: k for k, v in PATHS.items()}
HBM_PEAK = 8.0e12
PREC = {"fp32": tcolgen.FP32, "bf16": tcolgen.BF16, "fp8": tcolgen.FP8, "fp4": tcolgen.FP4}
PROBLEMS = {"kcol": tcolgen.KCOL, "ecp": tcolgen.ECP, "kpart": tcolgen.KPART, "bkpart": tcolgen.BKPART,
            "mscp": tcolgen.MSCP}
PROBLEM_NAMES = {0: "k-COL", 1: "ECP", 2: "k-partitioning", 3: "balanced k-partitioning", 4: "min-sum colouring"}


def workload(name: str, prec: str):
    p = PREC[prec]
    table = {
        "c1": lambda: tcolgen.case_c1(),
        "c2": lambda: tcolgen.case_c2(p),
        "c3": lambda: tcolgen.case_c3(p),
        "c4": lambda: tcolgen.case_c4(p),
        "c5": lambda: tcolgen.case_c5(p),
    }
    c = table[name]()
    c.precision = p
    c.stop_on_legal = 0
    return c


def gemm_flops(case, t: int):
    """Algorithmic flops of one contraction launch: 2 n^2 D k for A.S plus the same for the
    penalty product when lambda t or mu t is non-zero (real n and k, not padded)."""
    base = 2.0 * case.n * case.n * case.D * case.k
    pen = (case.lam * t != 0.0) or (case.mu * t != 0.0)
    return base, (base if pen else 0.0)


def mixed_peak(prec: str, f_as: float, f_pen: float) -> float:
    """Peak of a launch whose A.S pass runs at the operand dtype and whose penalty pass runs
    in bf16 (fp8 and fp4 precision) or the operand dtype: total flops over the ideal time."""
    p_as = PEAK[prec]
    p_pen = PEAK["bf16"] if prec in ("fp8", "fp4") else PEAK[prec]
    ideal = f_as / p_as + f_pen / p_pen
    return (f_as + f_pen) / ideal


def measured_traffic(config: dict, routes: dict):
    """HBM bytes per contraction launch from the committed counter summary (each launch form
    weighted by the timed iterations' penalty routes), when it was taken on this workload and
    tiling with the current kernel source; else None."""
    import hashlib
    try:
        fields = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                key, val = line.split(":", 1)
                fields[key.strip()] = val.strip()
        sha = hashlib.sha256(open(GEMM_SRC, "rb").read()).hexdigest()
        if fields.get("source_sha256") != sha:
            return None
        for key in ("workload", "tile_bm", "tile_ntw", "penalty", "path", "precision"):
            if fields.get(key) != str(config[key]):
                return None
        n_d = routes["dense"]
        n_s = routes["sparse"] + routes["no_penalty"]
        return (n_d * float(fields["traffic_bytes_dense_launch"]) +
                n_s * float(fields["traffic_bytes_sparse_launch"])) / (n_d + n_s)
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(case, A, W0, budget_s: float):
    import oracle
    p = oracle.Params.from_dict(case.params())
    W = W0.astype(np.float64)
    vel = np.zeros_like(W) if p.momentum else None
    t = 0
    steps = 0
    t0 = time.perf_counter()
    while True:
        r = oracle.iteration(p, t, A, W, want_grads=False, vel=vel)
        W, t = r.W, r.t
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 200:
            break
    return {"value": case.D * steps / el, "unit": "population-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} iterations of the same workload from the same W0 (single-threaded FP64 C "
                      f"oracle, {el:.1f} s)"}


def run_descent(args, torch, pk):
    """Colour-count descent on the planted n = 1000 graph (28 hidden colours, D = 128): k from
    --descent-k-first down while a legal colouring is found within --descent-steps iterations."""
    prec = args.precision or "fp4"
    case = workload("c3", prec)
    print(f"[bench] descent on {case.name} precision {prec}", file=sys.stderr, flush=True)
    A = case.adjacency()
    At = torch.from_numpy(A).cuda()
    prm = pk.Params.from_dict(case.params())
    pk.descent(At, prm, args.descent_k_first, args.descent_k_first, max_steps=5, attempts=1, seed=99)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, col = pk.descent(At, prm, args.descent_k_first, 1, max_steps=args.descent_steps, attempts=1, seed=0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    legal = None
    if col is not None:
        import oracle
        legal = int(oracle.fcolor(A, col.cpu().numpy()[None, :])[0]) == 0
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        p = oracle.Params.from_dict(dict(case.params(), k=args.descent_k_first))
        W = tcolgen.weights0(case.D, case.n, args.descent_k_first, 1000003 * args.descent_k_first)
        t1 = time.perf_counter()
        steps = 0
        t = 0
        while time.perf_counter() - t1 < args.cpu_seconds and steps < 200:
            r = oracle.iteration(p, t, A, W, want_grads=False)
            W, t = r.W, r.t
            steps += 1
        e1 = time.perf_counter() - t1
        cpu = {"value": case.D * steps / e1, "unit": "population-iterations/s", "cores": 1, "kind": "oracle",
               "sample": f"{steps} iterations at k = {args.descent_k_first} from the descent's first weights "
                         f"(single-threaded FP64 C oracle, {e1:.1f} s)"}
    out = {"metric": "population-iterations/s (descent)", "value": case.D * res["steps_total"] / el,
           "unit": "population-iterations/s", "n_gpus": 1, "wall_s": el, "higher_is_better": True,
           "dtype": prec, "data": "synthetic (seeded planted 28-partite graph, n = 1000)",
           "config": {"workload": case.name + "_descent", "k_first": args.descent_k_first,
                      "max_steps": args.descent_steps, "attempts": 1, "D": case.D},
           "result": dict(res, colouring_legal=legal), "cpu_baseline": cpu}
    print(json.dumps(out))


def run_batch(args, torch, pk):
    """The uneven batch: 16 graphs (n from 250 to 2000, p cycling .1/.5/.9, k their greedy
    colour counts, D = 16) stepped by one launch sequence; value = sum_g D_g steps / s.
    One contraction launch covers every graph: its A.S tiles for all of them, and the bf16
    penalty tiles of the graphs whose penalty took the dense route in that iteration."""
    prec = args.precision or "bf16"
    cases = tcolgen.cases_c5b(PREC[prec])
    for c in cases:
        c.stop_on_legal = 0
    G = len(cases)
    print(f"[bench] batch of {G} graphs, precision {prec}: generating inputs", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    graphs = [(torch.from_numpy(c.adjacency()).to(dev), torch.from_numpy(c.weights()).to(dev)) for c in cases]
    s = pk.Solver(graphs, [pk.Params.from_dict(c.params()) for c in cases])
    s.set_options(use_graph=0 if args.no_graph else 1, fused=PATHS[args.path],
                  tile_bm=args.tile_bm, tile_ntw=args.tile_ntw,
                  penalty=PENALTY_MODES[args.penalty])
    opts = s.options()
    s.step(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cnt0 = [s.counters(g) for g in range(G)]
    t_first = s.get_t()
    torch.cuda.synchronize()
    e0.record(stream)
    done, _ = s.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert done == args.steps
    cnt1 = [s.counters(g) for g in range(G)]
    routes = {k: sum(cnt1[g][k] - cnt0[g][k] for g in range(G)) for k in cnt0[0]}
    assert sum(routes.values()) == G * args.steps, routes
    dsum = sum(c.D for c in cases)
    print(f"[bench] timed {args.steps} steps (t = {t_first} .. {t_first + args.steps - 1}): "
          f"{ms / args.steps:.3f} ms/step; graph-iterations by penalty route {routes}", file=sys.stderr, flush=True)

    # the profiled iterations run each graph's own route; the back-to-back contraction
    # launches that give phases_ms['gemm'] repeat the last of them, so the flops of a launch
    # count the penalty tiles of the graphs that took the dense route there
    pc0 = [s.counters(g) for g in range(G)]
    ph = s.profile(args.profile_steps, as_only=True)
    pc1 = [s.counters(g) for g in range(G)]
    print(f"[bench] phases ms {json.dumps({k: round(v, 4) for k, v in ph.items()})}", file=sys.stderr, flush=True)
    f_as = f_pen = 0.0
    dense_graphs = 0
    for g, c in enumerate(cases):
        a, b = gemm_flops(c, 1)
        f_as += a
        frac_dense = (pc1[g]["dense"] - pc0[g]["dense"]) / args.profile_steps
        if opts["penalty"] != 2:
            f_pen += frac_dense * b
        dense_graphs += frac_dense
    achieved = (f_as + f_pen) / (ph["gemm"] / 1e3)
    peak = mixed_peak(prec, f_as, f_pen)
    as_s = ph["gemm_as_only"] / 1e3
    s.close()
    out = {
        "metric": "population-iterations/s (D*steps/s)", "value": dsum * args.steps / (ms / 1e3),
        "unit": "population-iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic (seeded Philox G(n,p) graphs and N(0, 0.01^2) weights)",
        "config": {"workload": "kcol_batch16_gnp_uneven", "graphs": G, "n": [c.n for c in cases],
                   "k": [c.k for c in cases], "D": cases[0].D, "precision": prec, "path": args.path,
                   "hipgraph": not args.no_graph, "tile_bm": opts["tile_bm"], "tile_ntw": opts["tile_ntw"],
                   "penalty": PENALTY_NAMES[opts["penalty"]]},
        "timed_iterations": {"t_first": t_first, "t_last": t_first + args.steps - 1,
                             "graph_iterations_by_penalty_route": routes},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": f"k_gemm over the {G} graphs (A.S pass + fitness gather + G store, and the bf16 "
                               f"penalty pass of the {dense_graphs:g} graphs on the dense route)",
                     "flops_per_launch": f_as + f_pen, "ms_per_launch": ph["gemm"]},
        "roofline_as_only": {"bound": "mfma", "achieved": f_as / as_s / 1e12, "peak": PEAK[prec] / 1e12,
                             "unit": "TFLOP/s", "frac": f_as / as_s / PEAK[prec], "ms_per_launch": ph["gemm_as_only"],
                             "kernel": f"k_gemm A.S pass alone over the {G} graphs (no gather, no store), "
                                       f"back to back"},
        "phases_ms": ph,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c5", choices=["c1", "c2", "c3", "c4", "c5", "c5b"],
                    help="c5b: the batch of 16 uneven graphs in one context")
    ap.add_argument("--precision", default=None, choices=list(PREC))
    ap.add_argument("--path", default="fast", choices=list(PATHS),
                    help="step schedule; batch: one launch per run of iterations over all graphs")
    ap.add_argument("--penalty", default="auto", choices=list(PENALTY_MODES),
                    help="penalty product: per-iteration choice (auto), dense MFMA pass, or sparse rows")
    ap.add_argument("--problem", default=None, choices=list(PROBLEMS),
                    help="run the workload's graph and sizes as another problem (default: its own)")
    ap.add_argument("--momentum", type=float, default=0.0, help="heavy-ball coefficient (0: plain step)")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 schedule's rate")
    ap.add_argument("--plain-steps", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--tile-bm", type=int, default=0)
    ap.add_argument("--tile-ntw", type=int, default=0)
    ap.add_argument("--descent", action="store_true",
                    help="time the colour-count descent driver instead of the step (planted n=1000, 28 colours)")
    ap.add_argument("--descent-k-first", type=int, default=34)
    ap.add_argument("--descent-steps", type=int, default=2000)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the population step runs on a single MI355X "
              "(a population would shard over GPUs by members). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1909_02261_amd as pk

    if args.descent:
        run_descent(args, torch, pk)
        return
    if args.workload == "c5b":
        run_batch(args, torch, pk)
        return

    prec = args.precision or {"c1": "fp32", "c2": "fp32", "c3": "fp4", "c4": "bf16", "c5": "fp4"}[args.workload]
    case = workload(args.workload, prec)
    if args.problem is not None and PROBLEMS[args.problem] != case.problem:
        # same graph and sizes, another problem; the added term (equity or colour cost) takes
        # the ECP's nu of the paper's parameter table
        case.problem = PROBLEMS[args.problem]
        case.nu = 1e-5 if case.problem in (tcolgen.ECP, tcolgen.BKPART, tcolgen.MSCP) else 0.0
        case.name = args.problem + "_" + case.name.split("_", 1)[1]
    if args.momentum:
        case.momentum = args.momentum
        case.name += f"_mom{args.momentum:g}"
    print(f"[bench] workload {case.name} precision {prec}: generating inputs", file=sys.stderr, flush=True)
    A = case.adjacency()
    W0 = case.weights()
    dev = torch.device("cuda:0")
    Wt = torch.from_numpy(W0).to(dev)
    At = torch.from_numpy(A).to(dev)
    s = pk.Solver([(At, Wt)], [pk.Params.from_dict(case.params())])
    s.set_options(use_graph=0 if args.no_graph else 1, fused=PATHS[args.path],
                  tile_bm=args.tile_bm, tile_ntw=args.tile_ntw,
                  penalty=PENALTY_MODES[args.penalty])
    if args.autotune:
        print("[bench] autotuning tile shape / penalty mode", file=sys.stderr, flush=True)
        s.autotune()
    opts = s.options()
    print(f"[bench] options {opts}; warmup {args.warmup}", file=sys.stderr, flush=True)
    s.step(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cnt0 = s.counters()
    t_first = s.get_t()
    torch.cuda.synchronize()
    e0.record(stream)
    done, _ = s.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert done == args.steps
    cnt1 = s.counters()
    routes = {k: cnt1[k] - cnt0[k] for k in cnt0}
    assert sum(routes.values()) == args.steps, routes
    value = case.D * args.steps / (ms / 1e3)
    print(f"[bench] timed {args.steps} steps (t = {t_first} .. {t_first + args.steps - 1}): "
          f"{ms / args.steps:.3f} ms/step; penalty routes {routes}", file=sys.stderr, flush=True)

    # per-kernel durations (HIP events around each launch on the same stream)
    ph = s.profile(args.profile_steps, as_only=True)
    print(f"[bench] phases ms {json.dumps({k: round(v, 4) for k, v in ph.items()})}", file=sys.stderr, flush=True)
    roof, roof_as, f_as, f_pen = contraction_roofline(case, prec, opts, ph, routes)

    parity = None
    if not args.no_cpu_baseline:
        print("[bench] one step of each penalty route against the oracle", file=sys.stderr, flush=True)
        parity = oracle_parity(s, case, A, torch)
    s.close()
    # the same fractions against this device's measured MFMA throughput (register-operand
    # chains on every CU, no memory traffic), beside the published peaks above
    pm_as = max(pk.mfma_peak(PREC[prec]) for _ in range(3)) * 1e12
    pm_pen = max(pk.mfma_peak(tcolgen.BF16) for _ in range(3)) * 1e12 if prec in ("fp8", "fp4") else pm_as
    n_it = args.steps
    n_d = routes["dense"]
    mixed_m = (n_it * f_as + n_d * f_pen) / (n_it * f_as / pm_as + n_d * f_pen / pm_pen)
    measured_peak = {"unit": "TFLOP/s", "operand": pm_as / 1e12, "penalty_operand": pm_pen / 1e12,
                     "k_gemm_step_peak": mixed_m / 1e12, "k_gemm_step_frac": roof["achieved"] * 1e12 / mixed_m,
                     "as_only_frac": roof_as["achieved"] * 1e12 / pm_as, "method": "tcol_mfma_peak"}
    print(f"[bench] measured MFMA peak {json.dumps(measured_peak)}", file=sys.stderr, flush=True)
    if args.calib_copy_mib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters scale the others
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {args.calib_copy_mib} MiB done", file=sys.stderr, flush=True)

    plain = None
    if not args.no_plain and case.momentum == 0.0:
        plain = plain_fp32_rate(case, A, W0, torch, pk, args.plain_steps)
        print(f"[bench] plain FP32 path {json.dumps(plain)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] oracle baseline ({args.cpu_seconds:.0f} s budget)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(case, A, W0, args.cpu_seconds)
        cpu["oracle_parity"] = parity

    config = {"workload": case.name, "problem": PROBLEM_NAMES[case.problem], "n": case.n,
              "k": case.k, "D": case.D, "p": case.p, "precision": prec, "path": args.path,
              "hipgraph": not args.no_graph, "tile_bm": opts["tile_bm"], "tile_ntw": opts["tile_ntw"],
              "penalty": PENALTY_NAMES[opts["penalty"]], "fused": opts["fused"]}
    if case.momentum:
        config["momentum"] = case.momentum
    roof["traffic"] = measured_traffic(config, routes)
    out = {
        "metric": "population-iterations/s (D*steps/s)",
        "value": value,
        "unit": "population-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic (seeded Philox G(n,p) graph and N(0, 0.01^2) weights)",
        "config": config,
        "timed_iterations": {"t_first": t_first, "t_last": t_first + args.steps - 1, "penalty_route": routes},
        "roofline": roof,
        "roofline_as_only": roof_as,
        "mfma_peak_measured": measured_peak,
        "plain_fp32": plain,
        "vs_plain_fp32": (value / plain["value"]) if plain else None,
        "phases_ms": ph,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def contraction_roofline(case, prec, opts, ph, routes):
    """Roofline of k_gemm over the timed step: every iteration runs the A.S pass (with the
    fitness gather and the store of G); the iterations whose penalty product took the dense
    route also run the bf16 penalty pass in the same launch.  achieved = the flops of the
    timed iterations' launches over their time, each launch form timed back to back
    (tcol_profile: 'gemm' with the penalty pass, 'gemm_as_store' without); peak = those
    flops over the time each pass takes at its operand's peak."""
    f_as, f_pen = gemm_flops(case, 1)
    if opts["penalty"] == 2:
        f_pen = 0.0                   # the sparse rows, not the contraction, take the penalty
    n_d, n_o = routes["dense"], routes["sparse"] + routes["no_penalty"]
    if f_pen == 0.0:
        n_o, n_d = n_o + n_d, 0
    t_d, t_o = ph["gemm"] / 1e3, ph["gemm_as_store"] / 1e3
    flops = (n_d + n_o) * f_as + n_d * f_pen
    secs = n_d * t_d + n_o * t_o
    p_as = PEAK[prec]
    p_pen = PEAK["bf16"] if prec in ("fp8", "fp4") else PEAK[prec]
    peak = flops / ((n_d + n_o) * f_as / p_as + n_d * f_pen / p_pen)
    achieved = flops / secs
    launches = {
        "with_penalty_pass": {"count": n_d, "ms": ph["gemm"], "flops": f_as + f_pen,
                              "frac": (f_as + f_pen) / t_d / mixed_peak(prec, f_as, f_pen)},
        "as_pass_and_store": {"count": n_o, "ms": ph["gemm_as_store"], "flops": f_as,
                              "frac": f_as / t_o / p_as},
    }
    roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": None,
            "kernel": "k_gemm over the timed iterations (A.S pass + fitness gather + G store, and the bf16 "
                      "penalty pass in the iterations whose penalty took the dense route)",
            "flops_per_launch": flops / (n_d + n_o), "ms_per_launch": secs * 1e3 / (n_d + n_o),
            "launches": launches}
    as_s = ph["gemm_as_only"] / 1e3
    roof_as = {"bound": "mfma", "achieved": f_as / as_s / 1e12, "peak": p_as / 1e12, "unit": "TFLOP/s",
               "frac": f_as / as_s / p_as, "ms_per_launch": ph["gemm_as_only"],
               "kernel": "k_gemm A.S pass alone (no fitness gather, no store), back to back"}
    return roof, roof_as, f_as, f_pen


def oracle_parity(s, case, A, torch):
    """One step of the timed workload from the solver's current W and t with each penalty
    route forced (1 dense pass, whose operand is bf16 in the low-precision modes; 2 sparse FP32
    rows), against the FP64 oracle's iteration from the same W: the norm-wise error of W'
    (max |diff| / max |ref|) against the oracle's iteration with the penalty operand in the
    precision the route declares (the 1e-5 bar of the tests), and against exact FP64 beside
    the bound that operand's rounding implies (max |diff| <= bound + 1e-5 max |ref|); colours
    and conflict counts after the step exact.  The solver's W, t and options are restored."""
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import orc_params, reference_step
    p = orc_params(case.params())
    keep = s.options()
    W_saved = s.W[0].clone()
    t = s.get_t()
    out = {"t": t}
    for name, pen, route in (("dense_penalty_pass", 1, "dense"), ("sparse_fp32_rows", 2, "sparse")):
        s.set_options(penalty=pen)
        W0 = s.W[0].cpu().numpy()
        ref, W_route, bound = reference_step(p, t, A, W0, route, case.precision)
        done, _ = s.step(1)
        W1 = s.W[0].cpu().numpy().astype(np.float64)
        scale = float(np.abs(ref.W).max())
        c, fc, _ = s.conflicts(0)
        c_ref = oracle.colors(W1)
        out[name] = {"W_err_vs_route_reference": float(np.abs(W1 - W_route).max() / np.abs(W_route).max()),
                     "W_err_vs_fp64": float(np.abs(W1 - ref.W).max() / scale),
                     "fp64_bound_from_operand_rounding": float(bound / scale),
                     "updated": done == 1 and ref.status == 0,
                     "colors_exact": bool(np.array_equal(c.cpu().numpy(), c_ref)),
                     "fcolor_exact": bool(np.array_equal(fc.cpu().numpy(), oracle.fcolor(A, c_ref)))}
        s.W[0].copy_(W_saved)
        s.set_t(t)
    s.set_options(**{k: keep[k] for k in ("penalty",)})
    torch.cuda.synchronize()
    return out


def plain_fp32_rate(case, A, W0, torch, pk, steps):
    """Population-iterations/s of the plain schedule (fused = 0: argmax, class sizes, S, dense
    penalty operand, contraction storing G, fitness, update as separate kernels) with every
    operand in FP32, on the same graph and initial weights, replayed from a hipGraph."""
    import copy
    c = copy.copy(case)
    c.precision = tcolgen.FP32
    dev = torch.device("cuda:0")
    Wt = torch.from_numpy(W0).to(dev)
    sp = pk.Solver([(torch.from_numpy(A).to(dev), Wt)], [pk.Params.from_dict(c.params())])
    sp.set_options(fused=0, use_graph=1)
    sp.step(3)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    done, _ = sp.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    assert done == steps
    ms = e0.elapsed_time(e1)
    sp.close()
    return {"value": case.D * steps / (ms / 1e3), "ms_per_step": ms / steps, "steps": steps,
            "schedule": "plain (fused = 0), FP32 operands, hipGraph replay, same graph and W0"}


if __name__ == "__main__":
    main()
