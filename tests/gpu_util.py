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
