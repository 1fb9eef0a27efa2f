"""Autotuner of the factorization parameters for a grid (or a family of grids).

The tuned parameters are the analysis and schedule options of ``chol_options``: the relaxed-amalgamation
thresholds (``zero_abs``, ``zero_rel``, ``max_width``), which trade explicit zeros in the supernodes against the
number of fronts and elimination-tree levels (launches), and ``pair_min`` (rank-128 trailing updates for a lone
wide front).  For every candidate the tuner runs the analysis on the host, builds a representative condensed
matrix on the device from the model's own derivative and assembly calls (objective Hessian at the starting
point, Sigma_x = 1, D = 100: positive definite, the pattern the IPM factors), and times a few factorizations
and solves on the device.  The candidate with the smallest median factor + solve time wins.  Every candidate
yields the same factor up to rounding (the pattern and pivot order are a function of the options, and the
oracle's analysis takes the same options), so tuning changes speed only.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import opf

INT_MAX = 2 ** 31 - 1

# candidate settings: the defaults first (ties keep them)
CANDIDATES = [
    dict(zero_abs=64, zero_rel=0.05, max_width=INT_MAX, pair_min=2048),
    dict(zero_abs=16, zero_rel=0.02, max_width=INT_MAX, pair_min=2048),
    dict(zero_abs=256, zero_rel=0.10, max_width=INT_MAX, pair_min=2048),
    dict(zero_abs=1024, zero_rel=0.20, max_width=INT_MAX, pair_min=2048),
    dict(zero_abs=64, zero_rel=0.05, max_width=256, pair_min=2048),
    dict(zero_abs=64, zero_rel=0.05, max_width=INT_MAX, pair_min=512),
]


def _representative_kkt(model, torch, stream):
    """Device K values of the model's condensed pattern at its starting point (y = 0, Sigma_x = 1, D = 100)."""
    n, m = model.n, model.m
    dev = "cuda"
    x0 = torch.tensor(model.initial_point(), dtype=torch.float64, device=dev)
    y = torch.zeros(m, dtype=torch.float64, device=dev)
    jac = torch.empty(model.nnzj, dtype=torch.float64, device=dev)
    hess = torch.empty(model.nnzh, dtype=torch.float64, device=dev)
    model.eval_derivs(opf.EVAL_JAC | opf.EVAL_HESS, x0, y, 1.0, jac=jac, hess=hess, stream=stream)
    sigx = torch.ones(n, dtype=torch.float64, device=dev)
    dvec = torch.full((m,), 100.0, dtype=torch.float64, device=dev)
    kval = torch.empty(model.nnzk, dtype=torch.float64, device=dev)
    model.condense(hess, jac, sigx, dvec, 0.0, kval, stream=stream)
    return kval


def time_candidate(model, kval, opts, torch, stream, reps=3):
    """(analysis seconds, median factor + solve milliseconds) of one candidate on the device."""
    cp, ri = model.kkt_pattern()
    t0 = time.perf_counter()
    C = opf.Cholesky(model.n, cp, ri, opts)
    t_an = time.perf_counter() - t0
    b = torch.ones(model.n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    assert C.factor(kval, stream=stream) == -1  # first factorization: device buffers, warm-up
    C.solve(b, x, stream=stream)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C.factor(kval, stream=stream)
        C.solve(b, x, stream=stream)
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0))
    C.close()
    return t_an, float(np.median(times))


def tune(models, candidates=None, reps=3, log=None):
    """Best chol_options for a list of models (summed median factor + solve time over the models) and the table
    of every candidate's times."""
    import torch
    candidates = candidates or CANDIDATES
    stream = torch.cuda.current_stream().cuda_stream
    kvals = [_representative_kkt(M, torch, stream) for M in models]
    table = []
    for cand in candidates:
        opts = opf.chol_options(**cand)
        tot_ms, tot_an = 0.0, 0.0
        for M, kv in zip(models, kvals):
            t_an, ms = time_candidate(M, kv, opts, torch, stream, reps)
            tot_ms += ms
            tot_an += t_an
        table.append({"options": dict(cand), "factor_solve_ms": tot_ms, "analysis_s": tot_an})
        if log:
            log(f"[autotune] {cand}: factor+solve {tot_ms:.3f} ms, analysis {tot_an:.2f} s")
    best = min(range(len(table)), key=lambda i: table[i]["factor_solve_ms"])
    return opf.chol_options(**candidates[best]), table[best]["options"], table
