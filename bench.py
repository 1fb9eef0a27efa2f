"""Benchmark: condensed-space IPM iterations per second on the 10,000-bus synthetic grid, one MI355X.

One step = one IPM iteration (Algorithm 1): derivative evaluation over the
templates, condensed assembly, supernodal Cholesky with inertia correction,
triangular solves with iterative refinement on the full system, filter line
search and the update -- every vector operation on the GPU.  The symbolic
analysis (once per topology) is outside the timed region and reported apart.

Prints one JSON line (see the contract in the design notes).
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (vector and MFMA)
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pmc_summary_path(config, kernel):
    return os.path.join(HERE, "profiles", f"{kernel.split()[0]}_{config}_pmc.md")


def factor_kernels_hash():
    """Hash of the source of the factorization kernels (diagonal block, panel solve, trailing update, dense-front
    tile launch): hardware-counter traffic recorded for them holds only while this is unchanged."""
    import hashlib
    src = open(os.path.join(HERE, "paper_2307_16830_amd", "csrc", "chol.hip")).read()
    a = src.index("constexpr int PW = ")
    b = src.index("// ---------------------------------------------------------------- solves")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def recorded_traffic(config, kernel):
    """HBM bytes per launch of the roofline kernel on this configuration, from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs, scaled by a reference copy), or None when no summary exists for the
    kernel and configuration or the kernels changed since the counters were taken."""
    try:
        text = open(pmc_summary_path(config, kernel)).read()
    except OSError:
        return None
    h = re.search(r"kernel-source-hash: ([0-9a-f]+)", text)
    t = re.search(r"traffic-bytes-per-launch: ([0-9.e+]+)", text)
    c = re.search(r"config: (\w+)", text)
    if not h or not t or not c or c.group(1) != config or h.group(1) != factor_kernels_hash():
        return None
    return float(t.group(1))


def _trace_grid(req):
    from paper_2307_16830_amd import gridgen
    seed, nb, ne, ng, lf = req
    return seed, gridgen.make_grid(nb, ne, ng, seed, load_factor=lf)


def serving_grids(nreq):
    """The first ``nreq`` requests of the serving trace (log-uniform 30..2,000 buses), generated on host
    processes; called before the GPU is touched."""
    import multiprocessing as mp
    from paper_2307_16830_amd import gridgen
    trace = gridgen.serving_trace(512)[:nreq]
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        return pool.map(_trace_grid, trace)


def pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def tune_serving(grids, nsample=6):
    """Autotuned factorization options for the serving trace: candidates timed on a sample of its requests
    spread over the size range (see paper_2307_16830_amd.autotune)."""
    from paper_2307_16830_amd import autotune, opf
    order = sorted(range(len(grids)), key=lambda k: grids[k][1].nbus)
    pick = [order[int(round(q * (len(order) - 1) / max(nsample - 1, 1)))] for q in range(nsample)]
    models = [opf.Model(grids[k][1]) for k in pick]
    best, best_dict, table = autotune.tune(models, log=log)
    return best, {"chosen": best_dict, "sample_buses": [int(grids[k][1].nbus) for k in pick],
                  "candidates": table}


def serving_bench(grids, slots, rate_factor):
    """Continuous-batching server vs one-at-a-time solves on the same GPU and the same requests.

    The one-at-a-time path creates, analyzes and solves each request alone on one stream; its service times
    give the sequential rate.  Arrivals are Poisson at ``rate_factor`` times that rate (SplitMix64 draws);
    the server gets each request at its arrival time, and the sequential path's latencies on the same
    arrivals follow from its service times (first come, first served)."""
    import torch
    from paper_2307_16830_amd import gridgen, opf

    copts, tuning = tune_serving(grids)

    def alone(g):
        M = opf.Model(g)
        ipm = opf.IPM(M, tol=1e-4, max_iter=500, chol_opts=copts)
        rc, it, obj = ipm.solve()
        torch.cuda.synchronize()
        return rc

    alone(grids[0][1])  # warm-up (first launches of every kernel)
    service, conv_seq = [], 0
    for tag, g in grids:
        t0 = time.perf_counter()
        conv_seq += alone(g) == opf.OK
        service.append(time.perf_counter() - t0)
    seq_rate = len(grids) / sum(service)
    u = gridgen.SplitMix64(4).uniform(len(grids))
    arrive = np.cumsum(-np.log1p(-u) / (rate_factor * seq_rate))
    lat_seq, t_free = [], 0.0
    for a, sv in zip(arrive, service):
        t_free = max(a, t_free) + sv
        lat_seq.append(t_free - a)
    def serve(at):
        srv = opf.Server(slots=slots, hbm_budget=8 << 30, chol_opts=copts)
        t0 = srv.now()
        for k, (tag, g) in enumerate(grids):
            while srv.now() - t0 < at[k]:
                time.sleep(2e-4)
            srv.submit(g, tag)
        res = {}
        while len(res) < len(grids):
            got = srv.poll(wait=True)
            if not got:
                raise RuntimeError("server went idle with results missing")
            for r in got:
                res[r["tag"]] = r
        st = srv.stats()
        srv.close()
        return res, st, max(r["t_done"] for r in res.values()) - t0

    g0 = opf.graph_stats()
    res_all, _, span_all = serve(np.zeros(len(grids)))  # every request at once: the server's capacity
    res, st, makespan = serve(arrive)
    g1 = opf.graph_stats()
    lat = [r["t_done"] - r["t_submit"] for r in res.values()]
    return {
        "requests": len(grids), "slots": slots,
        "workload": "serving trace: seeded grids, buses log-uniform on [30, 2000], loads x U(0.9, 1.1), tol 1e-4",
        "arrivals": f"Poisson at {rate_factor}x the sequential solve rate",
        "solves_per_s": len(grids) / makespan, "p50_ms": 1e3 * pct(lat, 50), "p99_ms": 1e3 * pct(lat, 99),
        "solves_per_s_all_at_once": len(grids) / span_all,
        "converged": sum(r["status"] == 1 for r in res.values()),
        "not_converged": sorted({(opf.status_name(r["status"]), r["message"][:120]) for r in res.values()
                                 if r["status"] != 1}),
        "peak_pool_bytes": st["peak_in_use"],
        "graph_captures": g1[0] - g0[0], "graph_capture_fallbacks": g1[1] - g0[1],
        "sequential": {"solves_per_s": seq_rate, "p50_ms": 1e3 * pct(lat_seq, 50), "p99_ms": 1e3 * pct(lat_seq, 99),
                       "converged": conv_seq},
        "autotune": tuning,
    }


def stage_probe(grid, reps=20, warm=5, flush_mib=1024):
    """The AD (every template: constraints, gradient, the x-dependent Jacobian entries and the Hessian, as the
    IPM evaluates them) and condensed-assembly kernels alone on one grid, each timed with HIP events cold (after
    writing a buffer larger than the last-level cache) and warm (back to back), median and p90 over `reps`
    runs after `warm` untimed ones, and their algorithmic HBM rates (values only, index maps excluded)."""
    import torch
    from paper_2307_16830_amd import opf
    M = opf.Model(grid)
    n, m = M.n, M.m
    dev = "cuda"
    x = torch.tensor(M.initial_point(), dtype=torch.float64, device=dev)
    y = torch.linspace(-1.0, 1.0, m, dtype=torch.float64, device=dev)
    f = torch.empty(1, dtype=torch.float64, device=dev)
    c = torch.empty(m, dtype=torch.float64, device=dev)
    g = torch.empty(n, dtype=torch.float64, device=dev)
    jac = torch.empty(M.nnzj, dtype=torch.float64, device=dev)
    hess = torch.empty(M.nnzh, dtype=torch.float64, device=dev)
    sigx = torch.ones(n, dtype=torch.float64, device=dev)
    dvec = torch.full((m,), 100.0, dtype=torch.float64, device=dev)
    kval = torch.empty(M.nnzk, dtype=torch.float64, device=dev)
    flush = torch.empty(flush_mib << 17, dtype=torch.float64, device=dev)
    what = opf.EVAL_C | opf.EVAL_GRAD | opf.EVAL_JAC | opf.EVAL_HESS
    M.eval_derivs(what, x, y, 1.0, c=c, grad=g, jac=jac, hess=hess)  # writes the constant Jacobian entries once
    ad = lambda: M.eval_derivs(what | opf.EVAL_JAC_VAR, x, y, 1.0, c=c, grad=g, jac=jac, hess=hess)
    asm = lambda: M.condense(hess, jac, sigx, dvec, 0.0, kval)
    ad()
    asm()
    N, E, G = grid.nbus, grid.nbranch, grid.ngen
    nconst = 10 * E + 2 * G + 1
    # AD: x and y in, template parameters in (per branch g, b, b/2 and two bus indices;
    # per bus pd, qd, gs, bs; per generator c2, c1 and its bus), c, gradient, the x-dependent Jacobian entries
    # and the Hessian out
    ad_bytes = 8.0 * (n + m) + 32.0 * E + 32.0 * N + 20.0 * G + 8.0 * (m + n + (M.nnzj - nconst) + M.nnzh)
    asm_bytes = 8.0 * (M.nnzh + M.nnzj + m + n + M.nnzk)
    out = {}
    for name, fn, nbytes in (("ad", ad, ad_bytes), ("assembly", asm, asm_bytes)):
        res = {}
        for mode in ("cold", "warm"):
            ts = []
            for _ in range(warm):
                fn()
            for _ in range(reps):
                if mode == "cold":
                    flush.fill_(1.0)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts))
            res[mode] = {"ms": ms, "p90_ms": pct(ts, 90), "gbs": nbytes / (ms * 1e-3) / 1e9,
                         "frac_hbm": nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
        res["algorithmic_bytes"] = nbytes
        out[name] = res
    del flush
    return out


def cpu_baseline(grid, budget_s):
    """The oracle (plain CPU reference) timed on one IPM iteration of the same grid, analysis excluded."""
    from oracle import ipm as oipm
    from oracle.model import Model as OModel
    cores = 1
    t0 = time.perf_counter()
    I = oipm.IPM(OModel(grid), oipm.Options(tol=1e-4))
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    I.step()
    t_step = time.perf_counter() - t0
    return {"value": 1.0 / t_step, "unit": "iter/s", "cores": cores, "kind": "oracle",
            "sample": f"one oracle IPM iteration (single thread) on the same grid; oracle setup and "
                      f"symbolic analysis excluded ({t_setup:.1f} s); iteration took {t_step:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="cfg2")
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graphs", action="store_true", help="plain kernel launches instead of graph replay")
    ap.add_argument("--chol-options", default=None, metavar="JSON",
                    help="factorization options for the IPM (chol_options fields, e.g. '{\"pair_min\": 1024}')")
    ap.add_argument("--stage-probe", default=None, metavar="CONFIG",
                    help="also time the AD and assembly kernels alone, cold and warm, on this configuration")
    ap.add_argument("--serving", type=int, default=512, metavar="REQUESTS",
                    help="also run this many requests of the serving trace through the batched server and one at "
                         "a time (0: skip)")
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--serving-rate", type=float, default=1.5)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of this many MiB (a reference kernel of known "
                         "traffic for hardware-counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)

    sgrids = serving_grids(args.serving) if args.serving > 0 else None  # host work, before the GPU is touched
    import torch
    from paper_2307_16830_amd import gridgen, opf

    if args.copy_calibration > 0:
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {nb} bytes read, {nb} bytes written")
        del src, dst
    N, E, G = gridgen.CONFIGS[args.config]
    log(f"[bench] generating {args.config}: {N} buses, {E} branches, {G} generators")
    grid = gridgen.make_config(args.config)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # the IPM runs on a stream of its own (default priority), so that its factorization and solve launch
    # sequences are captured into HIP graphs and replayed (ipm_options.graphs)
    stream = torch.cuda.Stream()
    M = opf.Model(grid, stream=stream.cuda_stream)
    t0 = time.perf_counter()
    # at 80k buses exact minimum degree stops once the minimum degree reaches 1,500 (the rest, ~42.6k columns,
    # is ordered by index into one dense front); below that the relative dense-tail rule alone applies
    ckw = dict(dense_abs=1500) if args.config == "cfg3" else {}
    if args.chol_options:
        ckw.update(json.loads(args.chol_options))
    copts = opf.chol_options(**ckw) if ckw else None
    ipm = opf.IPM(M, tol=args.tol, max_iter=10000, chol_opts=copts, stream=stream.cuda_stream,
                  graphs=0 if args.no_graphs else 1)
    torch.cuda.synchronize()
    t_analyze = time.perf_counter() - t0
    C = ipm.chol()
    log(f"[bench] n={M.n} m={M.m} nnzK={M.nnzk} nnzL={C.nnz_l} flops/factor={C.flops:.3e} "
        f"supernodes={C.nsuper} setup+analysis={t_analyze:.2f}s")
    infos = []

    def run(k):
        for _ in range(k):
            rc, info = ipm.step()
            if rc != 0:
                raise RuntimeError(f"IPM stopped with status {opf.status_name(rc)} at iteration {info['iter']}")
            infos.append(info)

    run(args.warmup)
    torch.cuda.synchronize()
    # timed region: exactly K IPM iterations, no per-launch instrumentation (graph replay stays on)
    C.timing(False)
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timed = infos[args.warmup:args.warmup + args.steps]
    kt_dense = {"launches": 0, "ms": 0.0, "flops": 0.0}
    if copts is not None and getattr(copts, "tile_min", 0) > 0:
        C.timing(["dense_front"])
        run(args.steps)
        torch.cuda.synchronize()
        kt_dense = C.timing_read()["dense_front"]
    # kernel-timing pass right after the timed region (same grid and factorization schedule, the next K
    # iterations, plain launches): events around every launch of the blocked path's trailing update
    C.timing(["trailing_update"])
    run(args.steps)
    torch.cuda.synchronize()
    kt_tu = C.timing_read()["trailing_update"]
    # diagnostic: every factorization kernel category over two more iterations
    C.timing(True)
    run(2)
    torch.cuda.synchronize()
    kt_all = C.timing_read()
    C.timing(False)
    ms = 1e3 * elapsed / args.steps
    fac_ms = np.mean([i["t_factor"] / max(i["factorizations"], 1) for i in timed])
    stage = {k: float(np.mean([i[k] for i in timed])) for k in ("t_ad", "t_assembly", "t_factor", "t_solve")}
    stage["t_rest"] = ms - sum(stage.values())
    log(f"[bench] {args.steps} iterations in {elapsed:.3f}s = {ms:.2f} ms/iter; stages (ms) {stage}; "
        f"refinement steps/iter {np.mean([i['ir_steps'] for i in timed]):.2f}, "
        f"factorizations/iter {np.mean([i['factorizations'] for i in timed]):.2f}")
    factor_tflops = C.flops / (fac_ms * 1e-3) / 1e12
    if kt_dense["launches"] > 0:
        kname = "dense_front (dependency-driven tile factorization of the dense fronts, FP64 MFMA)"
        kt, where = kt_dense, "HIP events around each launch in a pass of K iterations right after the timed region"
    else:
        kname = "blk_syrk (FP64 MFMA trailing update of the supernodal fronts)"
        kt, where = kt_tu, "HIP events around each launch in a pass of K iterations right after the timed region"
    avg_ms = kt["ms"] / max(kt["launches"], 1)
    flops_per_launch = kt["flops"] / max(kt["launches"], 1)
    # the supernodal Schur-complement update is a dense contraction: its bound is the FP64 MFMA rate and its
    # algorithmic work the factorization flops of the fronts the launch covers
    achieved_tflops = flops_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    tu_avg = kt_tu["ms"] / max(kt_tu["launches"], 1)
    log(f"[bench] factorization kernels per iteration (diagnostic pass): " +
        ", ".join(f"{k} {v['ms'] / 2:.2f} ms/{v['launches'] // 2} launches" for k, v in kt_all.items()))
    # algorithmic HBM bytes of the AD and assembly stages per iteration, values only (each evaluation's inputs
    # and outputs; template parameters and index maps excluded): Hessian (x, y in; H out), the new point (x in;
    # c, J, gradient out) and every line-search trial (x in; c out)
    trials = float(np.mean([i["ls_trials"] for i in timed]))
    # (the point evaluation rewrites only the x-dependent Jacobian entries: 10 E + 2 G + 1 are constant)
    nconst = 10 * E + 2 * G + 1
    ad_bytes = (8.0 * (M.n + M.m + M.nnzh) + 8.0 * (M.n + M.m + M.nnzj - nconst + M.n)
                + trials * 8.0 * (M.n + M.m))
    asm_bytes = 8.0 * (M.nnzh + M.nnzj + M.m + M.n + M.nnzk)
    out = {
        "metric": "ACOPF IPM iter/s at 10k buses",
        "value": args.steps / elapsed,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: synthetic polar ACOPF, {N} buses, {E} branches, {G} generators, "
                               f"n={M.n}, m={M.m}, tol={args.tol}",
                   "global_batch": 1, "parallelism": "single GPU"},
        "stages_ms": stage,
        "stage_gbs": {"ad": ad_bytes / (stage["t_ad"] * 1e-3) / 1e9 if stage["t_ad"] > 0 else None,
                      "assembly": asm_bytes / (stage["t_assembly"] * 1e-3) / 1e9 if stage["t_assembly"] > 0 else None,
                      "note": "algorithmic bytes (values only) over stage time from HIP events per iteration; "
                              "AD = Hessian + constraint/Jacobian/gradient evaluations of the iteration"},
        "analysis_s": t_analyze,
        "chol_options": ckw or "defaults",
        "roofline": {"bound": "mfma", "achieved": achieved_tflops, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / PEAK_FP64_TFLOPS, "traffic": recorded_traffic(args.config, kname),
                     "kernel": kname, "avg_launch_ms": avg_ms, "launches": kt["launches"],
                     "flops_per_launch": flops_per_launch,
                     "algorithmic_bytes_per_launch": kt["bytes"] / max(kt["launches"], 1), "timing": where,
                     "trailing_update": {"launches": kt_tu["launches"], "avg_launch_ms": tu_avg,
                                         "tflops": (kt_tu["flops"] / max(kt_tu["launches"], 1)) / (tu_avg * 1e-3)
                                         / 1e12 if tu_avg > 0 else None}},
        "factorization_tflops": factor_tflops,
        "factor_kernels_ms_per_iter": {k: v["ms"] / 2 for k, v in kt_all.items()},
    }
    del ipm, C, M
    if sgrids:
        log(f"[bench] serving: {len(sgrids)} requests, {args.serving_slots} slots")
        out["serving"] = serving_bench(sgrids, args.serving_slots, args.serving_rate)
        log(f"[bench] serving: {out['serving']}")
    if args.stage_probe:
        log(f"[bench] stage probe on {args.stage_probe}")
        out["stage_probe"] = {"config": args.stage_probe,
                              **stage_probe(gridgen.make_config(args.stage_probe))}
        log(f"[bench] stage probe: {out['stage_probe']}")
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on one iteration of the same grid")
        out["cpu_baseline"] = cpu_baseline(grid, 30.0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
