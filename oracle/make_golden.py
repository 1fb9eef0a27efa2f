"""Write stored expected IPM results computed by the oracle alone.

TEST INFRASTRUCTURE ONLY.  Runs the oracle's Algorithm 1 on one seeded
synthetic grid (inputs from the shared instance generator) and writes the
status, iteration count, final objective and final scaled optimality error
to ``tests/golden/ipm_<config>.json``.  The 10,000-bus solve takes tens of
minutes single-threaded, which is why its result is stored rather than
recomputed by the tests.

    python oracle/make_golden.py cfg2 [--tol 1e-4]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import ipm as oipm  # noqa: E402
from oracle.model import Model  # noqa: E402
from paper_2307_16830_amd import gridgen  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config")
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    grid = gridgen.make_config(a.config)
    t0 = time.perf_counter()
    I = oipm.IPM(Model(grid), oipm.Options(tol=a.tol))
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    st = I.solve(verbose=True)
    t_solve = time.perf_counter() - t0
    N, E, G = gridgen.CONFIGS[a.config]
    rec = {
        "config": a.config, "nbus": N, "nbranch": E, "ngen": G, "tol": a.tol,
        "status": int(st), "iterations": int(I.iter), "objective": float(I.model.objective(I.x)),
        "e0": float(I.log[-1]["E0"]) if I.log else None,
        "trajectory": [{"iter": int(r["iter"]), "obj": float(r["obj"]), "E0": float(r["E0"]), "mu": float(r["mu"]),
                        "dw": (None if r.get("dw") is None else float(r["dw"]))} for r in I.log],
        "source": "oracle/make_golden.py (oracle IPM only)",
        "oracle_seconds": {"setup": round(t_setup, 1), "solve": round(t_solve, 1)},
        "host": platform.processor() or platform.machine(),
    }
    out = a.out or os.path.join(ROOT, "tests", "golden", f"ipm_{a.config}.json")
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(f"wrote {out}: status {st}, {I.iter} iterations, objective {rec['objective']:.10g}", flush=True)


if __name__ == "__main__":
    main()
