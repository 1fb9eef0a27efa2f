"""Autotuner of the factorization options: it times every candidate on the device, returns the fastest, and
the returned options analyze bit-exactly like the oracle and factor to a valid solve."""
import numpy as np
import pytest

from oracle import chol as ochol
from oracle import kkt as okkt
from paper_2307_16830_amd import gridgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_autotune_picks_a_timed_candidate_that_stays_exact():
    from paper_2307_16830_amd import autotune, opf
    grids = [gridgen.make_grid(30, 41, 6, 1), gridgen.make_grid(300, 405, 60, 3)]
    models = [opf.Model(g) for g in grids]
    best, best_dict, table = autotune.tune(models, reps=2)
    assert len(table) == len(autotune.CANDIDATES)
    assert all(r["factor_solve_ms"] > 0 for r in table)
    assert best_dict in autotune.CANDIDATES
    assert min(r["factor_solve_ms"] for r in table) == next(r for r in table if r["options"] == best_dict)[
        "factor_solve_ms"]
    for M in models:
        cp, ri = M.kkt_pattern()
        C = opf.Cholesky(M.n, cp, ri, best)
        an = {k: best_dict[k] for k in ("zero_abs", "zero_rel", "max_width")}
        sym = ochol.analyze(M.n, cp, ri, ochol.AnalyzeOptions(dense_frac=0.5, dense_abs=2 ** 31 - 1, **an))
        assert np.array_equal(C.perm(), sym.perm) and np.array_equal(C.supernodes(), sym.snode_ptr)
        # a positive definite matrix of the pattern: diagonally dominant values
        colidx = np.repeat(np.arange(M.n), np.diff(cp))
        vals = np.where(ri == colidx, 10.0 + np.bincount(colidx, minlength=M.n)[colidx], -0.5)
        K = okkt.sym_from_lower(M.n, ri, colidx, vals)
        vals = np.where(ri == colidx, np.asarray(np.abs(K).sum(axis=1)).ravel()[colidx] + 1.0, -0.5)
        K = okkt.sym_from_lower(M.n, ri, colidx, vals)
        assert C.factor(torch.tensor(vals, device="cuda")) == -1
        b = np.random.default_rng(0).normal(size=M.n)
        x = C.solve(torch.tensor(b, device="cuda")).cpu().numpy()
        assert np.linalg.norm(K @ x - b) <= 1e-10 * np.linalg.norm(b)
