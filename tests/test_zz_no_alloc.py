"""chol_solve_noalloc (the allocation-free variant of chol_solve) against chol_solve, through the C ABI.

Two calls in a row on one device, the second on a smaller system, so the second call runs on the scratch
contents the first left behind; both results must equal chol_solve's bit for bit (same kernels, same
summation order) and meet the solve residual bound ||Kx - b|| / ||b|| <= 1e-10.
"""
import numpy as np
import pytest

from oracle import chol as ochol
from oracle import kkt as okkt
from tests._grids import config_grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

OPTS = dict(dense_frac=0.5, dense_abs=2 ** 31 - 1, max_width=2 ** 31 - 1, zero_abs=64, zero_rel=0.05)


def opf():
    from paper_2307_16830_amd import opf as _opf
    return _opf


def _system(case, seed):
    """Condensed matrix of a seeded grid (values from the oracle's formula; y = 0 keeps it positive definite)."""
    from oracle.model import Model as OModel
    g = config_grid(case)
    om = OModel(g)
    L = om.L
    x = om.flat_start()
    jr, jc, jv, _ = om.jacobian(x)
    hr, hc, hv, _ = om.hessian(x, np.zeros(L.m), 1.0)
    kr, kc = okkt.kkt_pattern(L.n, jr, jc, hr, hc)
    cp, ri = ochol.lower_csc(L.n, kr, kc)
    rng = np.random.default_rng(seed)
    Jm = okkt.jac_matrix(L.m, L.n, jr, jc, jv)
    vals = okkt.condensed_values(L.n, kr, kc, hr, hc, hv, Jm, rng.uniform(0.1, 10.0, L.n),
                                 10.0 ** rng.uniform(-1, 4, L.m), 0.0)
    return L.n, cp, ri, vals


def _check_case(case, nrhs, seed):
    O = opf()
    n, cp, ri, vals = _system(case, seed)
    C = O.Cholesky(n, cp, ri, O.chol_options(**OPTS))
    kd = torch.tensor(vals, device="cuda")
    assert C.factor(kd) == -1
    rng = np.random.default_rng(seed + 100)
    b = torch.tensor(rng.normal(size=(nrhs, n)), device="cuda")  # row r = right-hand side r (n-contiguous)
    ref = torch.empty_like(b)
    got = torch.full_like(b, float("nan"))
    C.solve(b.view(-1), ref.view(-1)) if nrhs == 1 else _solve_many(C, b, ref, False)
    C.solve_noalloc(b.view(-1), got.view(-1)) if nrhs == 1 else _solve_many(C, b, got, True)
    torch.cuda.synchronize()
    print(f"{case}: n={n} nrhs={nrhs} max |noalloc - solve| = {(got - ref).abs().max().item():.3e}", flush=True)
    assert torch.equal(got, ref)
    K = okkt.sym_from_lower(n, ri, np.repeat(np.arange(n), np.diff(cp)), vals)
    bh, xh = b.cpu().numpy(), got.cpu().numpy()
    for r in range(nrhs):
        assert np.linalg.norm(K @ xh[r] - bh[r]) / np.linalg.norm(bh[r]) <= 1e-10


def _solve_many(C, b, x, noalloc):
    """nrhs right-hand sides in one call (column-major n x nrhs = rows of the (nrhs, n) tensor)."""
    import ctypes
    O = opf()
    fn = O.lib().chol_solve_noalloc if noalloc else O.lib().chol_solve
    rc = fn(C._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), b.shape[0],
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, O.lib().opf_last_error()


def test_noalloc_solve_matches_solve_two_calls():
    # first call: 2,000 buses (a 1,129-column front takes the sync-free wide sweeps), two right-hand sides;
    # second call: the 30-bus grid, smaller than the first, on the scratch the first call left behind
    _check_case("cfg1", 2, seed=3)
    _check_case("cfg0", 1, seed=4)


def test_noalloc_rejects_factor_beyond_scratch():
    """A diagonal matrix of 5,000,000 columns needs 8 bytes per row twice (y and work): 80 MB > 64 MiB."""
    O = opf()
    n = 5_000_000
    cp = np.arange(n + 1, dtype=np.int32)
    ri = np.arange(n, dtype=np.int32)
    C = O.Cholesky(n, cp, ri, O.chol_options(**OPTS))
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    with pytest.raises(O.OpfError) as e:
        C.solve_noalloc(b, x)
    assert e.value.code == O.E_INVALID
    assert "scratch" in str(e.value)
