"""GPU parity of the LU factorization with a fixed pivot sequence (chol_options.ldlt: the symmetric form
P K P^T = L D L^T) against the oracle and closed forms, through the C ABI.

Tolerances, from the Cholesky bounds they follow: for positive definite K the unit factor is L_chol scaled by
its diagonal, so its entries agree to 1e-10 (1 + |l_ij|) and the pivots d_j = L_jj^2 to 2e-10 relative when
the Cholesky factors agree to 1e-10 of their column pivots; the dense indefinite matrices are built as
K = L D L^T from a well-conditioned unit L (off-diagonal entries U(-1, 1) / n), so their computed factors
are L and D to 1e-11 (n eps growth at n = 1,300); solves reach ||Kx - b|| / ||b|| <= 1e-10.
"""
import numpy as np
import pytest

from oracle import chol as ochol
from oracle import ipm as oipm
from oracle.model import Model as OModel
from paper_2307_16830_amd import gridgen
from tests.test_gpu_parity import CASES, OPTS, _block_system, _spd_system, dev, host, opf

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _factor_dict(lp, li, lx):
    n = len(lp) - 1
    out = {}
    for j in range(n):
        for p in range(lp[j], lp[j + 1]):
            out[(int(li[p]), j)] = lx[p]
    return out


@pytest.mark.parametrize("case", CASES)
def test_ldlt_factor_matches_oracle(case):
    M, kval = _spd_system(case)
    cp, ri = M.kkt_pattern()
    C = opf().Cholesky(M.n, cp, ri, opf().chol_options(**OPTS, ldlt=1))
    assert C.factor(kval) == -1
    assert C.inertia() == (M.n, 0)
    gpu = _factor_dict(*C.export_factor())
    sym = ochol.analyze(M.n, cp, ri, ochol.AnalyzeOptions(**OPTS))
    oc = ochol.Cholesky(M.n, cp, ri, sym.perm)
    assert oc.factor(host(kval), ldlt=True) == -1
    ref = _factor_dict(*oc.export())
    assert set(ref) <= set(gpu)
    assert all(gpu[k] == 0.0 for k in gpu if k not in ref)
    diag = [k for k in ref if k[0] == k[1]]
    off = [k for k in ref if k[0] != k[1]]
    d_g = np.array([gpu[k] for k in diag])
    d_o = np.array([ref[k] for k in diag])
    assert np.all(d_o > 0)
    assert np.max(np.abs(d_g - d_o) / d_o) < 2e-10
    l_g = np.array([gpu[k] for k in off])
    l_o = np.array([ref[k] for k in off])
    assert np.max(np.abs(l_g - l_o) / (1.0 + np.abs(l_o))) < 1e-10


def _dense_ldl(n, seed, dvals):
    """K = L D L^T with L unit lower (off-diagonal entries U(-1, 1) / n) and the given pivots: the exact
    L D L^T factors of K are L and D."""
    rng = np.random.default_rng(seed)
    L = np.tril(rng.uniform(-1.0, 1.0, size=(n, n)), -1) / n + np.eye(n)
    K = (L * dvals) @ L.T
    rows, cols = np.tril_indices(n)
    cp, ri = ochol.lower_csc(n, rows, cols)
    return K, L, cp, ri, K[ri, np.repeat(np.arange(n), np.diff(cp))]


@pytest.mark.parametrize("n", [65, 200, 333, 900, 1300])
def test_ldlt_dense_indefinite_front(n):
    """One dense front of n pivots (the blocked path, paired panels from 512 rows below) with pivots of both
    signs: the factor is L and D, the inertia the signs of D (Sylvester), the solve inverts K."""
    rng = np.random.default_rng(10 * n)
    dvals = rng.uniform(1.0, 2.0, n) * np.where(rng.random(n) < 0.4, -1.0, 1.0)
    K, Lx, cp, ri, vals = _dense_ldl(n, n, dvals)
    C = opf().Cholesky(n, cp, ri, opf().chol_options(pair_min=512, ldlt=1))
    assert C.nsuper == 1 and np.array_equal(C.perm(), np.arange(n))
    assert C.factor(dev(vals)) == -1
    assert C.inertia() == (int((dvals > 0).sum()), int((dvals < 0).sum()))
    lp, li, lx = C.export_factor()
    F = np.zeros((n, n))
    for j in range(n):
        F[li[lp[j]:lp[j + 1]], j] = lx[lp[j]:lp[j + 1]]
    assert np.max(np.abs(np.diag(F) - dvals) / np.abs(dvals)) <= 1e-11
    assert np.max(np.abs(np.tril(F, -1) - np.tril(Lx, -1))) <= 1e-11
    b = rng.normal(size=n)
    x = host(C.solve(dev(b)))
    assert np.linalg.norm(K @ x - b) / np.linalg.norm(b) <= 1e-10
    # Cholesky on the same matrix stops at the first negative pivot
    Cc = opf().Cholesky(n, cp, ri, opf().chol_options(pair_min=512))
    assert Cc.factor(dev(vals)) == int(np.argmax(dvals < 0))


@pytest.mark.parametrize("n,j", [(333, 17), (333, 64 * 2 + 17), (900, 64 * 7 + 33)])
def test_ldlt_zero_pivot_in_blocked_front(n, j):
    """A pivot of magnitude 5e-13 K_jj, of either sign, is rejected at tolerance 1e-12 (by the stand-alone
    diagonal kernel for j < 64, inside the trailing update after that); at 3e-12 it is accepted; the oracle
    reports the same column."""
    rng = np.random.default_rng(j)
    for sign in (1.0, -1.0):
        for frac, rejected in [(5e-13, True), (3e-12, False)]:
            dvals = rng.uniform(1.0, 2.0, n)
            dvals[j] = 1.0  # placeholder, set below from K_jj
            K, _, cp, ri, vals = _dense_ldl(n, j, dvals)
            # K_jj = sum_{t<j} L_jt^2 d_t + d_j: choose d_j = sign * frac * K_jj
            s = K[j, j] - dvals[j]
            dvals[j] = sign * frac * s / (1.0 - sign * frac)
            K, _, cp, ri, vals = _dense_ldl(n, j, dvals)
            C = opf().Cholesky(n, cp, ri, opf().chol_options(**OPTS, pivot_tol=1e-12, ldlt=1))
            bad = C.factor(dev(vals))
            oc = ochol.Cholesky(n, cp, ri, np.arange(n, dtype=np.int32))
            obad = oc.factor(vals, piv_tol=1e-12, ldlt=True)
            assert obad == (j if rejected else -1), (sign, frac, obad)
            assert bad == obad, (sign, frac, bad, obad)
            if not rejected:
                assert C.inertia() == (n - (sign < 0), int(sign < 0))


@pytest.mark.parametrize("sizes", [(333, 0, 0), (300, 280, 12), (320, 257, 65), (800, 790, 100)])
def test_ldlt_wide_front_solves_match_oracle(sizes):
    """Fronts with >= 256 pivots take the sync-free sweeps with unit-triangle block inverses, then D; a
    negated clique makes K indefinite."""
    A, cp, ri, vals = _block_system(*sizes, seed=sum(sizes) + 1)
    n = A.shape[0]
    a = sizes[0]
    # A is strictly diagonally dominant; negating the first clique's diagonal keeps it so, hence K has a
    # negative eigenvalues and nonsingular leading minors
    A[np.arange(a), np.arange(a)] *= -1.0
    colidx = np.repeat(np.arange(n), np.diff(cp))
    vals = A[ri, colidx]
    o = dict(OPTS, dense_frac=1.0)
    C = opf().Cholesky(n, cp, ri, opf().chol_options(**o, pair_min=0, ldlt=1))
    assert np.diff(C.supernodes()).max() >= 256
    sym = ochol.analyze(n, cp, ri, ochol.AnalyzeOptions(**o))
    oc = ochol.Cholesky(n, cp, ri, sym.perm)
    assert oc.factor(vals, ldlt=True) == -1
    assert C.factor(dev(vals)) == -1
    assert C.inertia() == oc.inertia()
    ev = np.linalg.eigvalsh(A)
    assert C.inertia() == (int((ev > 0).sum()), int((ev < 0).sum()))
    rng = np.random.default_rng(3)
    for rep in range(2):
        b = rng.normal(size=n)
        x = host(C.solve(dev(b)))
        xo = oc.solve(b)
        assert np.max(np.abs(x - xo)) <= 1e-11 * np.max(np.abs(xo)), rep
        assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-10


@pytest.mark.parametrize("seed", [1, 2, 5])
def test_ipm_with_ldlt_matches_oracle(seed):
    """Algorithm 1 with the inertia read from D (accepted when every pivot is positive) takes the oracle's
    Cholesky decisions: same status, iterations within +-2, objective to 1e-6."""
    g = gridgen.make_grid(30, 41, 6, seed)
    O = opf()
    ipm = O.IPM(O.Model(g), tol=1e-8, chol_opts=O.chol_options(ldlt=1))
    rc, iters, obj = ipm.solve()
    I = oipm.IPM(OModel(g), oipm.Options(tol=1e-8))
    assert I.solve() == oipm.Status.OK
    ref = I.model.objective(I.x)
    assert rc == O.OK, O.status_name(rc)
    assert abs(iters - I.iter) <= 2
    assert abs(obj - ref) <= 1e-6 * abs(ref)


def test_ipm_with_ldlt_cfg1_matches_cholesky_path():
    """2,000 buses (blocked fronts, wide-front sweeps): the LDL^T and Cholesky paths reach the same solution."""
    from tests._grids import config_grid
    g = config_grid("cfg1")
    O = opf()
    r1 = O.IPM(O.Model(g), tol=1e-4).solve()
    r2 = O.IPM(O.Model(g), tol=1e-4, chol_opts=O.chol_options(ldlt=1)).solve()
    assert r1[0] == r2[0] == O.OK
    assert abs(r1[1] - r2[1]) <= 2
    assert abs(r1[2] - r2[2]) <= 1e-6 * abs(r1[2])


def test_ldlt_rejects_the_tile_path():
    n = 4
    cp, ri = ochol.lower_csc(n, np.arange(n), np.arange(n))
    with pytest.raises(opf().OpfError):
        opf().Cholesky(n, cp, ri, opf().chol_options(ldlt=1, tile_min=64))
