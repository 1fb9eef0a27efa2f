"""Pins of the oracle's LU factorization with a fixed pivot sequence (symmetric form L D L^T) against dense
linear algebra: Doolittle's LU without pivoting written out, numpy's Cholesky for positive definite K,
eigenvalue signs (Sylvester's law of inertia) for indefinite K, and the relative pivot threshold."""
import numpy as np
import pytest

from oracle import chol as ochol
from tests.test_oracle_chol import _threshold_matrix, random_pattern


def _values(n, cp, ri, rng, shift):
    """Symmetric values on the pattern: off-diagonals N(0, 1), diagonal = row abs-sum * shift (shift > 1:
    positive definite; a mix of signs: indefinite)."""
    vals = rng.normal(size=len(ri))
    cols = np.repeat(np.arange(n), np.diff(cp))
    K = np.zeros((n, n))
    K[ri, cols] = vals
    K = K + np.tril(K, -1).T
    for j in range(n):
        K[j, j] = (np.sum(np.abs(K[j])) - abs(K[j, j]) + 1.0) * shift[j]
    diag = ri == cols
    vals[diag] = K[ri[diag], cols[diag]]
    return vals, K


def _dense_factor(ch, n):
    lp, li, lx = ch.export()
    F = np.zeros((n, n))
    for j in range(n):
        F[li[lp[j]:lp[j + 1]], j] = lx[lp[j]:lp[j + 1]]
    d = np.diag(F).copy()
    L = np.tril(F, -1) + np.eye(n)
    return L, d


def doolittle(A):
    """LU without pivoting by its definition, entry by entry (pure Python loops)."""
    n = A.shape[0]
    L = np.eye(n)
    U = np.zeros((n, n))
    for k in range(n):
        for j in range(k, n):
            U[k, j] = A[k, j] - sum(L[k, t] * U[t, j] for t in range(k))
        for i in range(k + 1, n):
            L[i, k] = (A[i, k] - sum(L[i, t] * U[t, k] for t in range(k))) / U[k, k]
    return L, U


@pytest.mark.parametrize("seed", range(3))
def test_ldlt_is_the_lu_without_pivoting(seed):
    rng = np.random.default_rng(700 + seed)
    n = 9
    (cp, ri), _ = random_pattern(n, 0.35, rng)
    shift = np.where(rng.random(n) < 0.4, -1.0, 1.0)
    vals, K = _values(n, cp, ri, rng, shift)
    sym = ochol.analyze(n, cp, ri)
    ch = ochol.Cholesky(n, cp, ri, sym.perm)
    assert ch.factor(vals, ldlt=True) == -1
    L, d = _dense_factor(ch, n)
    P = K[np.ix_(sym.perm, sym.perm)]
    Lu, U = doolittle(P)
    scale = np.max(np.abs(U))
    assert np.allclose(L, Lu, rtol=1e-10, atol=1e-10)
    assert np.allclose(np.diag(U), d, rtol=1e-10, atol=1e-12 * scale)
    assert np.allclose(U, np.diag(d) @ L.T, rtol=1e-10, atol=1e-12 * scale)


@pytest.mark.parametrize("seed", range(3))
def test_ldlt_of_positive_definite_matches_cholesky(seed):
    """For positive definite K: L = L_chol diag(L_chol)^{-1} and D = diag(L_chol)^2."""
    rng = np.random.default_rng(800 + seed)
    n = int(rng.integers(20, 60))
    (cp, ri), _ = random_pattern(n, 0.1, rng)
    vals, K = _values(n, cp, ri, rng, np.ones(n))
    sym = ochol.analyze(n, cp, ri)
    ch = ochol.Cholesky(n, cp, ri, sym.perm)
    assert ch.factor(vals, ldlt=True) == -1
    L, d = _dense_factor(ch, n)
    Lc = np.linalg.cholesky(K[np.ix_(sym.perm, sym.perm)])
    assert np.allclose(L, Lc / np.diag(Lc), rtol=1e-12, atol=1e-12)
    assert np.allclose(d, np.diag(Lc) ** 2, rtol=1e-12)
    assert ch.inertia() == (n, 0)


@pytest.mark.parametrize("seed", range(4))
def test_ldlt_inertia_and_solve_on_indefinite_matrices(seed):
    """Sylvester's law of inertia: the signs of D are the signs of K's eigenvalues; the solve inverts K."""
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(20, 60))
    (cp, ri), _ = random_pattern(n, 0.1, rng)
    shift = np.where(rng.random(n) < 0.3, -1.0, 1.0)
    vals, K = _values(n, cp, ri, rng, shift)
    sym = ochol.analyze(n, cp, ri)
    ch = ochol.Cholesky(n, cp, ri, sym.perm)
    assert ch.factor(vals) >= 0  # not positive definite: Cholesky stops
    assert ch.factor(vals, ldlt=True) == -1
    ev = np.linalg.eigvalsh(K)
    assert ch.inertia() == (int((ev > 0).sum()), int((ev < 0).sum()))
    assert ch.inertia()[1] > 0
    L, d = _dense_factor(ch, n)
    P = K[np.ix_(sym.perm, sym.perm)]
    assert np.allclose(L @ np.diag(d) @ L.T, P, rtol=1e-10, atol=1e-10 * np.max(np.abs(P)))
    b = rng.normal(size=n)
    x = ch.solve(b)
    assert np.allclose(K @ x, b, rtol=1e-9, atol=1e-9 * np.max(np.abs(b)))


@pytest.mark.parametrize("frac,tol,rejected", [
    (5e-13, 1e-12, True),
    (5e-13, 0.0, False),
    (-5e-13, 1e-12, True),   # a tiny negative pivot is rejected too: |d| is compared
    (-5e-13, 0.0, False),    # ... and accepted without a tolerance (nonzero)
    (-3e-12, 1e-12, False),  # negative but above the tolerance in magnitude: accepted
])
def test_ldlt_pivot_threshold_is_on_the_magnitude(frac, tol, rejected):
    n, cp, ri, vals, dense = _threshold_matrix(frac)
    sym = ochol.analyze(n, cp, ri)
    ch = ochol.Cholesky(n, cp, ri, sym.perm)
    bad = ch.factor(vals, piv_tol=tol, ldlt=True)
    if rejected:
        assert bad == 2 and sym.perm[bad] == 1
    else:
        assert bad == -1
        _, d = _dense_factor(ch, n)
        assert d[2] == pytest.approx(frac * 1e12, rel=1e-3)


def test_ldlt_zero_pivot_is_rejected():
    """[[0, 1], [1, 0]] is nonsingular but its first leading minor is 0: no LU without pivoting exists."""
    n = 2
    cp, ri = ochol.lower_csc(n, np.array([0, 1, 1]), np.array([0, 0, 1]))
    vals = np.array([0.0, 1.0, 0.0])
    ch = ochol.Cholesky(n, cp, ri, np.arange(n, dtype=np.int32))
    assert ch.factor(vals, ldlt=True) == 0
