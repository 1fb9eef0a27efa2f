"""Pins of the oracle's ordering, symbolic analysis and Cholesky against brute force and dense linear algebra."""
import math

import numpy as np
import pytest

from oracle import chol as ochol


def random_pattern(n, p, rng):
    A = rng.random((n, n)) < p
    A = np.tril(A | A.T, -1)
    rows, cols = np.nonzero(A)
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([cols, np.arange(n)])
    return ochol.lower_csc(n, rows, cols), A


def brute_min_degree(n, A, dense_frac=0.5, dense_abs=2 ** 31 - 1):
    """Elimination game on explicit adjacency sets (pure Python): smallest degree, ties to smallest index."""
    adj = [set() for _ in range(n)]
    r, c = np.nonzero(A)
    for i, j in zip(r.tolist(), c.tolist()):
        adj[i].add(j)
        adj[j].add(i)
    alive = set(range(n))
    order = []
    while alive:
        d, v = min((len(adj[u]), u) for u in alive)
        if d >= dense_frac * (len(alive) - 1) or d >= dense_abs:
            order.extend(sorted(alive))
            break
        order.append(v)
        nb = adj[v]
        for u in nb:
            adj[u] |= nb
            adj[u].discard(u)
            adj[u].discard(v)
        alive.discard(v)
        adj[v] = set()
    return np.array(order)


def dense_symbolic(n, A, perm):
    """Structure of L for P A P^T by boolean elimination on a dense matrix."""
    inv = np.empty(n, dtype=int)
    inv[perm] = np.arange(n)
    B = np.zeros((n, n), dtype=bool)
    r, c = np.nonzero(A)
    B[inv[r], inv[c]] = True
    B[inv[c], inv[r]] = True
    np.fill_diagonal(B, True)
    for k in range(n):
        rows = np.nonzero(B[k + 1:, k])[0] + k + 1
        B[np.ix_(rows, rows)] = True
    return np.tril(B)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("dense_frac", [0.5, 1.01])
def test_min_degree_matches_brute_force(seed, dense_frac):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    (cp, ri), A = random_pattern(n, 0.12, rng)
    got = ochol.min_degree(n, cp, ri, dense_frac=dense_frac)
    ref = brute_min_degree(n, A, dense_frac=dense_frac)
    assert np.array_equal(got, ref)


def test_dense_abs_cut():
    rng = np.random.default_rng(11)
    n = 30
    (cp, ri), A = random_pattern(n, 0.2, rng)
    got = ochol.min_degree(n, cp, ri, dense_frac=2.0, dense_abs=4)
    ref = brute_min_degree(n, A, dense_frac=2.0, dense_abs=4)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("seed", range(5))
def test_analysis_etree_colcounts_supernodes(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(10, 60))
    (cp, ri), A = random_pattern(n, 0.08, rng)
    opts = ochol.AnalyzeOptions(max_width=8, zero_abs=4, zero_rel=0.1)
    sym = ochol.analyze(n, cp, ri, opts)
    perm = sym.perm
    assert sorted(perm.tolist()) == list(range(n))
    Ls = dense_symbolic(n, A, perm)
    # etree: parent(j) = min{i > j: L(i,j) != 0}
    for j in range(n):
        below = np.nonzero(Ls[j + 1:, j])[0]
        assert sym.parent[j] == (below[0] + j + 1 if len(below) else -1)
    assert np.array_equal(sym.colcount, Ls.sum(axis=0))
    # postorder: every node's subtree is contiguous and ends at the node
    for j in range(n):
        p = sym.parent[j]
        if p >= 0:
            assert p > j
    # the permutation is the min-degree order composed with a postorder of its etree
    md = ochol.min_degree(n, cp, ri)
    Lmd = dense_symbolic(n, A, md)
    par_md = np.array([np.nonzero(Lmd[j + 1:, j])[0][0] + j + 1 if Lmd[j + 1:, j].any() else -1 for j in range(n)])
    post = _postorder(par_md)
    assert np.array_equal(perm, md[post])
    # supernodes: recompute with a direct Python implementation of the stated rules
    assert np.array_equal(sym.snode_ptr, _supernodes(sym.parent, sym.colcount, opts))


def _postorder(parent):
    n = len(parent)
    kids = [[] for _ in range(n)]
    for j in range(n):
        if parent[j] >= 0:
            kids[parent[j]].append(j)
    out = []

    def visit(v):
        for c in sorted(kids[v]):
            visit(c)
        out.append(v)

    for r in range(n):
        if parent[r] < 0:
            visit(r)
    return np.array(out)


def _supernodes(parent, cc, o):
    n = len(parent)
    nchild = np.zeros(n, dtype=int)
    for j in range(n):
        if parent[j] >= 0:
            nchild[parent[j]] += 1
    sn = [[0]]
    for j in range(1, n):
        if parent[j - 1] == j and cc[j - 1] == cc[j] + 1 and nchild[j] == 1:
            sn[-1].append(j)
        else:
            sn.append([j])
    first = [s[0] for s in sn]
    last = [s[-1] for s in sn]
    rows = [int(cc[s[0]]) for s in sn]
    zeros = [0] * len(sn)
    dead = [False] * len(sn)
    owner = {}
    for t, s in enumerate(sn):
        for j in s:
            owner[j] = t
    trap = lambda w, m: w * m - w * (w - 1) // 2  # noqa: E731
    for c in range(len(sn)):
        pc = parent[last[c]]
        if pc < 0:
            continue
        p = owner[pc]
        if last[c] + 1 != first[p]:
            continue
        nc, np_ = last[c] - first[c] + 1, last[p] - first[p] + 1
        nm, mm = nc + np_, nc + rows[p]
        z = zeros[c] + zeros[p] + trap(nm, mm) - trap(nc, rows[c]) - trap(np_, rows[p])
        if nm <= o.max_width and (z <= o.zero_abs or z <= o.zero_rel * trap(nm, mm)):
            first[p] = first[c]
            rows[p] = mm
            zeros[p] = z
            dead[c] = True
            for j in range(first[c], last[c] + 1):
                owner[j] = p
    return np.array([first[t] for t in range(len(sn)) if not dead[t]] + [n])


@pytest.mark.parametrize("seed", range(4))
def test_numeric_cholesky_matches_dense(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(10, 50))
    (cp, ri), A = random_pattern(n, 0.1, rng)
    # SPD values on the pattern: diagonally dominant
    vals = rng.normal(size=len(ri))
    cols = np.repeat(np.arange(n), np.diff(cp))
    diag = ri == cols
    K = np.zeros((n, n))
    K[ri, cols] = vals
    K = K + np.tril(K, -1).T
    for j in range(n):
        K[j, j] = np.sum(np.abs(K[j])) + 1.0
    vals[diag] = K[ri[diag], cols[diag]]
    sym = ochol.analyze(n, cp, ri)
    ch = ochol.Cholesky(n, cp, ri, sym.perm)
    assert ch.factor(vals) == -1
    lp, li, lx = ch.export()
    Ld = np.zeros((n, n))
    for j in range(n):
        Ld[li[lp[j]:lp[j + 1]], j] = lx[lp[j]:lp[j + 1]]
    P = K[np.ix_(sym.perm, sym.perm)]
    Lref = np.linalg.cholesky(P)
    assert np.allclose(Ld, Lref, rtol=1e-12, atol=1e-12 * np.max(np.abs(Lref)))
    b = rng.normal(size=n)
    x = ch.solve(b)
    assert np.allclose(x, np.linalg.solve(K, b), rtol=1e-10, atol=1e-12)


def test_not_positive_definite_reports_column():
    n = 4
    cp, ri = ochol.lower_csc(n, np.arange(n), np.arange(n))
    vals = np.array([1.0, 2.0, -1.0, 3.0])
    sym = ochol.analyze(n, cp, ri)
    ch = ochol.Cholesky(n, cp, ri, sym.perm)
    bad = ch.factor(vals)
    assert bad >= 0 and sym.perm[bad] == 2


def _threshold_matrix(frac):
    """3x3 matrix whose pivot for original column 1 is frac * K_11 exactly in real arithmetic:
    K = [[1, b, 0], [b, c, 0], [0, 0, 1e14]] with c = 1e12 and b^2 = c (1 - frac).  Column 2 is isolated, so
    minimum degree eliminates it first; the threshold pivot is the last one.  K_22 is the largest entry, so
    a threshold taken relative to max |K| instead of K_11 decides differently."""
    c = 1e12
    b = math.sqrt(c * (1.0 - frac))
    n = 3
    rows = np.array([0, 1, 1, 2])
    cols = np.array([0, 0, 1, 2])
    cp, ri = ochol.lower_csc(n, rows, cols)
    dense = np.array([[1.0, b, 0.0], [b, c, 0.0], [0.0, 0.0, 1e14]])
    colidx = np.repeat(np.arange(n), np.diff(cp))
    return n, cp, ri, dense[ri, colidx], dense


@pytest.mark.parametrize("frac,tol,rejected", [
    (5e-13, 1e-12, True),    # pivot 0.5 < 1e-12 * K_11 = 1: sign within rounding noise, rejected
    (5e-13, 0.0, False),     # textbook rule: positive, accepted
    (5e-13, 1e-13, False),   # 0.5 > 0.1
    (3e-12, 1e-12, False),   # 3 > 1
])
def test_pivot_threshold_is_relative_to_assembled_diagonal(frac, tol, rejected):
    """Pins the pivot acceptance rule d_j > tol * |K_jj| (Algorithm 1's inertia test on the condensed matrix):
    a comparison against L's diagonal (sqrt(d) ~ 0.7), against K_jj before the update, or against the
    largest entry of K would decide these cases differently."""
    n, cp, ri, vals, dense = _threshold_matrix(frac)
    sym = ochol.analyze(n, cp, ri)
    assert list(sym.perm) == [2, 0, 1]
    ch = ochol.Cholesky(n, cp, ri, sym.perm)
    bad = ch.factor(vals, piv_tol=tol)
    if rejected:
        assert bad == 2 and sym.perm[bad] == 1
    else:
        assert bad == -1
        lp, li, lx = ch.export()
        Ld = np.zeros((n, n))
        for j in range(n):
            Ld[li[lp[j]:lp[j + 1]], j] = lx[lp[j]:lp[j + 1]]
        # the accepted pivot is the Schur complement c - b^2 (exact up to the rounding of b^2)
        assert Ld[2, 2] ** 2 == pytest.approx(frac * 1e12, rel=1e-3)


def test_pivot_threshold_rejects_large_negative_pivot():
    """A pivot of large magnitude but negative sign is rejected at any tolerance (|d| must not be used)."""
    n = 2
    cp, ri = ochol.lower_csc(n, np.arange(n), np.arange(n))
    vals = np.array([1.0, -5.0])
    sym = ochol.analyze(n, cp, ri)
    ch = ochol.Cholesky(n, cp, ri, sym.perm)
    for tol in (0.0, 1e-12):
        bad = ch.factor(vals, piv_tol=tol)
        assert bad >= 0 and sym.perm[bad] == 1
