"""Oracle: condensed KKT system of the relaxed barrier problem (FP64, CPU).

TEST INFRASTRUCTURE ONLY.

Section IV-C of the paper: after eliminating the bound multipliers from the
full Newton system (the 7x7 block matrix) one obtains the augmented system,
and after eliminating the slack and multiplier steps the condensed system

    (W + dw I + Sx + J^T D J) dx = qx + J^T (qs + D qy),   D = Ss + dw I

(with the dual regularization dc = 0, so C = I).  This module forms those
objects from their definitions and implements the recovery of the other step
components.  Sign convention: the step is the Newton step on the residual map
F (rows of the first-order conditions, Section IV-C) and solves
``J_F d = R``; ``dy`` is the step of ``y`` itself.  (The paper's printed full
matrix carries +A^T in the x row, i.e. its dy is the step of -y; the printed
slack recovery ``C(dc qs - (qy + A dx))`` has the opposite sign of
``A dx - qy`` obtained by elimination -- the elimination result is used.)
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def kkt_pattern(n, jrow, jcol, hrow, hcol):
    """Structural lower pattern of K: diagonal, Hessian pattern, and every column pair of each Jacobian row.

    Returns (rows, cols) with row >= col, sorted by (col, row), unique.
    """
    jrow = np.asarray(jrow, dtype=np.int64)
    jcol = np.asarray(jcol, dtype=np.int64)
    order = np.lexsort((jcol, jrow))
    jr = jrow[order]
    jc = jcol[order]
    # group entries by row; pair every entry with every entry of its row
    uniq, start, counts = np.unique(jr, return_index=True, return_counts=True)
    rowlen = np.zeros(int(jr.max()) + 1 if len(jr) else 1, dtype=np.int64)
    rowstart = np.zeros_like(rowlen)
    rowlen[uniq] = counts
    rowstart[uniq] = start
    rep = rowlen[jr]
    a = np.repeat(np.arange(len(jr)), rep)
    grp_off = np.repeat(np.cumsum(rep) - rep, rep)
    b = rowstart[jr[a]] + (np.arange(len(a)) - grp_off)
    pr = np.maximum(jc[a], jc[b])
    pc = np.minimum(jc[a], jc[b])
    hrow = np.asarray(hrow, dtype=np.int64)
    hcol = np.asarray(hcol, dtype=np.int64)
    d = np.arange(n, dtype=np.int64)
    R = np.concatenate([d, hrow, pr])
    C = np.concatenate([d, hcol, pc])
    key = np.unique(C * n + R)
    return key % n, key // n


def sym_from_lower(n, rows, cols, vals):
    """Full symmetric sparse matrix (CSR) from lower COO entries (duplicates add)."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    off = rows != cols
    R = np.concatenate([rows, cols[off]])
    C = np.concatenate([cols, rows[off]])
    V = np.concatenate([vals, np.asarray(vals)[off]])
    return sp.csr_matrix((V, (R, C)), shape=(n, n))


def jac_matrix(m, n, jrow, jcol, jval):
    return sp.csr_matrix((jval, (jrow, jcol)), shape=(m, n))


def condensed_values(n, krow, kcol, hrow, hcol, hval, Jm, sigx, D, dw, hmag=None, jmag=None):
    """Values of K = W + dw I + Sx + J^T D J on the fixed pattern (krow, kcol).

    If ``hmag`` is given also returns the magnitude Wmag + Sx + dw + Jmag^T D Jmag
    used to scale parity tolerances, where Wmag and Jmag (a sparse matrix with
    the sparsity of J, default |J|) are the abs-sums of the product terms that
    formed each Hessian and Jacobian entry: an entry formed with cancellation
    carries rounding relative to its terms, not to its value.
    """
    W = sym_from_lower(n, hrow, hcol, hval)
    M = W + sp.diags(sigx + dw) + (Jm.T @ sp.diags(D) @ Jm)
    M = M.tocsr()
    vals = np.asarray(M[krow, kcol]).ravel()
    if hmag is None:
        return vals
    Wm = sym_from_lower(n, hrow, hcol, hmag)
    Ja = abs(Jm) if jmag is None else jmag
    Mm = (Wm + sp.diags(np.abs(sigx) + abs(dw)) + (Ja.T @ sp.diags(np.abs(D)) @ Ja)).tocsr()
    mags = np.asarray(Mm[krow, kcol]).ravel()
    return vals, mags


def lower_to_csc_values(n, krow, kcol, kval):
    """Reorder values given on (krow, kcol) into lower CSC order (columns, then rows ascending)."""
    order = np.lexsort((krow, kcol))
    return np.asarray(kval)[order]


def dense_M_full(W, J, dw, xl, xu, sl, su, x, s, zl, zu, vl, vu):
    """Dense full Newton matrix (rows x, s, y, zl, zu, vl, vu) for tiny problems.

    Infinite bounds keep their multiplier rows as identity rows (z = 0, dz = R).
    """
    n = W.shape[0]
    m = J.shape[0]
    N = n + m + m + n + n + m + m
    M = np.zeros((N, N))
    ox, os_, oy, ozl, ozu, ovl, ovu = 0, n, n + m, n + 2 * m, 2 * n + 2 * m, 3 * n + 2 * m, 3 * n + 3 * m
    I_n = np.eye(n)
    I_m = np.eye(m)
    M[ox:ox + n, ox:ox + n] = W + dw * I_n
    M[ox:ox + n, oy:oy + m] = -J.T
    M[ox:ox + n, ozl:ozl + n] = -I_n
    M[ox:ox + n, ozu:ozu + n] = I_n
    M[os_:os_ + m, os_:os_ + m] = dw * I_m
    M[os_:os_ + m, oy:oy + m] = I_m
    M[os_:os_ + m, ovl:ovl + m] = -I_m
    M[os_:os_ + m, ovu:ovu + m] = I_m
    M[oy:oy + m, ox:ox + n] = J
    M[oy:oy + m, os_:os_ + m] = -I_m
    fl = np.isfinite(xl)
    fu = np.isfinite(xu)
    gl = np.isfinite(sl)
    gu = np.isfinite(su)
    M[ozl:ozl + n, ox:ox + n] = np.diag(np.where(fl, zl, 0.0))
    M[ozl:ozl + n, ozl:ozl + n] = np.diag(np.where(fl, x - np.where(fl, xl, 0.0), 1.0))
    M[ozu:ozu + n, ox:ox + n] = -np.diag(np.where(fu, zu, 0.0))
    M[ozu:ozu + n, ozu:ozu + n] = np.diag(np.where(fu, np.where(fu, xu, 0.0) - x, 1.0))
    M[ovl:ovl + m, os_:os_ + m] = np.diag(np.where(gl, vl, 0.0))
    M[ovl:ovl + m, ovl:ovl + m] = np.diag(np.where(gl, s - np.where(gl, sl, 0.0), 1.0))
    M[ovu:ovu + m, os_:os_ + m] = -np.diag(np.where(gu, vu, 0.0))
    M[ovu:ovu + m, ovu:ovu + m] = np.diag(np.where(gu, np.where(gu, su, 0.0) - s, 1.0))
    return M
