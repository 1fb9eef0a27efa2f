"""Oracle: ctypes wrapper over ``chol_oracle.c`` (symbolic analysis, Cholesky, solves).

TEST INFRASTRUCTURE ONLY.  See ``chol_oracle.c`` for the fully specified
ordering, elimination tree, postorder and supernode rules it implements.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

from . import build as _build

_lib = None
I32P = ctypes.POINTER(ctypes.c_int32)
F64P = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.oracle_min_degree.argtypes = [ctypes.c_int32, I32P, I32P, ctypes.c_double, ctypes.c_int32, I32P]
        L.oracle_min_degree.restype = ctypes.c_int
        L.oracle_analyze.argtypes = [ctypes.c_int32, I32P, I32P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int64, ctypes.c_double, I32P, I32P, I32P, I32P, I32P]
        L.oracle_analyze.restype = ctypes.c_int
        L.oracle_chol_create.argtypes = [ctypes.c_int32, I32P, I32P, I32P]
        L.oracle_chol_create.restype = ctypes.c_void_p
        L.oracle_chol_free.argtypes = [ctypes.c_void_p]
        L.oracle_chol_nnz.argtypes = [ctypes.c_void_p]
        L.oracle_chol_nnz.restype = ctypes.c_int64
        L.oracle_chol_export.argtypes = [ctypes.c_void_p, I32P, I32P, F64P]
        L.oracle_chol_factor.argtypes = [ctypes.c_void_p, F64P, ctypes.c_double]
        L.oracle_chol_factor.restype = ctypes.c_int
        L.oracle_chol_solve.argtypes = [ctypes.c_void_p, F64P, F64P]
        L.oracle_ldlt_factor.argtypes = [ctypes.c_void_p, F64P, ctypes.c_double]
        L.oracle_ldlt_factor.restype = ctypes.c_int
        L.oracle_ldlt_solve.argtypes = [ctypes.c_void_p, F64P, F64P]
        _lib = L
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(I32P)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(F64P)


@dataclasses.dataclass
class AnalyzeOptions:
    """Ordering and amalgamation parameters (identical meaning on both sides)."""

    dense_frac: float = 0.5
    dense_abs: int = 2 ** 31 - 1
    max_width: int = 2 ** 31 - 1
    zero_abs: int = 64
    zero_rel: float = 0.05


@dataclasses.dataclass
class Symbolic:
    perm: np.ndarray
    parent: np.ndarray
    colcount: np.ndarray
    snode_ptr: np.ndarray


def lower_csc(n, rows, cols):
    """Lower-triangular CSC pattern (colptr, rowind) of a symmetric pattern given as (row>=col) pairs."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    assert np.all(rows >= cols)
    key = np.unique(cols * n + rows)
    c = key // n
    r = key % n
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, c + 1, 1)
    return np.cumsum(colptr).astype(np.int32), r.astype(np.int32)


def min_degree(n, colptr, rowind, dense_frac=0.5, dense_abs=2 ** 31 - 1):
    cp, cpp = _i32(colptr)
    ri, rip = _i32(rowind)
    order = np.zeros(n, dtype=np.int32)
    rc = lib().oracle_min_degree(n, cpp, rip, float(dense_frac), int(dense_abs), order.ctypes.data_as(I32P))
    if rc != 0:
        raise MemoryError("oracle_min_degree failed")
    return order


def analyze(n, colptr, rowind, opts: AnalyzeOptions | None = None) -> Symbolic:
    o = opts or AnalyzeOptions()
    cp, cpp = _i32(colptr)
    ri, rip = _i32(rowind)
    perm = np.zeros(n, dtype=np.int32)
    parent = np.zeros(n, dtype=np.int32)
    cc = np.zeros(n, dtype=np.int32)
    sp = np.zeros(n + 1, dtype=np.int32)
    ns = ctypes.c_int32(0)
    rc = lib().oracle_analyze(n, cpp, rip, float(o.dense_frac), int(o.dense_abs), int(o.max_width),
                              int(o.zero_abs), float(o.zero_rel), perm.ctypes.data_as(I32P),
                              parent.ctypes.data_as(I32P), cc.ctypes.data_as(I32P), sp.ctypes.data_as(I32P),
                              ctypes.byref(ns))
    if rc != 0:
        raise MemoryError("oracle_analyze failed")
    return Symbolic(perm, parent, cc, sp[: ns.value + 1].copy())


class Cholesky:
    """Numeric Cholesky of P K P^T for a fixed lower CSC pattern and permutation."""

    def __init__(self, n, colptr, rowind, perm):
        self.n = int(n)
        self._cp, cpp = _i32(colptr)
        self._ri, rip = _i32(rowind)
        self._perm, pp = _i32(perm)
        self._h = lib().oracle_chol_create(self.n, cpp, rip, pp)
        if not self._h:
            raise MemoryError("oracle_chol_create failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_chol_free(h)
            self._h = None

    @property
    def nnz(self):
        return int(lib().oracle_chol_nnz(self._h))

    def factor(self, values, piv_tol=0.0, ldlt=False):
        """Returns -1 if every pivot is accepted, else the first failing pivot column (permuted numbering).
        Cholesky: a pivot is accepted when it exceeds piv_tol * |K_jj| (0: K positive definite).  ``ldlt``: the
        LU factorization with the fixed pivot sequence in its symmetric form L D L^T, a pivot accepted when
        |d| exceeds piv_tol * |K_jj| (0: when it is nonzero); the factor then holds D on its diagonal."""
        v, vp = _f64(values)
        assert v.shape[0] == self._ri.shape[0]
        fn = lib().oracle_ldlt_factor if ldlt else lib().oracle_chol_factor
        rc = fn(self._h, vp, float(piv_tol))
        if rc < 0:
            raise MemoryError("oracle factorization failed")
        self._ldlt = bool(ldlt)
        return -1 if rc == 0 else rc - 1

    def solve(self, b):
        b, bp = _f64(b)
        x = np.zeros(self.n)
        fn = lib().oracle_ldlt_solve if getattr(self, "_ldlt", False) else lib().oracle_chol_solve
        fn(self._h, bp, x.ctypes.data_as(F64P))
        return x

    def inertia(self):
        """(positive, negative) pivot counts of the last L D L^T factorization."""
        lp, _, lx = self.export()
        d = lx[lp[:-1]]
        return int((d > 0).sum()), int((d < 0).sum())

    def export(self):
        """(colptr, rowind, values) of L in the permuted numbering."""
        nnz = self.nnz
        lp = np.zeros(self.n + 1, dtype=np.int32)
        li = np.zeros(nnz, dtype=np.int32)
        lx = np.zeros(nnz)
        lib().oracle_chol_export(self._h, lp.ctypes.data_as(I32P), li.ctypes.data_as(I32P),
                                 lx.ctypes.data_as(F64P))
        return lp, li, lx
