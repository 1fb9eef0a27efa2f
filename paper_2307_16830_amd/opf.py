"""Thin ctypes binding over ``libopf.so`` (declared in ``include/opf.h``).

Argument marshalling only: every numeric step runs in the HIP library.
Device buffers are torch tensors on ``cuda`` (PyTorch provides memory and
streams); host outputs are numpy arrays.  Loading fails loudly if the library
has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libopf.so")

I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)
F64P = ctypes.POINTER(ctypes.c_double)
VP = ctypes.c_void_p

OK, E_INVALID, E_NOMEM, E_DEVICE, E_STATE, E_NOT_PD, E_MAXITER, E_LINESEARCH, E_NUMERIC, E_BUDGET = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
EVAL_F, EVAL_C, EVAL_GRAD, EVAL_JAC, EVAL_HESS, EVAL_JAC_VAR = 1, 2, 4, 8, 16, 32
EXPORTED = [
    "opf_last_error", "opf_default_options", "opf_create", "opf_destroy", "opf_dims", "opf_structure", "opf_bounds", "opf_initial_point",
    "opf_eval_derivs", "kkt_pattern", "kkt_condense", "chol_default_options", "chol_analyze", "chol_destroy",
    "chol_info", "chol_perm", "chol_etree", "chol_supernodes", "chol_supernode_rows", "chol_factor", "chol_solve",
    "chol_solve_noalloc", "chol_graph_stats", "chol_inertia",
    "chol_export_factor", "ipm_default_options", "ipm_create", "ipm_destroy", "ipm_step", "ipm_solve",
    "ipm_get_iterate", "ipm_chol", "ipm_get_state", "ipm_set_state", "ipm_direction", "chol_timing",
    "chol_timing_read", "serve_default_options", "opf_serve_create", "opf_serve_submit", "opf_serve_poll",
    "opf_serve_get_x", "opf_serve_stats", "opf_serve_now", "opf_serve_destroy",
]


class OpfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class GridC(ctypes.Structure):
    _fields_ = [("nbus", ctypes.c_int32), ("nbranch", ctypes.c_int32), ("ngen", ctypes.c_int32),
                ("ref_bus", ctypes.c_int32), ("base_mva", ctypes.c_double)] + \
               [(k, F64P) for k in ("pd", "qd", "gs", "bs", "vmin", "vmax")] + \
               [("f", I32P), ("t", I32P)] + [(k, F64P) for k in ("r", "x", "b", "rate", "angmin", "angmax")] + \
               [("gbus", I32P)] + [(k, F64P) for k in ("c2", "c1", "c0", "pmin", "pmax", "qmin", "qmax")]


class OpfOptions(ctypes.Structure):
    _fields_ = [("assembly", ctypes.c_int32)]


class IpmResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32)] + \
               [(k, ctypes.c_double) for k in ("objective", "e0", "inf_pr", "inf_du")] + \
               [("factorizations", ctypes.c_int32), ("ir_steps", ctypes.c_int32)] + \
               [(k, ctypes.c_double) for k in ("t_ad", "t_assembly", "t_factor", "t_solve", "t_total")] + \
               [("x", VP), ("s", VP), ("y", VP)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k not in ("x", "s", "y")}


class CholOptions(ctypes.Structure):
    _fields_ = [("dense_frac", ctypes.c_double), ("dense_abs", ctypes.c_int32), ("max_width", ctypes.c_int32),
                ("zero_abs", ctypes.c_int64), ("zero_rel", ctypes.c_double), ("pivot_tol", ctypes.c_double),
                ("tile_min", ctypes.c_int32), ("pair_min", ctypes.c_int32), ("pair_panels", ctypes.c_int32),
                ("ldlt", ctypes.c_int32)]


class IpmOptions(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("max_ir", ctypes.c_int32),
                ("ir_tol", ctypes.c_double), ("mu_init", ctypes.c_double), ("bound_relax", ctypes.c_double),
                ("pivot_tol", ctypes.c_double), ("graphs", ctypes.c_int32), ("soc", ctypes.c_int32)]


class ServeOptions(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("hbm_budget", ctypes.c_int64), ("ipm", IpmOptions),
                ("chol", CholOptions)]


class ServeResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("objective", ctypes.c_double), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("footprint", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("message", ctypes.c_char * 160)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["message"] = d["message"].decode(errors="replace")
        return d


class IterInfo(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32)] + [(k, ctypes.c_double) for k in
                                             ("obj", "e0", "inf_pr", "inf_du", "mu", "delta_w", "alpha",
                                              "alpha_z")] + \
               [(k, ctypes.c_int32) for k in ("ls_trials", "ir_steps", "factorizations")] + \
               [(k, ctypes.c_double) for k in ("t_ad", "t_assembly", "t_factor", "t_solve", "t_total")] + \
               [("soc_steps", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2307_16830_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.opf_last_error.restype = ctypes.c_char_p
        L.opf_default_options.argtypes = [ctypes.POINTER(OpfOptions)]
        L.opf_default_options.restype = None
        L.opf_create.argtypes = [ctypes.POINTER(GridC), ctypes.POINTER(OpfOptions), VP, ctypes.POINTER(VP)]
        L.opf_destroy.argtypes = [VP]
        L.opf_dims.argtypes = [VP, I32P, I32P, I64P, I64P, I64P]
        L.opf_structure.argtypes = [VP, I32P, I32P, I32P, I32P]
        L.opf_bounds.argtypes = [VP, F64P, F64P, F64P, F64P]
        L.opf_initial_point.argtypes = [VP, F64P]
        L.opf_eval_derivs.argtypes = [VP, ctypes.c_uint, VP, VP, ctypes.c_double, VP, VP, VP, VP, VP, VP]
        L.kkt_pattern.argtypes = [VP, I32P, I32P]
        L.kkt_condense.argtypes = [VP, VP, VP, VP, VP, ctypes.c_double, VP, VP, VP, VP, VP]
        L.chol_default_options.argtypes = [ctypes.POINTER(CholOptions)]
        L.chol_default_options.restype = None
        L.chol_analyze.argtypes = [ctypes.c_int32, I32P, I32P, ctypes.POINTER(CholOptions), ctypes.POINTER(VP)]
        L.chol_destroy.argtypes = [VP]
        L.chol_info.argtypes = [VP, I32P, I64P, F64P, I64P]
        L.chol_perm.argtypes = [VP, I32P]
        L.chol_etree.argtypes = [VP, I32P, I32P]
        L.chol_supernodes.argtypes = [VP, I32P]
        L.chol_supernode_rows.argtypes = [VP, I64P, I32P]
        L.chol_factor.argtypes = [VP, VP, VP, I32P]
        L.chol_solve.argtypes = [VP, VP, VP, ctypes.c_int32, VP]
        L.chol_solve_noalloc.argtypes = [VP, VP, VP, ctypes.c_int32, VP]
        L.chol_graph_stats.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.chol_inertia.argtypes = [VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.chol_export_factor.argtypes = [VP, I64P, I32P, F64P]
        L.chol_timing.argtypes = [VP, ctypes.c_int]
        L.chol_timing_read.argtypes = [VP, F64P, I64P, F64P, F64P]
        L.ipm_default_options.argtypes = [ctypes.POINTER(IpmOptions)]
        L.ipm_default_options.restype = None
        L.ipm_create.argtypes = [VP, ctypes.POINTER(IpmOptions), ctypes.POINTER(CholOptions), VP, ctypes.POINTER(VP)]
        L.ipm_destroy.argtypes = [VP]
        L.ipm_step.argtypes = [VP, ctypes.POINTER(IterInfo)]
        L.ipm_solve.argtypes = [VP, ctypes.POINTER(IpmResult)]
        L.ipm_get_iterate.argtypes = [VP, F64P, F64P, F64P]
        L.ipm_chol.argtypes = [VP]
        L.ipm_chol.restype = VP
        L.ipm_get_state.argtypes = [VP] + [F64P] * 9
        L.ipm_set_state.argtypes = [VP] + [F64P] * 7 + [ctypes.c_double, ctypes.c_double]
        L.ipm_direction.argtypes = [VP] + [F64P] * 8 + [I32P]
        L.serve_default_options.argtypes = [ctypes.POINTER(ServeOptions)]
        L.serve_default_options.restype = None
        L.opf_serve_create.argtypes = [ctypes.POINTER(ServeOptions), ctypes.POINTER(VP)]
        L.opf_serve_submit.argtypes = [VP, ctypes.POINTER(GridC), ctypes.c_int64]
        L.opf_serve_poll.argtypes = [VP, ctypes.POINTER(ServeResult), ctypes.c_int32, I32P, ctypes.c_int32]
        L.opf_serve_get_x.argtypes = [VP, ctypes.c_int64, F64P, ctypes.c_int32]
        L.opf_serve_stats.argtypes = [VP, I64P, I64P, I32P, I32P]
        L.opf_serve_now.argtypes = []
        L.opf_serve_now.restype = ctypes.c_double
        L.opf_serve_destroy.argtypes = [VP]
        _lib = L
    return _lib


def _check(rc, what=""):
    if rc < 0:
        raise OpfError(rc, f"{what}: {lib().opf_last_error().decode(errors='replace')}")
    return rc


def _p(a, ctype):
    return a.ctypes.data_as(ctype)


def _dptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device buffers must be contiguous cuda tensors"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream)


def chol_options(**kw):
    o = CholOptions()
    lib().chol_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def ipm_options(**kw):
    o = IpmOptions()
    lib().ipm_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _grid_struct(grid, keep):
    """opf_grid view of a generated grid; ``keep`` holds the arrays alive while the struct is used."""
    g = GridC()
    g.nbus, g.nbranch, g.ngen = grid.nbus, grid.nbranch, grid.ngen
    g.ref_bus, g.base_mva = int(grid.ref_bus), float(grid.base_mva)
    for k in ("pd", "qd", "gs", "bs", "vmin", "vmax", "r", "x", "b", "rate", "angmin", "angmax",
              "c2", "c1", "c0", "pmin", "pmax", "qmin", "qmax"):
        a = np.ascontiguousarray(getattr(grid, k), dtype=np.float64)
        keep[k] = a
        setattr(g, k, _p(a, F64P))
    for k in ("f", "t", "gbus"):
        a = np.ascontiguousarray(getattr(grid, k), dtype=np.int32)
        keep[k] = a
        setattr(g, k, _p(a, I32P))
    return g


class Model:
    """An ACOPF instance on the device (wraps ``opf_model``)."""

    def __init__(self, grid, assembly=0, stream=None):
        self._keep = {}
        g = _grid_struct(grid, self._keep)
        o = OpfOptions()
        lib().opf_default_options(ctypes.byref(o))
        o.assembly = int(assembly)
        h = VP()
        # the uploads run at the model's first device use, on `stream` (None: the null stream, so that host-only
        # queries never touch the GPU)
        st = ctypes.c_void_p(stream) if stream is not None else None
        _check(lib().opf_create(ctypes.byref(g), ctypes.byref(o), st, ctypes.byref(h)), "opf_create")
        self._h = h
        self._keep = None
        n, m = ctypes.c_int32(), ctypes.c_int32()
        nj, nh, nk = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().opf_dims(h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(nj), ctypes.byref(nh),
                              ctypes.byref(nk)), "opf_dims")
        self.n, self.m, self.nnzj, self.nnzh, self.nnzk = n.value, m.value, nj.value, nh.value, nk.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.opf_destroy(self._h)
        self._h = None

    __del__ = close

    def structure(self):
        jr = np.zeros(self.nnzj, np.int32)
        jc = np.zeros(self.nnzj, np.int32)
        hr = np.zeros(self.nnzh, np.int32)
        hc = np.zeros(self.nnzh, np.int32)
        _check(lib().opf_structure(self._h, _p(jr, I32P), _p(jc, I32P), _p(hr, I32P), _p(hc, I32P)), "opf_structure")
        return jr, jc, hr, hc

    def bounds(self):
        xl, xu = np.zeros(self.n), np.zeros(self.n)
        gl, gu = np.zeros(self.m), np.zeros(self.m)
        _check(lib().opf_bounds(self._h, _p(xl, F64P), _p(xu, F64P), _p(gl, F64P), _p(gu, F64P)), "opf_bounds")
        return xl, xu, gl, gu

    def initial_point(self):
        x0 = np.zeros(self.n)
        _check(lib().opf_initial_point(self._h, _p(x0, F64P)), "opf_initial_point")
        return x0

    def kkt_pattern(self):
        cp = np.zeros(self.n + 1, np.int32)
        ri = np.zeros(self.nnzk, np.int32)
        _check(lib().kkt_pattern(self._h, _p(cp, I32P), _p(ri, I32P)), "kkt_pattern")
        return cp, ri

    def eval_derivs(self, what, x, y=None, obj_weight=1.0, f=None, c=None, grad=None, jac=None, hess=None,
                    stream=None):
        _check(lib().opf_eval_derivs(self._h, what, _dptr(x), _dptr(y), float(obj_weight), _dptr(f), _dptr(c),
                                     _dptr(grad), _dptr(jac), _dptr(hess), _stream(stream)), "opf_eval_derivs")

    def condense(self, hess, jac, sigx, dvec, delta_w, kval, qx=None, v=None, rhs=None, stream=None):
        _check(lib().kkt_condense(self._h, _dptr(hess), _dptr(jac), _dptr(sigx), _dptr(dvec), float(delta_w),
                                  _dptr(kval), _dptr(qx), _dptr(v), _dptr(rhs), _stream(stream)), "kkt_condense")


class Cholesky:
    """Symbolic analysis (host) + numeric factor/solve (device) of a lower CSC pattern (wraps ``chol_sym``)."""

    def __init__(self, n, colptr, rowind, opts=None, handle=None):
        self.n = int(n)
        self._owned = handle is None
        if handle is None:
            cp = np.ascontiguousarray(colptr, dtype=np.int32)
            ri = np.ascontiguousarray(rowind, dtype=np.int32)
            h = VP()
            o = opts if opts is not None else chol_options()
            _check(lib().chol_analyze(self.n, _p(cp, I32P), _p(ri, I32P), ctypes.byref(o), ctypes.byref(h)),
                   "chol_analyze")
            self._h = h
        else:
            self._h = VP(handle)
        ns, nl, fb = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        fl = ctypes.c_double()
        _check(lib().chol_info(self._h, ctypes.byref(ns), ctypes.byref(nl), ctypes.byref(fl), ctypes.byref(fb)),
               "chol_info")
        self.nsuper, self.nnz_l, self.flops, self.factor_bytes = ns.value, nl.value, fl.value, fb.value

    def close(self):
        if self._owned and getattr(self, "_h", None) and _lib is not None:
            _lib.chol_destroy(self._h)
        self._h = None

    __del__ = close

    def perm(self):
        p = np.zeros(self.n, np.int32)
        _check(lib().chol_perm(self._h, _p(p, I32P)), "chol_perm")
        return p

    def etree(self):
        par = np.zeros(self.n, np.int32)
        cc = np.zeros(self.n, np.int32)
        _check(lib().chol_etree(self._h, _p(par, I32P), _p(cc, I32P)), "chol_etree")
        return par, cc

    def supernodes(self):
        sp = np.zeros(self.nsuper + 1, np.int32)
        _check(lib().chol_supernodes(self._h, _p(sp, I32P)), "chol_supernodes")
        return sp

    def supernode_rows(self):
        rp = np.zeros(self.nsuper + 1, np.int64)
        _check(lib().chol_supernode_rows(self._h, _p(rp, I64P), None), "chol_supernode_rows")
        rows = np.zeros(int(rp[-1]), np.int32)
        _check(lib().chol_supernode_rows(self._h, _p(rp, I64P), _p(rows, I32P)), "chol_supernode_rows")
        return rp, rows

    def factor(self, kval, stream=None):
        """Returns -1 when every pivot was accepted (Cholesky: K positive definite; ``ldlt``: no zero pivot), else
        the failing pivot index (no exception)."""
        bad = ctypes.c_int32(-1)
        rc = lib().chol_factor(self._h, _dptr(kval), _stream(stream), ctypes.byref(bad))
        if rc == E_NOT_PD:
            return bad.value
        _check(rc, "chol_factor")
        return -1

    def inertia(self):
        """(positive, negative) pivot counts of the last successful factorization (``chol_inertia``)."""
        p, q = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().chol_inertia(self._h, ctypes.byref(p), ctypes.byref(q)), "chol_inertia")
        return p.value, q.value

    def solve(self, b, x=None, stream=None):
        if x is None:
            import torch
            x = torch.empty_like(b)
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        _check(lib().chol_solve(self._h, _dptr(b), _dptr(x), nrhs, _stream(stream)), "chol_solve")
        return x

    def solve_noalloc(self, b, x, stream=None):
        """``chol_solve_noalloc``: the same solve with the library's static per-GPU scratch (no allocation);
        ``x`` must be given."""
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        _check(lib().chol_solve_noalloc(self._h, _dptr(b), _dptr(x), nrhs, _stream(stream)), "chol_solve_noalloc")
        return x

    TIMING_CATEGORIES = ("assembly", "small_fronts", "diag_block", "panel_solve", "trailing_update", "dense_front")

    def timing(self, categories=True):
        """Bracket the launches of the given categories (names from TIMING_CATEGORIES, or a bit mask;
        empty / 0 disables) with HIP events; resets the totals."""
        if isinstance(categories, (int, bool)):
            mask = (1 << len(self.TIMING_CATEGORIES)) - 1 if categories is True else int(categories)
        else:
            mask = sum(1 << self.TIMING_CATEGORIES.index(c) for c in categories)
        _check(lib().chol_timing(self._h, mask), "chol_timing")

    def timing_read(self):
        nc = len(self.TIMING_CATEGORIES)
        ms = np.zeros(nc)
        nl = np.zeros(nc, np.int64)
        fl = np.zeros(nc)
        by = np.zeros(nc)
        _check(lib().chol_timing_read(self._h, _p(ms, F64P), _p(nl, I64P), _p(fl, F64P), _p(by, F64P)),
               "chol_timing_read")
        return {k: {"ms": ms[i], "launches": int(nl[i]), "flops": fl[i], "bytes": by[i]}
                for i, k in enumerate(self.TIMING_CATEGORIES)}

    def export_factor(self, values=True):
        lp = np.zeros(self.n + 1, np.int64)
        li = np.zeros(self.nnz_l, np.int32)
        lx = np.zeros(self.nnz_l) if values else None
        _check(lib().chol_export_factor(self._h, _p(lp, I64P), _p(li, I32P), _p(lx, F64P) if values else None),
               "chol_export_factor")
        return lp, li, lx


class IPM:
    """Device-resident condensed-space IPM on one model (wraps ``ipm_state``)."""

    def __init__(self, model: Model, tol=1e-4, max_iter=500, chol_opts=None, stream=None, **kw):
        self.model = model
        o = ipm_options(tol=tol, max_iter=max_iter, **kw)
        h = VP()
        _check(lib().ipm_create(model.handle, ctypes.byref(o), ctypes.byref(chol_opts) if chol_opts else None,
                                _stream(stream), ctypes.byref(h)), "ipm_create")
        self._h = h
        self.log = []

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ipm_destroy(self._h)
        self._h = None

    __del__ = close

    def chol(self):
        return Cholesky(self.model.n, None, None, handle=lib().ipm_chol(self._h))

    def step(self):
        """One iteration; returns (status, info dict): 0 continue, 1 converged, <0 failure."""
        info = IterInfo()
        rc = lib().ipm_step(self._h, ctypes.byref(info))
        d = info.as_dict()
        self.log.append(d)
        if rc < 0 and rc not in (E_MAXITER, E_LINESEARCH, E_NUMERIC, E_NOT_PD):
            _check(rc, "ipm_step")
        return rc, d

    def solve(self):
        """Algorithm 1 to convergence: (status, iterations, objective); the whole ``ipm_result`` (totals, stage
        times, final optimality error) is left in ``self.result``."""
        r = IpmResult()
        rc = lib().ipm_solve(self._h, ctypes.byref(r))
        self.result = r.as_dict()
        if rc < 0 and rc not in (E_MAXITER, E_LINESEARCH, E_NUMERIC, E_NOT_PD):
            _check(rc, "ipm_solve")
        return rc, r.iterations, r.objective

    def get_state(self):
        n, m = self.model.n, self.model.m
        arrs = [np.zeros(k) for k in (n, m, m, n, n, m, m)]
        mu, dw = ctypes.c_double(), ctypes.c_double()
        _check(lib().ipm_get_state(self._h, *[_p(a, F64P) for a in arrs], ctypes.byref(mu), ctypes.byref(dw)),
               "ipm_get_state")
        return arrs, mu.value, dw.value

    def set_state(self, x, s, y, zl, zu, vl, vu, mu, dw_last=0.0):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, s, y, zl, zu, vl, vu)]
        _check(lib().ipm_set_state(self._h, *[_p(a, F64P) for a in arrs], float(mu), float(dw_last)),
               "ipm_set_state")

    def direction(self):
        """Newton direction of the current state: (list of 7 arrays, delta_w, ir_steps)."""
        n, m = self.model.n, self.model.m
        arrs = [np.zeros(k) for k in (n, m, m, n, n, m, m)]
        dw, ir = ctypes.c_double(), ctypes.c_int32()
        _check(lib().ipm_direction(self._h, *[_p(a, F64P) for a in arrs], ctypes.byref(dw), ctypes.byref(ir)),
               "ipm_direction")
        return arrs, dw.value, ir.value

    def iterate(self):
        x, s, y = np.zeros(self.model.n), np.zeros(self.model.m), np.zeros(self.model.m)
        _check(lib().ipm_get_iterate(self._h, _p(x, F64P), _p(s, F64P), _p(y, F64P)), "ipm_get_iterate")
        return x, s, y


def graph_stats():
    """(captures, fallbacks): launch sequences captured into HIP graphs so far in this process, and captures that
    failed and ran as plain launches instead."""
    c, f = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().chol_graph_stats(ctypes.byref(c), ctypes.byref(f)), "chol_graph_stats")
    return c.value, f.value


def status_name(rc):
    return {OK: "OK", 1: "CONVERGED", E_INVALID: "E_INVALID", E_NOMEM: "E_NOMEM", E_DEVICE: "E_DEVICE",
            E_STATE: "E_STATE", E_NOT_PD: "E_NOT_PD", E_MAXITER: "E_MAXITER", E_LINESEARCH: "E_LINESEARCH",
            E_NUMERIC: "E_NUMERIC", E_BUDGET: "E_BUDGET"}.get(rc, str(rc))


def serve_options(slots=8, hbm_budget=8 << 30, tol=1e-4, max_iter=500, chol_opts=None, **ipm_kw):
    o = ServeOptions()
    lib().serve_default_options(ctypes.byref(o))
    o.slots, o.hbm_budget = int(slots), int(hbm_budget)
    o.ipm.tol, o.ipm.max_iter = float(tol), int(max_iter)
    for k, v in ipm_kw.items():
        setattr(o.ipm, k, v)
    if chol_opts is not None:
        o.chol = chol_opts
    return o


class Server:
    """Continuous-batching ACOPF solve server (wraps ``opf_server``): submit grids at any time; each is
    admitted by device footprint into a worker slot and solved on that slot's stream."""

    def __init__(self, **kw):
        h = VP()
        _check(lib().opf_serve_create(ctypes.byref(serve_options(**kw)), ctypes.byref(h)), "opf_serve_create")
        self._h = h

    def submit(self, grid, tag):
        keep = {}
        g = _grid_struct(grid, keep)
        _check(lib().opf_serve_submit(self._h, ctypes.byref(g), int(tag)), "opf_serve_submit")

    def poll(self, wait=True, max_results=64):
        """Finished results (dicts, oldest first); with ``wait`` blocks until one is ready or all is done."""
        buf = (ServeResult * max_results)()
        cnt = ctypes.c_int32()
        _check(lib().opf_serve_poll(self._h, buf, max_results, ctypes.byref(cnt), 1 if wait else 0),
               "opf_serve_poll")
        return [buf[i].as_dict() for i in range(cnt.value)]

    def x(self, tag, n):
        out = np.empty(n)
        _check(lib().opf_serve_get_x(self._h, int(tag), _p(out, F64P), int(n)), "opf_serve_get_x")
        return out

    def stats(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        c, d = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().opf_serve_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)),
               "opf_serve_stats")
        return {"in_use": a.value, "peak_in_use": b.value, "running": c.value, "queued": d.value}

    @staticmethod
    def now():
        return lib().opf_serve_now()

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.opf_serve_destroy(self._h)
        self._h = None

    __del__ = close


INF = math.inf
