"""CPU-side checks of the C-ABI library: it loads, exports every declared symbol, and its host logic
(structure, bounds, condensed pattern, symbolic analysis) is bit-exact with the oracle.  No device
compute is called: device uploads are deferred to the first device use."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import chol as ochol
from oracle import kkt as okkt
from oracle.model import Model as OModel
from paper_2307_16830_amd import gridgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OPTS = dict(dense_frac=0.5, dense_abs=2 ** 31 - 1, max_width=2 ** 31 - 1, zero_abs=64, zero_rel=0.05)


def opf():
    from paper_2307_16830_amd import opf as _opf
    return _opf


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "opf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_]+)\s*\(", text)) - {"if", "sizeof"})


def test_library_exports_every_declared_symbol():
    lib = opf().lib()
    syms = declared_symbols()
    assert len(syms) >= 25
    for name in syms:
        assert hasattr(lib, name), name
    assert set(opf().EXPORTED) <= set(syms)


def test_invalid_grid_is_rejected():
    g = gridgen.make_grid(5, 6, 2, 1)
    g.f[0] = 99
    with pytest.raises(opf().OpfError) as e:
        opf().Model(g)
    assert e.value.code == opf().E_INVALID


def _break(g, what):
    if what == "self_loop":
        g.t[1] = g.f[1]
    elif what == "to_out_of_range":
        g.t[2] = -1
    elif what == "zero_impedance":
        g.r[0] = 0.0
        g.x[0] = 0.0
    elif what == "rating":
        g.rate[3] = 0.0
    elif what == "gen_bus":
        g.gbus[0] = len(g.pd)
    elif what == "gen_limits":
        g.pmin[1] = g.pmax[1] + 1.0
    elif what == "vm_bounds":
        g.vmin[4] = g.vmax[4] + 0.01
    elif what == "vm_zero":
        g.vmin[0] = 0.0
    elif what == "ref_bus":
        g.ref_bus = len(g.pd)
    elif what == "base_mva":
        g.base_mva = 0.0


@pytest.mark.parametrize("what", ["self_loop", "to_out_of_range", "zero_impedance", "rating", "gen_bus",
                                  "gen_limits", "vm_bounds", "vm_zero", "ref_bus", "base_mva"])
def test_each_grid_check_rejects(what):
    """Every grid check (shared by opf_create and the solve server's submission) turns its bad input into
    E_INVALID with a message naming the problem, and the unbroken grid is accepted."""
    g = gridgen.make_grid(8, 10, 3, 2)
    opf().Model(g)
    _break(g, what)
    with pytest.raises(opf().OpfError) as e:
        opf().Model(g)
    assert e.value.code == opf().E_INVALID
    assert "invalid grid" in str(e.value)


@pytest.mark.parametrize("case", ["cfg0", (40, 55, 8, 3), "cfg1"])
def test_host_structure_and_symbolic_match_oracle(case):
    g = gridgen.make_config(case) if isinstance(case, str) else gridgen.make_grid(*case)
    M = opf().Model(g)
    om = OModel(g)
    x0 = om.flat_start()
    assert np.array_equal(M.initial_point(), x0)
    xl, xu, gl, gu = M.bounds()
    for a, b in ((xl, om.xl), (xu, om.xu), (gl, om.gl), (gu, om.gu)):
        assert np.array_equal(a, b)
    jr, jc, hr, hc = M.structure()
    ojr, ojc, _, _ = om.jacobian(x0)
    ohr, ohc, _, _ = om.hessian(x0, np.zeros(om.L.m), 1.0)
    assert sorted(zip(jr.tolist(), jc.tolist())) == sorted(zip(ojr.tolist(), ojc.tolist()))
    assert sorted(zip(hr.tolist(), hc.tolist())) == sorted(zip(ohr.tolist(), ohc.tolist()))
    cp, ri = M.kkt_pattern()
    kr, kc = okkt.kkt_pattern(om.L.n, ojr, ojc, ohr, ohc)
    ocp, ori = ochol.lower_csc(om.L.n, kr, kc)
    assert np.array_equal(cp, ocp) and np.array_equal(ri, ori)
    C = opf().Cholesky(M.n, cp, ri, opf().chol_options(**OPTS))
    sym = ochol.analyze(M.n, cp, ri, ochol.AnalyzeOptions(**OPTS))
    par, cc = C.etree()
    assert np.array_equal(C.perm(), sym.perm)
    assert np.array_equal(par, sym.parent)
    assert np.array_equal(cc, sym.colcount)
    assert np.array_equal(C.supernodes(), sym.snode_ptr)
    # supernode row structures equal the union of the oracle's column structures
    oc = ochol.Cholesky(M.n, cp, ri, sym.perm)
    lp, li, _ = oc.export()
    rp, rows = C.supernode_rows()
    sp = sym.snode_ptr
    for t in range(len(sp) - 1):
        cols = range(sp[t], sp[t + 1])
        union = set(range(sp[t], sp[t + 1]))
        for j in cols:
            union |= set(li[lp[j]:lp[j + 1]].tolist())
        got = rows[rp[t]:rp[t + 1]]
        assert list(got[:sp[t + 1] - sp[t]]) == list(cols)
        assert sorted(got.tolist()) == sorted(union)


@pytest.mark.parametrize("opts", [dict(max_width=8, zero_abs=0, zero_rel=0.0),
                                  dict(dense_frac=0.3, max_width=32, zero_abs=16, zero_rel=0.2),
                                  dict(dense_abs=40)])
def test_symbolic_options_bit_exact(opts):
    g = gridgen.make_grid(200, 270, 30, 9)
    M = opf().Model(g)
    cp, ri = M.kkt_pattern()
    o = dict(OPTS)
    o.update(opts)
    C = opf().Cholesky(M.n, cp, ri, opf().chol_options(**o))
    sym = ochol.analyze(M.n, cp, ri, ochol.AnalyzeOptions(**o))
    assert np.array_equal(C.perm(), sym.perm)
    assert np.array_equal(C.etree()[0], sym.parent)
    assert np.array_equal(C.supernodes(), sym.snode_ptr)


def random_pattern(rng, n):
    """Lower CSC pattern (diagonal included) of a random symmetric graph: a few components, some dense rows,
    isolated vertices and many equal degrees, so the ordering's tie-breaking and its dense cut are exercised."""
    edges = set()
    kind = rng.integers(4)
    if kind == 0:  # sparse random graph
        for _ in range(int(n * rng.uniform(0.5, 3.0))):
            a, b = rng.integers(n, size=2)
            edges.add((max(a, b), min(a, b)))
    elif kind == 1:  # grid-like: a path plus chords, all degrees nearly equal
        for i in range(1, n):
            if rng.random() < 0.9:
                edges.add((i, i - 1))
        for _ in range(n // 4):
            a, b = rng.integers(n, size=2)
            edges.add((max(a, b), min(a, b)))
    elif kind == 2:  # a few dense rows over a sparse background
        for _ in range(n):
            a, b = rng.integers(n, size=2)
            edges.add((max(a, b), min(a, b)))
        for h in rng.integers(n, size=3):
            for j in rng.choice(n, size=n // 2, replace=False):
                edges.add((max(h, j), min(h, j)))
    else:  # disjoint cliques and stars
        start = 0
        while start < n:
            size = int(rng.integers(1, 9))
            block = range(start, min(n, start + size))
            for a in block:
                for b in block:
                    if a > b and (rng.random() < 0.7 or b == start):
                        edges.add((a, b))
            start += size
    cols = [[j] for j in range(n)]
    for a, b in edges:
        if a != b:
            cols[b].append(a)
    cp = np.zeros(n + 1, dtype=np.int32)
    ri = []
    for j in range(n):
        c = sorted(set(cols[j]))
        ri.extend(c)
        cp[j + 1] = cp[j] + len(c)
    return cp, np.array(ri, dtype=np.int32)


@pytest.mark.parametrize("seed", range(40))
def test_symbolic_bit_exact_on_random_patterns(seed):
    """Exact minimum degree (degrees recounted lazily from lower bounds), etree, column counts and supernodes
    against the oracle's explicit elimination-graph ordering and column-union symbolic factorization."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 160))
    cp, ri = random_pattern(rng, n)
    o = dict(OPTS)
    if seed % 3 == 1:
        o.update(dense_frac=0.3)
    if seed % 3 == 2:
        o.update(dense_abs=int(rng.integers(2, 12)), zero_abs=0, zero_rel=0.0)
    C = opf().Cholesky(n, cp, ri, opf().chol_options(**o))
    sym = ochol.analyze(n, cp, ri, ochol.AnalyzeOptions(**o))
    assert np.array_equal(C.perm(), sym.perm)
    par, cc = C.etree()
    assert np.array_equal(par, sym.parent)
    assert np.array_equal(cc, sym.colcount)
    assert np.array_equal(C.supernodes(), sym.snode_ptr)


def test_chol_analyze_rejects_bad_patterns():
    O = opf()
    with pytest.raises(O.OpfError):
        O.Cholesky(3, np.array([0, 1, 2, 2]), np.array([0, 1]))  # column 2 lacks its diagonal
    with pytest.raises(O.OpfError):
        O.Cholesky(2, np.array([0, 1, 2]), np.array([1, 1]))  # entry above the diagonal


def test_serving_defaults_and_argument_checks():
    O = opf()
    o = O.ServeOptions()
    O.lib().serve_default_options(ctypes.byref(o))
    assert o.slots == 8 and o.hbm_budget == 8 << 30
    assert o.ipm.tol == 1e-4 and o.chol.dense_frac == 0.5
    # argument errors are reported before any device work
    h = ctypes.c_void_p()
    bad = O.ServeOptions()
    O.lib().serve_default_options(ctypes.byref(bad))
    bad.slots = 0
    assert O.lib().opf_serve_create(ctypes.byref(bad), ctypes.byref(h)) == O.E_INVALID
    assert O.lib().opf_serve_submit(None, None, 0) == O.E_INVALID
    assert O.lib().opf_serve_destroy(None) == O.OK
    assert O.lib().opf_serve_now() > 0


def test_factor_storage_is_the_lower_block_trapezoid():
    """Each front keeps only its lower part: 64-column panels, panel p holding rows 64p.. of its columns, so
    the device factor takes about half the bytes of full m x m squares."""
    g = gridgen.make_config("cfg1")
    M = opf().Model(g)
    cp, ri = M.kkt_pattern()
    C = opf().Cholesky(M.n, cp, ri, opf().chol_options(**OPTS))
    rp, _ = C.supernode_rows()
    total = square = 0
    for m in np.diff(rp).tolist():
        square += m * m
        for c0 in range(0, m, 64):
            total += min(64, m - c0) * (m - c0)
    assert C.factor_bytes == 8 * total
    assert max(np.diff(rp)) > 1000  # a front large enough for the halving to show
    assert C.factor_bytes < 0.7 * 8 * square  # small fronts (m <= 64) stay whole squares
