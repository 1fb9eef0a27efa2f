"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerances (derived from the arithmetic, see the design notes): derivative,
constraint and condensed-matrix entries agree to 1e-12 of the abs-sum of the
terms forming them (``mag``); patterns, permutations, elimination trees and
supernode partitions are bit-exact; solves reach ||Kx - b|| / ||b|| <= 1e-10;
IPM objectives agree to 1e-6 relative and iteration counts to +-2.
"""
import numpy as np
import pytest

from oracle import chol as ochol
from oracle import ipm as oipm
from oracle import kkt as okkt
from oracle.model import Model as OModel, canonical
from paper_2307_16830_amd import gridgen
from tests._grids import config_grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12
OPTS = dict(dense_frac=0.5, dense_abs=2 ** 31 - 1, max_width=2 ** 31 - 1, zero_abs=64, zero_rel=0.05)
# 80k buses: minimum degree stops at degree 1,500 (a ~42.6k-column dense root), as in the benchmark
OPTS_CFG3 = dict(OPTS, dense_abs=1500)


def opts_for(case):
    return OPTS_CFG3 if case == "cfg3" else OPTS


def opf():
    from paper_2307_16830_amd import opf as _opf
    return _opf


def dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def grid_for(name):
    if name in gridgen.CONFIGS:
        return config_grid(name)
    N, E, G, seed = name
    return gridgen.make_grid(N, E, G, seed)


def random_xy(om, seed):
    rng = np.random.default_rng(seed)
    L = om.L
    x = om.flat_start()
    x[L.ova:L.ova + L.N] = rng.uniform(-0.3, 0.3, L.N)
    x[L.ovm:L.ovm + L.N] = rng.uniform(0.94, 1.06, L.N)
    x[L.opg:L.opg + L.G] = rng.uniform(0.0, 1.0, L.G)
    x[L.oqg:L.oqg + L.G] = rng.uniform(-0.5, 0.5, L.G)
    x[L.op:] = rng.uniform(-1.0, 1.0, L.n - L.op)
    y = rng.normal(scale=10.0, size=L.m)
    return x, y


def assert_close(got, ref, mag, what):
    err = np.abs(got - ref)
    lim = RTOL * mag + 1e-300
    bad = np.flatnonzero(err > lim)
    assert bad.size == 0, f"{what}: {bad.size} entries out of tolerance; worst {np.max(err / np.maximum(mag, 1e-300))}"


CASES = ["cfg0", (12, 16, 3, 5), "cfg1"]


@pytest.mark.parametrize("case", CASES + ["cfg2", "cfg3"])
def test_derivatives_match_oracle(case):
    g = grid_for(case)
    g.gs[:] = np.linspace(0, 0.02, g.nbus)  # exercise the shunt terms of the balance rows
    M = opf().Model(g)
    om = OModel(g)
    x, y = random_xy(om, 1)
    w = 0.37
    f = torch.zeros(1, dtype=torch.float64, device="cuda")
    c = torch.zeros(M.m, dtype=torch.float64, device="cuda")
    gr = torch.zeros(M.n, dtype=torch.float64, device="cuda")
    jac = torch.zeros(M.nnzj, dtype=torch.float64, device="cuda")
    hess = torch.zeros(M.nnzh, dtype=torch.float64, device="cuda")
    O = opf()
    M.eval_derivs(O.EVAL_F | O.EVAL_C | O.EVAL_GRAD | O.EVAL_JAC | O.EVAL_HESS, dev(x), dev(y), w, f, c, gr, jac, hess)
    cr, cm = om.constraints(x)
    assert_close(host(c), cr, cm, "constraints")
    grr, grm = om.gradient(x)
    assert_close(host(gr), grr, grm, "gradient")
    fo = om.objective(x)
    assert abs(host(f)[0] - fo) <= 1e-13 * abs(fo)
    jr, jc, hr, hc = M.structure()
    ojr, ojc, ojv, ojm = om.jacobian(x)
    a = canonical(jr, jc, host(jac), np.zeros(len(jr)), shape=(M.m, M.n))
    b = canonical(ojr, ojc, ojv, ojm, shape=(M.m, M.n))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert_close(a[2], b[2], b[3], "jacobian")
    ohr, ohc, ohv, ohm = om.hessian(x, y, w)
    a = canonical(hr, hc, host(hess), np.zeros(len(hr)), shape=(M.n, M.n))
    b = canonical(ohr, ohc, ohv, ohm, shape=(M.n, M.n))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert_close(a[2], b[2], b[3], "hessian")


@pytest.mark.parametrize("case", ["cfg0", (12, 16, 3, 5)])
def test_variable_only_jacobian_keeps_constant_entries(case):
    """OPF_EVAL_JAC_VAR rewrites exactly the entries that depend on x: over a full evaluation at another
    point it reproduces the full evaluation bit for bit, and into a NaN-filled buffer it leaves NaN in
    exactly the 10E + 2G + 1 constant entries (unit flow coefficients, angle rows, generator and arc columns
    of the balance rows, reference row), whose oracle values do not move with x."""
    g = grid_for(case)
    M = opf().Model(g)
    om = OModel(g)
    O = opf()
    x1, _ = random_xy(om, 3)
    x2, _ = random_xy(om, 4)
    full = torch.zeros(M.nnzj, dtype=torch.float64, device="cuda")
    M.eval_derivs(O.EVAL_JAC, dev(x1), jac=full)
    buf = torch.zeros(M.nnzj, dtype=torch.float64, device="cuda")
    M.eval_derivs(O.EVAL_JAC, dev(x2), jac=buf)
    M.eval_derivs(O.EVAL_JAC | O.EVAL_JAC_VAR, dev(x1), jac=buf)
    assert np.array_equal(host(buf).view(np.int64), host(full).view(np.int64))
    nanbuf = torch.full((M.nnzj,), float("nan"), dtype=torch.float64, device="cuda")
    M.eval_derivs(O.EVAL_JAC | O.EVAL_JAC_VAR, dev(x1), jac=nanbuf)
    kept = np.isnan(host(nanbuf))
    assert kept.sum() == 10 * g.nbranch + 2 * g.ngen + 1
    jr, jc, _, _ = M.structure()
    key = jr.astype(np.int64) * M.n + jc
    assert not np.intersect1d(key[kept], key[~kept]).size  # no position mixes constant and variable terms
    a1 = canonical(jr[kept], jc[kept], host(full)[kept], np.zeros(kept.sum()), shape=(M.m, M.n))
    o1 = om.jacobian(x1)
    o2 = om.jacobian(x2)
    b1 = canonical(o1[0], o1[1], o1[2], o1[3], shape=(M.m, M.n))
    b2 = canonical(o2[0], o2[1], o2[2], o2[3], shape=(M.m, M.n))
    pos = {(r, c): k for k, (r, c) in enumerate(zip(b1[0], b1[1]))}
    idx = np.array([pos[(r, c)] for r, c in zip(a1[0], a1[1])])
    assert np.array_equal(b1[2][idx], b2[2][idx])
    assert np.array_equal(a1[2], b1[2][idx])
    with pytest.raises(O.OpfError):
        M.eval_derivs(O.EVAL_JAC_VAR, dev(x1), jac=nanbuf)


def _condensed_inputs(om, M, seed, dw):
    rng = np.random.default_rng(seed)
    x, y = random_xy(om, seed)
    sigx = rng.uniform(0.0, 10.0, M.n)
    D = 10.0 ** rng.uniform(-2, 6, M.m)
    return x, y, sigx, D, dw


@pytest.mark.parametrize("case", CASES + ["cfg2", "cfg3"])
def test_condensed_matrix_and_rhs_match_oracle(case):
    g = grid_for(case)
    M = opf().Model(g)
    om = OModel(g)
    x, y, sigx, D, dw = _condensed_inputs(om, M, 2, 0.25)
    O = opf()
    jac = torch.zeros(M.nnzj, dtype=torch.float64, device="cuda")
    hess = torch.zeros(M.nnzh, dtype=torch.float64, device="cuda")
    M.eval_derivs(O.EVAL_JAC | O.EVAL_HESS, dev(x), dev(y), 1.0, jac=jac, hess=hess)
    kval = torch.zeros(M.nnzk, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(3)
    qx = rng.normal(size=M.n)
    v = rng.normal(size=M.m)
    rhs = torch.zeros(M.n, dtype=torch.float64, device="cuda")
    M.condense(hess, jac, dev(sigx), dev(D), dw, kval, dev(qx), dev(v), rhs)
    cp, ri = M.kkt_pattern()
    ojr, ojc, ojv, ojm = om.jacobian(x)
    ohr, ohc, ohv, ohm = om.hessian(x, y, 1.0)
    kr, kc = okkt.kkt_pattern(M.n, ojr, ojc, ohr, ohc)
    ocp, ori = ochol.lower_csc(M.n, kr, kc)
    assert np.array_equal(cp, ocp) and np.array_equal(ri, ori)
    Jm = okkt.jac_matrix(M.m, M.n, ojr, ojc, ojv)
    Jmag = okkt.jac_matrix(M.m, M.n, ojr, ojc, ojm)
    vals, mags = okkt.condensed_values(M.n, kr, kc, ohr, ohc, ohv, Jm, sigx, D, dw, hmag=ohm, jmag=Jmag)
    assert_close(host(kval), vals, mags, "K")
    ref = qx + Jm.T @ v
    mag = np.abs(qx) + Jmag.T @ np.abs(v)
    assert_close(host(rhs), ref, mag, "rhs")
    # bitwise reproducible (gather assembly, no atomics)
    k2 = torch.zeros_like(kval)
    M.condense(hess, jac, dev(sigx), dev(D), dw, k2)
    assert torch.equal(kval, k2)


def _spd_system(case, seed=4):
    g = grid_for(case)
    M = opf().Model(g)
    om = OModel(g)
    rng = np.random.default_rng(seed)
    x, _ = random_xy(om, seed)
    y = np.zeros(M.m)  # W = obj Hessian >= 0, so K is positive definite
    sigx = rng.uniform(0.1, 10.0, M.n)
    D = 10.0 ** rng.uniform(-1, 4, M.m)
    O = opf()
    jac = torch.zeros(M.nnzj, dtype=torch.float64, device="cuda")
    hess = torch.zeros(M.nnzh, dtype=torch.float64, device="cuda")
    M.eval_derivs(O.EVAL_JAC | O.EVAL_HESS, dev(x), dev(y), 1.0, jac=jac, hess=hess)
    kval = torch.zeros(M.nnzk, dtype=torch.float64, device="cuda")
    M.condense(hess, jac, dev(sigx), dev(D), 0.0, kval)
    return M, kval


@pytest.mark.parametrize("case", CASES + ["cfg2", "cfg3"])
def test_symbolic_analysis_bit_exact(case):
    M, _ = _spd_system(case)
    cp, ri = M.kkt_pattern()
    C = opf().Cholesky(M.n, cp, ri, opf().chol_options(**opts_for(case)))
    sym = ochol.analyze(M.n, cp, ri, ochol.AnalyzeOptions(**opts_for(case)))
    par, cc = C.etree()
    assert np.array_equal(C.perm(), sym.perm)
    assert np.array_equal(par, sym.parent)
    assert np.array_equal(cc, sym.colcount)
    assert np.array_equal(C.supernodes(), sym.snode_ptr)


@pytest.mark.parametrize("case", CASES)
def test_cholesky_factor_matches_oracle(case):
    M, kval = _spd_system(case)
    cp, ri = M.kkt_pattern()
    C = opf().Cholesky(M.n, cp, ri, opf().chol_options(**OPTS))
    assert C.factor(kval) == -1
    lp, li, lx = C.export_factor()
    sym = ochol.analyze(M.n, cp, ri, ochol.AnalyzeOptions(**OPTS))
    oc = ochol.Cholesky(M.n, cp, ri, sym.perm)
    kv = host(kval)
    assert oc.factor(kv) == -1
    olp, oli, olx = oc.export()
    # GPU pattern (supernodal, with explicit zeros) contains the oracle's pattern;
    # entries agree on it and the explicit zeros are exactly zero
    n = M.n
    gpu = {}
    for j in range(n):
        for p in range(lp[j], lp[j + 1]):
            gpu[(int(li[p]), j)] = lx[p]
    ref = {}
    for j in range(n):
        for p in range(olp[j], olp[j + 1]):
            ref[(int(oli[p]), j)] = olx[p]
    assert set(ref) <= set(gpu)
    extra = [gpu[k] for k in gpu if k not in ref]
    assert all(v == 0.0 for v in extra)
    keys = list(ref)
    a = np.array([gpu[k] for k in keys])
    b = np.array([ref[k] for k in keys])
    scale = np.array([abs(ref[(k[1], k[1])]) for k in keys])
    assert np.max(np.abs(a - b) / scale) < 1e-10


@pytest.mark.parametrize("case", CASES + ["cfg2", "cfg3"])
def test_solve_residual(case):
    M, kval = _spd_system(case)
    cp, ri = M.kkt_pattern()
    C = opf().Cholesky(M.n, cp, ri, opf().chol_options(**opts_for(case)))
    assert C.factor(kval) == -1
    rng = np.random.default_rng(7)
    b = rng.normal(size=(2, M.n))
    for r in range(2):
        xr = C.solve(dev(b[r]))
        K = okkt.sym_from_lower(M.n, ri, np.repeat(np.arange(M.n), np.diff(cp)), host(kval))
        res = K @ host(xr) - b[r]
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 1e-10


def test_not_positive_definite_detected():
    M, kval = _spd_system("cfg0")
    cp, ri = M.kkt_pattern()
    C = opf().Cholesky(M.n, cp, ri, opf().chol_options(**OPTS))
    bad = C.factor(-kval)
    assert bad == 0
    sym = ochol.analyze(M.n, cp, ri, ochol.AnalyzeOptions(**OPTS))
    oc = ochol.Cholesky(M.n, cp, ri, sym.perm)
    assert oc.factor(-host(kval)) == 0
    # one bad diagonal entry: both report the same pivot
    kv = host(kval).copy()
    col = np.repeat(np.arange(M.n), np.diff(cp))
    diag = np.flatnonzero(ri == col)
    victim = diag[M.n // 2]
    kv[victim] = -1e3
    b1 = C.factor(dev(kv))
    b2 = oc.factor(kv)
    assert b1 == b2 >= 0


@pytest.mark.parametrize("seed", [1, 2])
def test_ipm_cfg0_matches_oracle(seed):
    g = gridgen.make_grid(30, 41, 6, seed)
    O = opf()
    M = O.Model(g)
    ipm = O.IPM(M, tol=1e-8)
    rc, iters, obj = ipm.solve()
    I = oipm.IPM(OModel(g), oipm.Options(tol=1e-8))
    st = I.solve()
    assert st == oipm.Status.OK
    assert rc == O.OK, O.status_name(rc)
    assert abs(iters - I.iter) <= 2
    assert abs(obj - I.model.objective(I.x)) <= 1e-6 * abs(obj)


@pytest.mark.parametrize("n", [65, 100, 200, 333, 768, 900, 1100, 1300])
def test_dense_front_blocked_cholesky(n):
    """A dense SPD matrix is one supernode: exercises the blocked path (LDS diagonal block, panel solve, MFMA
    update), up to fronts of 1,300 pivots; with pair_min = 512 the fronts of 768 pivots and more pair their
    leading panels (rank-128 trailing updates) while a pair leaves at least 512 rows below it (4, 6, 8 and 12
    paired steps), then go on with single panels."""
    rng = np.random.default_rng(n)
    A = rng.normal(size=(n, n))
    K = A @ A.T + n * np.eye(n)
    rows, cols = np.tril_indices(n)
    cp, ri = ochol.lower_csc(n, rows, cols)
    colidx = np.repeat(np.arange(n), np.diff(cp))
    C = opf().Cholesky(n, cp, ri, opf().chol_options(pair_min=512))
    assert C.nsuper == 1
    assert C.factor(dev(K[ri, colidx])) == -1
    lp, li, lx = C.export_factor()
    perm = C.perm()
    L = np.zeros((n, n))
    for j in range(n):
        L[li[lp[j]:lp[j + 1]], j] = lx[lp[j]:lp[j + 1]]
    Lref = np.linalg.cholesky(K[np.ix_(perm, perm)])
    assert np.max(np.abs(L - Lref)) <= 1e-12 * np.max(np.abs(Lref))


@pytest.mark.parametrize("n,g", [(900, 3), (1300, 4), (1300, 8)])
def test_dense_front_panel_groups(n, g):
    """Panels grouped g at a time (the group's earlier steps update only its next panel, its last step applies
    all g panels to the rest of the front, rank 64 g) give the same factor as the textbook Cholesky."""
    rng = np.random.default_rng(n + g)
    A = rng.normal(size=(n, n))
    K = A @ A.T + n * np.eye(n)
    rows, cols = np.tril_indices(n)
    cp, ri = ochol.lower_csc(n, rows, cols)
    colidx = np.repeat(np.arange(n), np.diff(cp))
    C = opf().Cholesky(n, cp, ri, opf().chol_options(pair_min=384, pair_panels=g))
    assert C.factor(dev(K[ri, colidx])) == -1
    lp, li, lx = C.export_factor()
    perm = C.perm()
    L = np.zeros((n, n))
    for j in range(n):
        L[li[lp[j]:lp[j + 1]], j] = lx[lp[j]:lp[j + 1]]
    Lref = np.linalg.cholesky(K[np.ix_(perm, perm)])
    assert np.max(np.abs(L - Lref)) <= 1e-12 * np.max(np.abs(Lref))


def _block_system(a, b, c, seed):
    """SPD matrix of two cliques (a and b vertices) joined by a separator of c vertices adjacent to both:
    with dense-row detection off, each clique is a front with many pivots and c rows below them."""
    n = a + b + c
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    sep = list(range(a + b, n))
    for blk in (range(0, a), range(a, a + b)):
        idx = np.array(list(blk) + sep, dtype=np.int64)
        if len(idx):
            A[np.ix_(idx, idx)] = rng.uniform(-1.0, 1.0, size=(len(idx), len(idx)))
    A = 0.5 * (A + A.T)
    np.fill_diagonal(A, 0.0)
    np.fill_diagonal(A, np.abs(A).sum(axis=1) + 1.0)
    rows, cols = np.nonzero(np.tril(A))
    cp, ri = ochol.lower_csc(n, rows, cols)
    colidx = np.repeat(np.arange(n), np.diff(cp))
    return A, cp, ri, A[ri, colidx]


@pytest.mark.parametrize("sizes", [(333, 0, 0), (1000, 0, 0), (300, 280, 12), (260, 300, 70), (320, 257, 65),
                                   (800, 790, 100), (1100, 1050, 90)])
def test_wide_front_solves_match_oracle(sizes):
    """Fronts with >= 256 pivots (with and without rows below them) go through the sync-free block
    solves; the solution must match the oracle's factor-and-solve on the same matrix."""
    A, cp, ri, vals = _block_system(*sizes, seed=sum(sizes))
    n = A.shape[0]
    o = dict(OPTS, dense_frac=1.0)
    C = opf().Cholesky(n, cp, ri, opf().chol_options(**o, pair_min=1024 if n > 2000 else 0))
    rp, rows = C.supernode_rows()
    sp = C.supernodes()
    widths = np.diff(sp)
    mrows = np.diff(rp)
    assert widths.max() >= 256
    if sizes[2] > 0:
        assert np.any((widths >= 256) & (mrows > widths))  # a wide front with rows below its pivots
    sym = ochol.analyze(n, cp, ri, ochol.AnalyzeOptions(**o))
    oc = ochol.Cholesky(n, cp, ri, sym.perm)
    assert oc.factor(vals) == -1
    assert C.factor(dev(vals)) == -1
    rng = np.random.default_rng(7)
    for rep in range(3):  # repeated solves reuse the ready flags with new epochs
        b = rng.normal(size=n)
        x = host(C.solve(dev(b)))
        xo = oc.solve(b)
        assert np.max(np.abs(x - xo)) <= 1e-11 * np.max(np.abs(xo)), rep
        assert np.max(np.abs(A @ x - b)) <= 1e-12 * np.max(np.abs(b)) * n


def _oracle_direction(I):
    g = I.grad(I.x)
    Jm = I.jac(I.x)
    c = I.cons(I.x)
    hr, hc, hv = I.hess(I.x, I.y)
    F = I.residuals(I.mu, g, Jm, c)
    d, dw, trials, nir = I.direction(I.mu, hr, hc, hv, Jm, F)
    return d, dw, nir


@pytest.mark.parametrize("case,tol,iters", [("cfg0", 1e-8, 0), ("cfg0", 1e-8, 1), ("cfg0", 1e-8, 6),
                                            ("cfg0", 1e-4, 3), ("cfg1", 1e-4, 0), ("cfg1", 1e-4, 4)])
def test_newton_direction_matches_oracle(case, tol, iters):
    """Same primal-dual state in, same Newton direction out (regularization, condensation, IR)."""
    g = grid_for(case)
    I = oipm.IPM(OModel(g), oipm.Options(tol=tol))
    for _ in range(iters):
        assert I.step() is None
    O = opf()
    M = O.Model(g)
    ipm = O.IPM(M, tol=tol)
    ipm.set_state(I.x, I.s, I.y, I.zl, I.zu, I.vl, I.vu, I.mu, I.dw_last)
    dg, dwg, nirg = ipm.direction()
    do, dwo, niro = _oracle_direction(I)
    assert dwg == dwo
    errs = [np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300) for a, b in zip(dg, do)]
    assert max(errs) <= 1e-6, errs


@pytest.mark.skip(reason="the dependency-driven tile factorization (chol_options.tile_min) did not finish on its "
                         "first device run on this 768-column front; it stays off until the cause is shown")
@pytest.mark.parametrize("n", [768, 1300])
def test_tile_path_dense_front(n):
    rng = np.random.default_rng(n)
    A = rng.normal(size=(n, n))
    K = A @ A.T + n * np.eye(n)
    rows, cols = np.tril_indices(n)
    cp, ri = ochol.lower_csc(n, rows, cols)
    colidx = np.repeat(np.arange(n), np.diff(cp))
    C = opf().Cholesky(n, cp, ri, opf().chol_options(**OPTS, tile_min=768))
    assert C.factor(dev(K[ri, colidx])) == -1
    lp, li, lx = C.export_factor()
    L = np.zeros((n, n))
    for j in range(n):
        L[li[lp[j]:lp[j + 1]], j] = lx[lp[j]:lp[j + 1]]
    Lref = np.linalg.cholesky(K)
    assert np.max(np.abs(L - Lref)) <= 1e-12 * np.max(np.abs(Lref))
