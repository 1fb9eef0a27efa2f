"""Pins of the oracle's model and derivatives against closed forms, textbook special cases and complex-step."""
import numpy as np
import pytest

from oracle.model import Model, canonical, dense_from_lower
from paper_2307_16830_amd import gridgen
from tests._grids import grid_from, random_point



def small_grid(seed=1):
    return gridgen.make_grid(30, 41, 6, seed)


def test_sizes_match_formulation():
    # n = 2N + 2G + 4E and m = 2N + 1 + 7E; the 10k-bus config matches the paper's 10000_goc row
    # shape (76.8k variables, 112.4k constraints, Table II) to within a few percent.
    m = Model(small_grid())
    assert (m.L.n, m.L.m) == (236, 348)
    N, E, G = gridgen.CONFIGS["cfg2"]
    n, mm = 2 * N + 2 * G + 4 * E, 2 * N + 1 + 7 * E
    assert (n, mm) == (76000, 114501)
    assert abs(n / 76.8e3 - 1) < 0.02 and abs(mm / 112.4e3 - 1) < 0.03


def test_flat_start_special_cases():
    """At va = 0, vm = 1: p_a = 0, q_a = -b_c/2 and d p_a / d va_i = x / (r^2 + x^2) (DC power flow)."""
    g = small_grid()
    m = Model(g)
    x0 = m.flat_start()
    phip, _, phiq, _ = m.flows(x0)
    E = g.nbranch
    assert np.allclose(phip, 0.0, atol=1e-15)
    assert np.allclose(phiq, -np.concatenate([g.b, g.b]) / 2, atol=1e-15)
    jr, jc, jv, _ = m.jacobian(x0)
    L = m.L
    # row of active flow on arc a (a < E, from f to t): entry at va_f equals -d phi_p / d va_f = -x/(r^2+x^2)
    for a in range(E):
        row = L.rp + a
        sel = (jr == row) & (jc == L.ova + g.f[a])
        assert sel.sum() == 1
        assert jv[sel][0] == pytest.approx(-g.x[a] / (g.r[a] ** 2 + g.x[a] ** 2), rel=1e-14)


def test_lossless_and_loss_identities():
    rng = np.random.default_rng(0)
    g = small_grid()
    g.r[:] = 0.0
    g.b[:] = 0.0
    m = Model(g)
    x = random_point(m, rng)
    phip, _, phiq, _ = m.flows(x)
    E = g.nbranch
    assert np.allclose(phip[:E] + phip[E:], 0.0, atol=1e-13)
    # with resistance: p_fr + p_to = g (vi^2 + vj^2 - 2 vi vj cos th) >= 0
    g2 = small_grid()
    g2.b[:] = 0.0
    m2 = Model(g2)
    x = random_point(m2, rng)
    phip, _, _, _ = m2.flows(x)
    va, vm = x[:g2.nbus], x[g2.nbus:2 * g2.nbus]
    f, t = g2.f, g2.t
    gs = g2.r / (g2.r ** 2 + g2.x ** 2)
    loss = gs * (vm[f] ** 2 + vm[t] ** 2 - 2 * vm[f] * vm[t] * np.cos(va[f] - va[t]))
    assert np.allclose(phip[:E] + phip[E:], loss, rtol=1e-12, atol=1e-14)
    assert np.all(loss >= 0)


def _dense_jac(m, x):
    jr, jc, jv, _ = m.jacobian(x)
    J = np.zeros((m.L.m, m.L.n), dtype=np.result_type(jv, float))
    np.add.at(J, (jr, jc), jv)
    return J


@pytest.mark.parametrize("seed", [1, 2])
def test_jacobian_complex_step(seed):
    """Every Jacobian entry equals the complex-step derivative of c(x) (exact to ~1e-15)."""
    g = gridgen.make_grid(12, 16, 3, seed)
    g.gs[:] = np.linspace(0.0, 0.05, g.nbus)
    g.bs[:] = np.linspace(-0.05, 0.05, g.nbus)
    m = Model(g)
    rng = np.random.default_rng(seed)
    x = random_point(m, rng)
    J = _dense_jac(m, x)
    h = 1e-30
    Jcs = np.zeros_like(J)
    for k in range(m.L.n):
        xc = x.astype(complex)
        xc[k] += 1j * h
        c, _ = m.constraints(xc)
        Jcs[:, k] = c.imag / h
    scale = np.maximum(1.0, np.abs(J))
    assert np.max(np.abs(J - Jcs) / scale) < 1e-13
    # the COO pattern has no duplicates
    jr, jc, _, _ = m.jacobian(x)
    assert len(np.unique(jr * m.L.n + jc)) == len(jr)


@pytest.mark.parametrize("seed", [1, 3])
def test_hessian_complex_step(seed):
    """Lagrangian Hessian (lower, duplicates added) equals the complex-step derivative of grad L = w grad f - J^T y."""
    g = gridgen.make_grid(10, 13, 3, seed)
    g.gs[:] = 0.03
    g.bs[:] = -0.02
    m = Model(g)
    rng = np.random.default_rng(seed)
    x = random_point(m, rng)
    y = rng.normal(size=m.L.m)
    w = 0.37
    hr, hc, hv, _ = m.hessian(x, y, w)
    assert np.all(hr >= hc)
    H = dense_from_lower(m.L.n, hr, hc, hv)
    h = 1e-30
    Hcs = np.zeros((m.L.n, m.L.n))
    for k in range(m.L.n):
        xc = x.astype(complex)
        xc[k] += 1j * h
        gr, _ = m.gradient(xc)
        J = _dense_jac(m, xc)
        gl = w * gr - J.T @ y
        Hcs[:, k] = gl.imag / h
    assert np.allclose(H, H.T)
    assert np.max(np.abs(H - Hcs) / np.maximum(1.0, np.abs(H))) < 1e-12


def test_gradient_and_objective_central_difference():
    g = small_grid()
    m = Model(g)
    x = random_point(m, np.random.default_rng(5))
    gr, _ = m.gradient(x)
    for k in range(m.L.opg, m.L.opg + m.L.G):
        e = np.zeros(m.L.n)
        h = 1e-4
        e[k] = h
        fd = (m.objective(x + e) - m.objective(x - e)) / (2 * h)  # exact for a quadratic
        assert fd == pytest.approx(gr[k], rel=1e-9)
    assert np.count_nonzero(gr) == m.L.G


def test_magnitude_bounds_value():
    g = small_grid()
    m = Model(g)
    x = random_point(m, np.random.default_rng(7))
    c, cm = m.constraints(x)
    assert np.all(np.abs(c) <= cm * (1 + 1e-15) + 1e-300)
    jr, jc, jv, jm = m.jacobian(x)
    assert np.all(np.abs(jv) <= jm * (1 + 1e-15))
    hr, hc, hv, hm = m.hessian(x, np.random.default_rng(1).normal(size=m.L.m), 1.0)
    assert np.all(np.abs(hv) <= hm * (1 + 1e-15) + 1e-300)


def test_balance_rows_closed_form():
    """Two buses, one branch: balance rows equal the flow sums minus generation plus load and shunt terms."""
    g = grid_from(2, [(0, 1, 0.01, 0.1, 0.02, 2.0)], [(0, 0.02, 20.0, 0.0, 3.0, -1.0, 1.0)], pd=[0.0, 0.8],
                  gs=[0.01, 0.02], bs=[0.03, -0.01])
    m = Model(g)
    x = random_point(m, np.random.default_rng(3))
    c, _ = m.constraints(x)
    L = m.L
    va, vm, pg, qg, p, q = m.unpack(x)
    assert c[L.rpb + 0] == pytest.approx(p[0] - pg[0] + 0.0 + 0.01 * vm[0] ** 2, rel=1e-14, abs=1e-15)
    assert c[L.rpb + 1] == pytest.approx(p[1] + 0.8 + 0.02 * vm[1] ** 2, rel=1e-14)
    assert c[L.rqb + 0] == pytest.approx(q[0] - qg[0] + 0.24 * 0 - 0.03 * vm[0] ** 2, rel=1e-14, abs=1e-15)
    assert c[L.rqb + 1] == pytest.approx(q[1] + 0.24 - (-0.01) * vm[1] ** 2, rel=1e-14)


def test_canonical_sums_duplicates():
    r, c, v, mg = canonical([1, 0, 1, 1], [0, 0, 0, 1], [1.0, 2.0, 3.0, -4.0], [1.0, 2.0, 3.0, 4.0], shape=(2, 2))
    assert list(r) == [0, 1, 1] and list(c) == [0, 0, 1]
    assert list(v) == [2.0, 4.0, -4.0] and list(mg) == [2.0, 4.0, 4.0]
