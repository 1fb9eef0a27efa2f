"""Pins of the oracle IPM: closed-form optima of special cases and an independent KKT check at the
30-bus solution (E0 <= 1e-8)."""
import numpy as np
import pytest

from oracle import ipm as oipm
from oracle.model import Model
from paper_2307_16830_amd import gridgen
from tests._grids import grid_from


def economic_dispatch(c2, c1, pmin, pmax, demand):
    """Equal-marginal-cost dispatch: 2 c2 p + c1 = lam clipped to [pmin, pmax], sum p = demand (bisection)."""
    lo, hi = -1e7, 1e7
    for _ in range(200):
        lam = 0.5 * (lo + hi)
        p = np.clip((lam - c1) / (2 * c2), pmin, pmax)
        if p.sum() < demand:
            lo = lam
        else:
            hi = lam
    return np.clip((lam - c1) / (2 * c2), pmin, pmax)


@pytest.mark.parametrize("demand", [0.8, 2.9])
def test_single_bus_economic_dispatch(demand):
    gens = [(0, 0.02, 20.0, 0.0, 1.5, -1.0, 1.0), (0, 0.05, 15.0, 0.0, 1.0, -1.0, 1.0),
            (0, 0.01, 35.0, 0.2, 2.0, -1.0, 1.0)]
    g = grid_from(1, [], gens, pd=[demand])
    I = oipm.IPM(Model(g), oipm.Options(tol=1e-8))
    st = I.solve()
    assert st == oipm.Status.OK
    base = 100.0
    c2 = np.array([x[1] for x in gens]) * base ** 2
    c1 = np.array([x[2] for x in gens]) * base
    p = economic_dispatch(c2, c1, np.array([x[3] for x in gens]), np.array([x[4] for x in gens]), demand)
    ref = float(np.sum(c2 * p * p + c1 * p))
    got = I.model.objective(I.x)
    assert got == pytest.approx(ref, rel=1e-6)
    pg = I.x[I.model.L.opg:I.model.L.opg + 3]
    assert np.allclose(pg, p, atol=1e-5)


def test_two_bus_lossless_closed_form():
    """r = 0, no charging: all load is served over the line, so pg = Pd and f = c2 Pd^2 + c1 Pd."""
    g = grid_from(2, [(0, 1, 0.0, 0.1, 0.0, 5.0)], [(0, 0.03, 25.0, 0.0, 3.0, -2.0, 2.0)], pd=[0.0, 1.2])
    I = oipm.IPM(Model(g), oipm.Options(tol=1e-8))
    assert I.solve() == oipm.Status.OK
    ref = 0.03 * 1e4 * 1.2 ** 2 + 25.0 * 100 * 1.2
    assert I.model.objective(I.x) == pytest.approx(ref, rel=1e-6)


def test_cfg0_reaches_1e8_and_kkt_holds_independently():
    g = gridgen.make_config("cfg0")
    m = Model(g)
    I = oipm.IPM(m, oipm.Options(tol=1e-8))
    st = I.solve()
    assert st == oipm.Status.OK
    assert I.log[-1]["E0"] <= 1e-8
    x = I.x
    # primal feasibility of the relaxed problem, recomputed from the model (unscaled)
    c, _ = m.constraints(x)
    eq = m.gl == m.gu
    assert np.max(np.abs(c[eq])) <= 3e-8 / np.min(I.sc[eq])
    assert np.all(c[~eq] >= m.gl[~eq] - 1e-7) and np.all(c[~eq] <= m.gu[~eq] + 1e-7)
    assert np.all(x >= m.xl - 1e-7) and np.all(x <= m.xu + 1e-7)
    # stationarity of the scaled Lagrangian with the returned multipliers
    jr, jc, jv, _ = m.jacobian(x)
    gr, _ = m.gradient(x)
    Jty = np.zeros(m.L.n)
    np.add.at(Jty, jc, I.sc[jr] * jv * I.y[jr])
    r = I.sf * gr - Jty - I.zl + I.zu
    assert np.max(np.abs(r)) <= 1e-8 * max(1.0, np.max(np.abs(I.y)) / 100)
    # the objective is below the unrelaxed flat-start cost and positive
    assert 0 < m.objective(x) < m.objective(m.flat_start()) * 2


@pytest.mark.parametrize("seed", [0, 2, 4, 9])
def test_other_cfg0_seeds_converge(seed):
    g = gridgen.make_grid(30, 41, 6, seed)
    I = oipm.IPM(Model(g), oipm.Options(tol=1e-8))
    assert I.solve() == oipm.Status.OK
    assert I.iter < 100
