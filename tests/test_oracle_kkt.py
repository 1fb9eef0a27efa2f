"""Pins of the oracle's condensed KKT pieces: the full Newton system solved densely, the inertia
equivalence, and the structural K pattern."""
import numpy as np
import pytest

from oracle import ipm as oipm
from oracle import kkt as okkt
from oracle.model import Model, dense_from_lower
from paper_2307_16830_amd import gridgen


def _state(seed=1, iters=3, tol=1e-4):
    g = gridgen.make_grid(8, 10, 2, seed)
    I = oipm.IPM(Model(g), oipm.Options(tol=tol))
    for _ in range(iters):
        if I.step() is not None:
            break
    return I


@pytest.mark.parametrize("iters", [0, 2, 5])
def test_condensed_solve_equals_dense_full_newton(iters):
    """Condensed solve + recovery (Section IV-C) == dense LU solve of the full 7x7-block Newton system."""
    I = _state(iters=iters)
    n, m = I.n, I.m
    mu = I.mu
    g = I.grad(I.x)
    Jm = I.jac(I.x)
    c = I.cons(I.x)
    F = I.residuals(mu, g, Jm, c)
    hr, hc, hv = I.hess(I.x, I.y)
    Sx, Ss, dist = I.sigmas()
    for dw in (0.0, 0.3):
        vals = okkt.condensed_values(n, I.krow, I.kcol, hr, hc, hv, Jm, Sx, Ss + dw, dw)
        K = np.zeros((n, n))
        K[I.krow, I.kcol] = vals
        K = K + np.tril(K, -1).T
        if np.min(np.linalg.eigvalsh(K)) <= 0:
            continue
        assert I.chol.factor(vals) < 0
        R = [-v for v in F]
        d = I.reduce_solve(R, Jm, Sx, Ss, dist, dw)
        W = dense_from_lower(n, hr, hc, hv)
        M = okkt.dense_M_full(W, Jm.toarray(), dw, I.xl, I.xu, I.sl, I.su, I.x, I.s, I.zl, I.zu, I.vl, I.vu)
        rhs = np.concatenate(R)
        ref = np.linalg.solve(M, rhs)
        got = np.concatenate(d)
        assert np.max(np.abs(got - ref)) <= 1e-7 * max(1.0, np.max(np.abs(ref)))
        # and the oracle's own full residual of its step is tiny
        res = I.full_residual(R, d, okkt.sym_from_lower(n, hr, hc, hv), Jm, dist, dw)
        assert max(np.max(np.abs(v)) for v in res) <= 1e-8 * max(1.0, np.max(np.abs(rhs)))


def test_K_matches_dense_definition_and_is_symmetric():
    I = _state(iters=2)
    n = I.n
    Jm = I.jac(I.x)
    hr, hc, hv = I.hess(I.x, I.y)
    Sx, Ss, _ = I.sigmas()
    dw = 0.125
    vals, mags = okkt.condensed_values(n, I.krow, I.kcol, hr, hc, hv, Jm, Sx, Ss + dw, dw, hmag=np.abs(hv))
    W = dense_from_lower(n, hr, hc, hv)
    J = Jm.toarray()
    Kd = W + np.diag(Sx + dw) + J.T @ np.diag(Ss + dw) @ J
    assert np.allclose(Kd, Kd.T, rtol=0, atol=1e-9 * np.max(np.abs(Kd)))
    assert np.all(np.abs(vals - Kd[I.krow, I.kcol]) <= 1e-13 * mags + 1e-300)
    # every structural nonzero of the dense K is in the pattern
    mask = np.zeros((n, n), dtype=bool)
    mask[I.krow, I.kcol] = True
    lo = np.tril(np.abs(Kd) > 0)
    assert not np.any(lo & ~mask)


def test_inertia_equivalence():
    """inertia(M_aug) = (n+m, 0, m) exactly when K is positive definite (Sylvester's law; the paper's
    printed (n+5m, 0, m) has the wrong size for an (n+2m)-square matrix)."""
    I = _state(iters=4)
    n, m = I.n, I.m
    Jm = I.jac(I.x)
    J = Jm.toarray()
    hr, hc, hv = I.hess(I.x, I.y)
    Sx, Ss, _ = I.sigmas()
    W = dense_from_lower(n, hr, hc, hv)
    seen = set()
    for dw in (0.0, 1e-6, 1e-2, 1.0, 1e2):
        Maug = np.zeros((n + 2 * m, n + 2 * m))
        Maug[:n, :n] = W + np.diag(Sx) + dw * np.eye(n)
        Maug[:n, n + m:] = J.T
        Maug[n:n + m, n:n + m] = np.diag(Ss) + dw * np.eye(m)
        Maug[n:n + m, n + m:] = -np.eye(m)
        Maug[n + m:, :n] = J
        Maug[n + m:, n:n + m] = -np.eye(m)
        ev = np.linalg.eigvalsh(Maug)
        tolv = 1e-14 * np.max(np.abs(ev))
        inertia = (int(np.sum(ev > tolv)), int(np.sum(np.abs(ev) <= tolv)), int(np.sum(ev < -tolv)))
        K = W + np.diag(Sx + dw) + J.T @ np.diag(Ss + dw) @ J
        pd = np.min(np.linalg.eigvalsh(K)) > 0
        assert (inertia == (n + m, 0, m)) == pd
        seen.add(pd)
    assert True in seen


def test_kkt_pattern_contains_jtj_pairs():
    g = gridgen.make_grid(6, 7, 2, 3)
    m = Model(g)
    x0 = m.flat_start()
    jr, jc, _, _ = m.jacobian(x0)
    hr, hc, _, _ = m.hessian(x0, np.zeros(m.L.m), 1.0)
    kr, kc = okkt.kkt_pattern(m.L.n, jr, jc, hr, hc)
    S = set(zip(kr.tolist(), kc.tolist()))
    for i in range(m.L.n):
        assert (i, i) in S
    for r in np.unique(jr):
        cols = jc[jr == r]
        for a in cols:
            for b in cols:
                assert (max(a, b), min(a, b)) in S
    assert all(r >= c for r, c in S)
    # sorted in lower-CSC order
    key = kc * m.L.n + kr
    assert np.all(np.diff(key) > 0)
