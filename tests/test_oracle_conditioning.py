"""Pins of the conditioning study (oracle/conditioning.py): the paper's known limitation that the condensed
matrix K ends up worse conditioned than the augmented system it is reduced from (Section V-B), the inertia
equivalence at every unregularized iterate (Section IV-C), and the sparse extreme-eigenvalue path against
dense eigenvalues."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import conditioning as cond
from paper_2307_16830_amd import gridgen


@pytest.mark.parametrize("seed", [1, 2])
def test_condensed_matrix_ends_worse_conditioned(seed):
    """At the solution of a 30-bus grid K is worse conditioned than M_aug (at tol 1e-4, where both are well
    inside FP64's range), and K's conditioning grows with the inverse tolerance: the equality rows' slack
    bounds are +-tol, so Sigma_s and with it the largest eigenvalue of J^T D J scale like 1/tol."""
    from oracle import ipm as oipm
    from oracle.model import Model
    grid = gridgen.make_grid(30, 41, 6, seed)
    kap = {}
    for tol in (1e-4, 1e-6):
        I = oipm.IPM(Model(grid), oipm.Options(tol=tol))
        assert I.solve() == 0
        K, Maug = cond.systems(I, 0.0)
        kap[tol] = (cond.kappa(K)[0], cond.kappa(Maug)[0])
    assert kap[1e-4][0] > kap[1e-4][1]
    assert kap[1e-6][0] > kap[1e-6][1]
    assert kap[1e-6][0] > 30 * kap[1e-4][0]


def test_augmented_inertia_at_unregularized_iterates():
    grid = gridgen.make_config("cfg0")
    from oracle import ipm as oipm
    from oracle.model import Model
    I = oipm.IPM(Model(grid), oipm.Options(tol=1e-4))
    checked = 0
    while checked < 3 and I.step() is None:
        if I.log[-1]["dw"] == 0.0:
            # the step just taken factored K(0) successfully: M_aug at the new point with dw = 0 is checked only
            # when K is positive definite there
            K, Maug = cond.systems(I, 0.0)
            if np.all(np.linalg.eigvalsh(K.toarray()) > 0):
                assert cond.inertia(Maug) == (I.n + I.m, 0, I.m)
                checked += 1
    assert checked >= 3


def test_sparse_extreme_eigenvalues_match_dense():
    rng = np.random.default_rng(3)
    n = 300
    A = sp.random(n, n, density=0.02, random_state=4)
    A = (A + A.T + sp.diags(rng.uniform(0.1, 10.0, n))).tocsr()
    A = A - sp.diags(np.full(n, 0.05))
    dense = cond.kappa(A)
    old = cond.DENSE_LIMIT
    try:
        cond.DENSE_LIMIT = 10
        sparse = cond.kappa(A)
    finally:
        cond.DENSE_LIMIT = old
    assert sparse[1] == pytest.approx(dense[1], rel=1e-5)
    assert sparse[2] == pytest.approx(dense[2], rel=1e-5)
