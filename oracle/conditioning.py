"""Conditioning of the condensed and augmented Newton systems along an IPM run (oracle side).

TEST INFRASTRUCTURE AND ANALYSIS ONLY.  The paper's stated limitation (Section V-B, known limitations) is
that the condensed matrix K = W + Sigma_x + delta_w I + J^T D J becomes far worse conditioned than the
augmented system it is reduced from as the barrier parameter shrinks, so that the condensed-space method
is reliable only to moderate tolerances.  This module follows the oracle's Algorithm 1 step by step and,
after every iteration, forms

    M_aug = [[W + Sigma_x + delta_w I, 0,                J^T],
             [0,                       Sigma_s + delta_w I, -I],
             [J,                       -I,               0  ]]        (size n + 2m)

and K (the Schur complement of its lower-right block), and reports the 2-norm condition numbers
kappa = max |lambda| / min |lambda| of both (symmetric matrices).  Small systems use dense eigenvalues;
larger ones the extreme eigenvalues from sparse Lanczos (largest magnitude, and smallest magnitude by
shift-invert at 0 through a sparse LU).

    python oracle/conditioning.py cfg0 --tol 1e-8
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import ipm as oipm  # noqa: E402
from oracle import kkt as okkt  # noqa: E402
from oracle.model import Model  # noqa: E402

DENSE_LIMIT = 4000


def systems(I: oipm.IPM, dw: float):
    """(K, M_aug) as scipy sparse matrices at the IPM's current iterate, with regularization dw."""
    n, m = I.n, I.m
    Sx, Ss, _ = I.sigmas()
    hr, hc, hv = I.hess(I.x, I.y)
    W = okkt.sym_from_lower(n, hr, hc, hv).tocsr()
    J = I.jac(I.x).tocsr()
    H = W + sp.diags(Sx + dw)
    D = Ss + dw
    K = (H + J.T @ sp.diags(D) @ J).tocsr()
    Im = sp.identity(m, format="csr")
    Maug = sp.bmat([[H, None, J.T], [None, sp.diags(D), -Im], [J, -Im, None]], format="csr")
    return K, Maug


def kappa(A) -> tuple[float, float, float]:
    """(kappa_2, largest |lambda|, smallest |lambda|) of a symmetric matrix."""
    if A.shape[0] <= DENSE_LIMIT:
        ev = np.abs(np.linalg.eigvalsh(A.toarray()))
        hi, lo = float(ev.max()), float(ev.min())
    else:
        hi = float(abs(spla.eigsh(A, k=1, which="LM", return_eigenvectors=False, tol=1e-6)[0]))
        lo = float(abs(spla.eigsh(A.tocsc(), k=1, sigma=0.0, which="LM", return_eigenvectors=False, tol=1e-6)[0]))
    return (hi / lo if lo > 0 else float("inf")), hi, lo


def inertia(A) -> tuple[int, int, int]:
    """(positive, zero, negative) eigenvalue counts of a small symmetric matrix (dense), zero to 1e-12 relative."""
    ev = np.linalg.eigvalsh(A.toarray())
    t = 1e-12 * np.max(np.abs(ev))
    return int(np.sum(ev > t)), int(np.sum(np.abs(ev) <= t)), int(np.sum(ev < -t))


def trajectory(grid, tol: float, max_iter: int = 500, every: int = 1, log=None):
    """Run the oracle IPM; after every ``every``-th iteration record mu, delta_w and both condition numbers at
    the iterate the step was computed from."""
    I = oipm.IPM(Model(grid), oipm.Options(tol=tol, max_iter=max_iter))
    rows = []
    while True:
        state = (I.x.copy(), I.s.copy(), I.y.copy(), I.zl.copy(), I.zu.copy(), I.vl.copy(), I.vu.copy(),
                 I.dw_last)
        it = I.iter
        st = I.step()
        if st is not None:
            break
        rec = I.log[-1]
        if it % every == 0:
            x, s, y, zl, zu, vl, vu, dwl = state
            saved = (I.x, I.s, I.y, I.zl, I.zu, I.vl, I.vu)
            I.x, I.s, I.y, I.zl, I.zu, I.vl, I.vu = x, s, y, zl, zu, vl, vu
            K, Maug = systems(I, rec["dw"])
            kK = kappa(K)
            kM = kappa(Maug)
            I.x, I.s, I.y, I.zl, I.zu, I.vl, I.vu = saved
            row = {"iter": it, "mu": rec["mu"], "dw": rec["dw"], "E0": rec["E0"], "kappa_K": kK[0],
                   "kappa_Maug": kM[0]}
            rows.append(row)
            if log:
                log(row)
    return I, st, rows


def main():
    from paper_2307_16830_amd import gridgen
    ap = argparse.ArgumentParser()
    ap.add_argument("config")
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--every", type=int, default=1)
    ap.add_argument("--max-iter", type=int, default=500)
    a = ap.parse_args()
    grid = gridgen.make_config(a.config)

    def log(r):
        print(f"{r['iter']:4d} mu={r['mu']:.1e} dw={r['dw']:.1e} E0={r['E0']:.2e} "
              f"kappa(K)={r['kappa_K']:.3e} kappa(M_aug)={r['kappa_Maug']:.3e}", flush=True)

    I, st, rows = trajectory(grid, a.tol, a.max_iter, a.every, log)
    print(f"status {st} after {I.iter} iterations, final E0 {I.log[-1]['E0']:.3e}")


if __name__ == "__main__":
    main()
