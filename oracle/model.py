"""Oracle: polar ACOPF model values and hand-derived derivatives (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
HIP path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s CPU-baseline leg may import it; the product path never does.

The model is the paper's ACOPF written as 15 computational patterns (Section
III-B): (1) generation cost, (2) reference angle, (3-6) active/reactive flow
from/to, (7) angle difference, (8-9) apparent-power limits from/to,
(10-11) active/reactive balance with (12-13) generator and (14-15) arc-flow
contributions.  It is the PowerModels polar form with arc-flow variables, with
tap ratio 1, zero phase shift and the line charging split evenly between the
two ends.  Variables, in order: ``[va(N), vm(N), pg(G), qg(G), p(2E), q(2E)]``;
arc ``a < E`` is branch ``a`` oriented from->to, arc ``E + l`` is branch ``l``
oriented to->from.  Constraint rows, in order: reference angle (1), active
flow definitions (2E), reactive flow definitions (2E), angle differences (E),
thermal limits (2E), active balances (N), reactive balances (N); hence
``n = 2N + 2G + 4E`` and ``m = 2N + 1 + 7E``.

The Lagrangian follows the paper's sign convention L = f - y^T g (Section
II-A), so the Hessian returned is ``obj_weight * grad^2 f - sum_i y_i grad^2 c_i``.

Every value is returned with a *magnitude*: the sum of the absolute values of
the product terms that were added to form it.  Rounding differences between
two correct implementations are bounded by a small multiple of
``eps * magnitude``, which is what the parity tolerances are scaled by.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Layout:
    N: int
    E: int
    G: int

    @property
    def n(self):
        return 2 * self.N + 2 * self.G + 4 * self.E

    @property
    def m(self):
        return 2 * self.N + 1 + 7 * self.E

    # variable offsets
    @property
    def ova(self):
        return 0

    @property
    def ovm(self):
        return self.N

    @property
    def opg(self):
        return 2 * self.N

    @property
    def oqg(self):
        return 2 * self.N + self.G

    @property
    def op(self):
        return 2 * self.N + 2 * self.G

    @property
    def oq(self):
        return 2 * self.N + 2 * self.G + 2 * self.E

    # row offsets
    @property
    def rref(self):
        return 0

    @property
    def rp(self):
        return 1

    @property
    def rq(self):
        return 1 + 2 * self.E

    @property
    def rang(self):
        return 1 + 4 * self.E

    @property
    def rth(self):
        return 1 + 5 * self.E

    @property
    def rpb(self):
        return 1 + 7 * self.E

    @property
    def rqb(self):
        return 1 + 7 * self.E + self.N


def _terms(*ts):
    """Sum of product terms and the sum of their absolute values."""
    v = ts[0]
    mg = np.abs(ts[0])
    for t in ts[1:]:
        v = v + t
        mg = mg + np.abs(t)
    return v, mg


class Model:
    """Polar ACOPF instance in the oracle's own representation."""

    def __init__(self, grid):
        self.grid = grid
        N, E, G = grid.nbus, grid.nbranch, grid.ngen
        self.L = Layout(N, E, G)
        L = self.L
        base = float(grid.base_mva)
        f = np.asarray(grid.f, dtype=np.int64)
        t = np.asarray(grid.t, dtype=np.int64)
        # series admittance g + j b = 1 / (r + j x)
        z2 = grid.r ** 2 + grid.x ** 2
        gser = grid.r / z2
        bser = -grid.x / z2
        # arc data: from-end bus i, to-end bus j, branch l
        self.ai = np.concatenate([f, t])
        self.aj = np.concatenate([t, f])
        self.al = np.concatenate([np.arange(E), np.arange(E)])
        self.ag = np.concatenate([gser, gser])
        self.ab = np.concatenate([bser, bser])
        self.abc = np.concatenate([grid.b / 2.0, grid.b / 2.0])  # charging at this end
        self.f, self.t = f, t
        # objective coefficients on per-unit pg (cost data is per MW)
        self.c2 = grid.c2 * base * base
        self.c1 = grid.c1 * base
        self.c0 = grid.c0.copy()
        self.gbus = np.asarray(grid.gbus, dtype=np.int64)
        # bounds
        n, m = L.n, L.m
        xl = np.full(n, -np.inf)
        xu = np.full(n, np.inf)
        xl[L.ovm:L.ovm + N] = grid.vmin
        xu[L.ovm:L.ovm + N] = grid.vmax
        xl[L.opg:L.opg + G] = grid.pmin
        xu[L.opg:L.opg + G] = grid.pmax
        xl[L.oqg:L.oqg + G] = grid.qmin
        xu[L.oqg:L.oqg + G] = grid.qmax
        arate = np.concatenate([grid.rate, grid.rate])
        xl[L.op:L.op + 2 * E] = -arate
        xu[L.op:L.op + 2 * E] = arate
        xl[L.oq:L.oq + 2 * E] = -arate
        xu[L.oq:L.oq + 2 * E] = arate
        gl = np.zeros(m)
        gu = np.zeros(m)
        gl[L.rang:L.rang + E] = grid.angmin
        gu[L.rang:L.rang + E] = grid.angmax
        gl[L.rth:L.rth + 2 * E] = -np.inf
        gu[L.rth:L.rth + 2 * E] = arate ** 2
        self.xl, self.xu, self.gl, self.gu = xl, xu, gl, gu
        self.ref = int(grid.ref_bus)

    # ------------------------------------------------------------------ helpers
    def unpack(self, x):
        L = self.L
        va = x[L.ova:L.ova + L.N]
        vm = x[L.ovm:L.ovm + L.N]
        pg = x[L.opg:L.opg + L.G]
        qg = x[L.oqg:L.oqg + L.G]
        p = x[L.op:L.op + 2 * L.E]
        q = x[L.oq:L.oq + 2 * L.E]
        return va, vm, pg, qg, p, q

    def flat_start(self):
        """va = 0, vm = 1, pg = Pmax/2, qg = 0, arc flows equal to the flow functions at that point."""
        L = self.L
        x = np.zeros(L.n)
        x[L.ovm:L.ovm + L.N] = 1.0
        x[L.opg:L.opg + L.G] = 0.5 * self.grid.pmax
        x[L.oqg:L.oqg + L.G] = 0.0
        phip, _, phiq, _ = self.flows(x)
        x[L.op:L.op + 2 * L.E] = phip
        x[L.oq:L.oq + 2 * L.E] = phiq
        return x

    def _arc_state(self, x):
        va, vm, *_ = self.unpack(x)
        i, j = self.ai, self.aj
        th = va[i] - va[j]
        return vm[i], vm[j], np.cos(th), np.sin(th)

    def flows(self, x):
        """Active/reactive flow functions phi_p, phi_q of every arc, with magnitudes."""
        vi, vj, c, s = self._arc_state(x)
        g, b, bc = self.ag, self.ab, self.abc
        phip = _terms(g * vi * vi, -vi * vj * g * c, -vi * vj * b * s)
        phiq = _terms(-(b + bc) * vi * vi, -vi * vj * g * s, vi * vj * b * c)
        return phip[0], phip[1], phiq[0], phiq[1]

    # ------------------------------------------------------------------ values
    def objective(self, x):
        """f = sum_g c2 pg^2 + c1 pg + c0 (pattern 1)."""
        pg = self.unpack(x)[2]
        v = np.sum(self.c2 * pg * pg + self.c1 * pg + self.c0)
        return v if np.iscomplexobj(v) else float(v)

    def gradient(self, x):
        """Dense gradient of f, with magnitudes."""
        L = self.L
        pg = self.unpack(x)[2]
        g = np.zeros(L.n, dtype=x.dtype)
        gm = np.zeros(L.n)
        v, mg = _terms(2.0 * self.c2 * pg, self.c1)
        g[L.opg:L.opg + L.G] = v
        gm[L.opg:L.opg + L.G] = mg
        return g, gm

    def constraints(self, x):
        """Constraint values c(x) in row order, with magnitudes."""
        L = self.L
        N, E = L.N, L.E
        va, vm, pg, qg, p, q = self.unpack(x)
        c = np.zeros(L.m, dtype=x.dtype)
        cm = np.zeros(L.m)
        c[L.rref] = va[self.ref]
        cm[L.rref] = abs(va[self.ref])
        phip, phipm, phiq, phiqm = self.flows(x)
        c[L.rp:L.rp + 2 * E] = p - phip
        cm[L.rp:L.rp + 2 * E] = np.abs(p) + phipm
        c[L.rq:L.rq + 2 * E] = q - phiq
        cm[L.rq:L.rq + 2 * E] = np.abs(q) + phiqm
        v, mg = _terms(va[self.f], -va[self.t])
        c[L.rang:L.rang + E] = v
        cm[L.rang:L.rang + E] = mg
        v, mg = _terms(p * p, q * q)
        c[L.rth:L.rth + 2 * E] = v
        cm[L.rth:L.rth + 2 * E] = mg
        # balances: arc sums (pattern 14-15) and generator sums (12-13) by explicit scatter
        grid = self.grid
        pb = grid.pd + grid.gs * vm * vm
        pbm = (np.abs(grid.pd) + np.abs(grid.gs * vm * vm)).real
        qb = grid.qd - grid.bs * vm * vm
        qbm = (np.abs(grid.qd) + np.abs(grid.bs * vm * vm)).real
        pb = pb.copy()
        qb = qb.copy()
        np.add.at(pb, self.ai, p)
        np.add.at(pbm, self.ai, np.abs(p))
        np.add.at(qb, self.ai, q)
        np.add.at(qbm, self.ai, np.abs(q))
        np.add.at(pb, self.gbus, -pg)
        np.add.at(pbm, self.gbus, np.abs(pg))
        np.add.at(qb, self.gbus, -qg)
        np.add.at(qbm, self.gbus, np.abs(qg))
        c[L.rpb:L.rpb + N] = pb
        cm[L.rpb:L.rpb + N] = pbm
        c[L.rqb:L.rqb + N] = qb
        cm[L.rqb:L.rqb + N] = qbm
        return c, cm

    # ------------------------------------------------------------------ Jacobian
    def jacobian(self, x):
        """Constraint Jacobian as COO triplets (row, col, val, mag); no duplicate (row, col) pairs."""
        L = self.L
        N, E, G = L.N, L.E, L.G
        va, vm, pg, qg, p, q = self.unpack(x)
        vi, vj, c, s = self._arc_state(x)
        g, b, bc = self.ag, self.ab, self.abc
        i, j = self.ai, self.aj
        A = np.arange(2 * E)
        R, C, V, M = [], [], [], []

        def add(rows, cols, val, mag):
            R.append(np.atleast_1d(rows))
            C.append(np.atleast_1d(cols))
            V.append(np.atleast_1d(val))
            M.append(np.atleast_1d(mag))

        one = np.ones(2 * E)
        # reference angle
        add(L.rref, L.ova + self.ref, 1.0, 1.0)
        # active flow rows: p_a - phi_p
        rp = L.rp + A
        add(rp, L.op + A, one, one)
        # d(-phi_p)/d va_i = -vi vj (g s - b c)
        v, mg = _terms(-vi * vj * g * s, vi * vj * b * c)
        add(rp, L.ova + i, v, mg)
        add(rp, L.ova + j, -v, mg)
        # d(-phi_p)/d vm_i = -(2 g vi - vj (g c + b s))
        v, mg = _terms(-2.0 * g * vi, vj * g * c, vj * b * s)
        add(rp, L.ovm + i, v, mg)
        # d(-phi_p)/d vm_j = vi (g c + b s)
        v, mg = _terms(vi * g * c, vi * b * s)
        add(rp, L.ovm + j, v, mg)
        # reactive flow rows: q_a - phi_q
        rq = L.rq + A
        add(rq, L.oq + A, one, one)
        # phi_q = -(b+bc) vi^2 - vi vj (g s - b c); d phi_q/d va_i = -vi vj (g c + b s)
        v, mg = _terms(vi * vj * g * c, vi * vj * b * s)
        add(rq, L.ova + i, v, mg)
        add(rq, L.ova + j, -v, mg)
        # d(-phi_q)/d vm_i = 2 (b+bc) vi + vj (g s - b c)
        v, mg = _terms(2.0 * (b + bc) * vi, vj * g * s, -vj * b * c)
        add(rq, L.ovm + i, v, mg)
        # d(-phi_q)/d vm_j = vi (g s - b c)
        v, mg = _terms(vi * g * s, -vi * b * c)
        add(rq, L.ovm + j, v, mg)
        # angle differences
        El = np.arange(E)
        add(L.rang + El, L.ova + self.f, np.ones(E), np.ones(E))
        add(L.rang + El, L.ova + self.t, -np.ones(E), np.ones(E))
        # thermal limits
        add(L.rth + A, L.op + A, 2.0 * p, np.abs(2.0 * p))
        add(L.rth + A, L.oq + A, 2.0 * q, np.abs(2.0 * q))
        # balances
        Nb = np.arange(N)
        add(L.rpb + Nb, L.ovm + Nb, 2.0 * self.grid.gs * vm, np.abs(2.0 * self.grid.gs * vm))
        add(L.rqb + Nb, L.ovm + Nb, -2.0 * self.grid.bs * vm, np.abs(2.0 * self.grid.bs * vm))
        add(L.rpb + i, L.op + A, one, one)
        add(L.rqb + i, L.oq + A, one, one)
        Gk = np.arange(G)
        add(L.rpb + self.gbus, L.opg + Gk, -np.ones(G), np.ones(G))
        add(L.rqb + self.gbus, L.oqg + Gk, -np.ones(G), np.ones(G))
        V = [np.broadcast_to(v, r.shape) for v, r in zip(V, R)]
        M = [np.broadcast_to(v, r.shape).real.astype(np.float64) for v, r in zip(M, R)]
        return (np.concatenate(R).astype(np.int64), np.concatenate(C).astype(np.int64),
                np.concatenate(V), np.concatenate(M))

    # ------------------------------------------------------------------ Hessian
    def hessian(self, x, y, obj_weight=1.0):
        """Lower triangle of obj_weight * grad^2 f - sum_i y_i grad^2 c_i as COO (row >= col).

        Entries may repeat (one per contributing constraint); duplicates add.
        """
        L = self.L
        N, E, G = L.N, L.E, L.G
        va, vm, pg, qg, p, q = self.unpack(x)
        vi, vj, c, s = self._arc_state(x)
        g, b, bc = self.ag, self.ab, self.abc
        i, j = self.ai, self.aj
        A = np.arange(2 * E)
        R, C, V, M = [], [], [], []

        def add(r, cc, val, mag):
            r = np.atleast_1d(r)
            cc = np.atleast_1d(cc)
            hi = np.maximum(r, cc)
            lo = np.minimum(r, cc)
            R.append(hi)
            C.append(lo)
            V.append(np.atleast_1d(val))
            M.append(np.atleast_1d(mag))

        # Flow rows c = p_a - phi_p: W gets -y * (-grad^2 phi_p) = +y grad^2 phi_p.
        yp = y[L.rp + A]
        # grad^2 phi_p over (va_i, va_j, vm_i, vm_j), with Cc = g c + b s, S = g s - b c:
        #   (va_i,va_i)=vi vj Cc, (va_i,va_j)=-vi vj Cc, (va_j,va_j)=vi vj Cc
        #   (va_i,vm_i)= vj S, (va_i,vm_j)= vi S, (va_j,vm_i)=-vj S, (va_j,vm_j)=-vi S
        #   (vm_i,vm_i)= 2 g, (vm_i,vm_j)=-Cc, (vm_j,vm_j)=0
        Cc = _terms(g * c, b * s)
        S = _terms(g * s, -b * c)
        self._flow_block(add, yp, vi, vj, Cc, S, two_diag=_terms(2.0 * g), i=i, j=j)
        # Flow rows c = q_a - phi_q: +y grad^2 phi_q with
        #   (va,va) block uses vi vj S, cross terms use -Cc, (vm_i,vm_i) = -2 (b + bc), (vm_i,vm_j) = -S
        yq = y[L.rq + A]
        negC = (-Cc[0], Cc[1])
        negS = (-S[0], S[1])
        self._flow_block(add, yq, vi, vj, S, negC, two_diag=_terms(-2.0 * (b + bc)), i=i, j=j,
                         cross_vm=negS)
        # thermal rows c = p^2 + q^2: -y * 2 on (p_a, p_a) and (q_a, q_a)
        yt = y[L.rth + A]
        add(L.op + A, L.op + A, -2.0 * yt, np.abs(2.0 * yt))
        add(L.oq + A, L.oq + A, -2.0 * yt, np.abs(2.0 * yt))
        # balance rows: -y_P * 2 Gs and +y_Q * 2 Bs on (vm_i, vm_i)
        Nb = np.arange(N)
        ypb = y[L.rpb + Nb]
        yqb = y[L.rqb + Nb]
        v, mg = _terms(-2.0 * ypb * self.grid.gs)
        add(L.ovm + Nb, L.ovm + Nb, v, mg)
        v, mg = _terms(2.0 * yqb * self.grid.bs)
        add(L.ovm + Nb, L.ovm + Nb, v, mg)
        # objective
        Gk = np.arange(G)
        v, mg = _terms(obj_weight * 2.0 * self.c2)
        add(L.opg + Gk, L.opg + Gk, v * np.ones(G), mg * np.ones(G))
        V = [np.broadcast_to(v, r.shape) for v, r in zip(V, R)]
        M = [np.broadcast_to(v, r.shape).real.astype(np.float64) for v, r in zip(M, R)]
        return (np.concatenate(R).astype(np.int64), np.concatenate(C).astype(np.int64),
                np.concatenate(V), np.concatenate(M))

    def _flow_block(self, add, y, vi, vj, Daa, Dav, two_diag, i, j, cross_vm=None):
        """y times the 4x4 second-derivative block of one flow function.

        ``Daa`` gives the angle-angle factor (times vi vj), ``Dav`` the angle-voltage
        factor, ``two_diag`` the (vm_i, vm_i) entry and ``cross_vm`` the (vm_i, vm_j)
        entry (defaults to -Daa).
        """
        L = self.L
        if cross_vm is None:
            cross_vm = (-Daa[0], Daa[1])
        vvi = L.ova + i
        vvj = L.ova + j
        mmi = L.ovm + i
        mmj = L.ovm + j
        ay = np.abs(y)
        vv = vi * vj
        add(vvi, vvi, y * vv * Daa[0], ay * vv * Daa[1])
        add(vvi, vvj, -y * vv * Daa[0], ay * vv * Daa[1])
        add(vvj, vvj, y * vv * Daa[0], ay * vv * Daa[1])
        add(vvi, mmi, y * vj * Dav[0], ay * vj * Dav[1])
        add(vvi, mmj, y * vi * Dav[0], ay * vi * Dav[1])
        add(vvj, mmi, -y * vj * Dav[0], ay * vj * Dav[1])
        add(vvj, mmj, -y * vi * Dav[0], ay * vi * Dav[1])
        add(mmi, mmi, y * two_diag[0], ay * two_diag[1])
        add(mmi, mmj, y * cross_vm[0], ay * cross_vm[1])
        add(mmj, mmj, y * 0.0, ay * 0.0)


def canonical(rows, cols, vals, mags=None, shape=None):
    """Sort COO by (row, col) and sum duplicates; returns (rows, cols, vals, mags)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if mags is None:
        mags = np.abs(vals)
    ncol = int(cols.max()) + 1 if shape is None else int(shape[1])
    key = rows * ncol + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    uniq, start = np.unique(key, return_index=True)
    v = np.add.reduceat(np.asarray(vals)[order], start) if len(order) else np.zeros(0)
    mg = np.add.reduceat(np.asarray(mags)[order], start) if len(order) else np.zeros(0)
    return uniq // ncol, uniq % ncol, v, mg


def dense_from_lower(n, rows, cols, vals):
    """Symmetric dense matrix from lower-triangle COO (duplicates add)."""
    Hd = np.zeros((n, n))
    np.add.at(Hd, (rows, cols), vals)
    off = rows != cols
    np.add.at(Hd, (cols[off], rows[off]), vals[off])
    return Hd


PI3 = math.pi / 3
