"""Seeded synthetic power grids shaped like the paper's ACOPF workloads.

This module produces *input data only*: bus, branch and generator arrays of a
polar AC optimal power flow instance (the PowerModels/rosetta-opf polar model
the paper solves, Section V-A).  It holds none of the method's arithmetic and
is shared by the CPU oracle and the HIP path as their common input.

The paper measures on pglib-opf ``goc``/``pegase`` cases, which are not
available here; these grids stand in for them with the same structure
(sparse meshed graphs, a generator on a fraction of the buses, a load at every
bus, thermal limits on every branch).

Random numbers come from SplitMix64 (Steele, Lea and Flood, 2014), used as a
counter-based generator: draw ``k`` of stream ``seed`` is
``mix64(seed + (k + 1) * 0x9E3779B97F4A7C15)`` and a uniform on [0, 1) is
``(draw >> 11) * 2**-53``.  Draws are consumed in a fixed order: bus
permutation, tree parents, chord endpoints, per-branch (r, x, b, rate),
generator buses, per-generator (c2, c1, pmax), per-bus Pd.

Generation recipe (per bus count N, branch count E, generator count G):

* topology: a random recursive tree over a random permutation of the buses
  (bus ``pi[i]`` attaches to ``pi[U{0..i-1}]``) plus ``E - (N - 1)`` uniform
  chords with no self loops and no parallel branches;
* branch: r ~ U(0.001, 0.05), x ~ U(0.01, 0.3), charging b ~ U(0, 0.05),
  thermal rating ~ U(0.5, 2.0) (per unit), angle limits +-pi/3;
* generators at G distinct random buses: c2 ~ U(0.01, 0.1), c1 ~ U(10, 40),
  c0 = 0 (cost in $/MWh with a 100 MVA base), Pg in [0, U(0.5, 3)],
  Qg in [-1, 1];
* loads Pd ~ U(0, 0.5), Qd = 0.3 Pd at every bus; 0.94 <= Vm <= 1.06;
  reference angle at bus 0; bus shunts zero.

Feasibility repair.  The raw distributions give less generation capacity than
load at 10k and 80k buses, and the narrow voltage band with reactances up to
0.3 p.u. makes some raw instances infeasible at every size.  Loads are first
scaled by ``min(1, 0.75 * sum(Pmax) / sum(Pd))``; then they are scaled by
further factors of 0.9 until a fast-decoupled AC power flow (generators at
|V| = 1.03 or 1.00 dispatched in proportion to Pmax, slack at the largest
generator) certifies a strictly feasible operating point: load-bus voltages
in [0.945, 1.055], generator Q within 95% of its limits, slack P within
[0, Pmax], angle differences below 0.9 pi/3.  Every rating is then raised to at least
1.1 times the certified apparent flow at either branch end.  The total load
multiplier and the number of raised ratings are recorded in the grid.

At 80,000 buses the fast-decoupled iteration diverges at every load level
(branches with r/x up to 5 break its decoupling assumption), so that grid
takes the lighter DC repair instead (``repair="dc"``): after the first load
scaling, a DC power flow (B theta = P over 1/x susceptances, generators
dispatched in proportion to Pmax, bus 0 as the angle reference) sets every
rating to at least 1.25 * 1.044 * |P_DC| of its branch.  No AC operating point
is certified there.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class SplitMix64:
    """Counter-based SplitMix64 stream; ``uniform(n)`` returns the next n draws in [0, 1)."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.counter = 0

    def raw(self, n: int) -> np.ndarray:
        k = np.arange(self.counter + 1, self.counter + 1 + n, dtype=np.uint64)
        self.counter += n
        with np.errstate(over="ignore"):
            return _mix64(self.seed + k * GOLDEN_GAMMA)

    def uniform(self, n: int) -> np.ndarray:
        return (self.raw(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclasses.dataclass
class Grid:
    """Host structure-of-arrays description of one polar ACOPF instance (per unit, base 100 MVA)."""

    # buses [N]
    pd: np.ndarray
    qd: np.ndarray
    gs: np.ndarray
    bs: np.ndarray
    vmin: np.ndarray
    vmax: np.ndarray
    # branches [E]
    f: np.ndarray  # int32 from-bus
    t: np.ndarray  # int32 to-bus
    r: np.ndarray
    x: np.ndarray
    b: np.ndarray  # total line charging
    rate: np.ndarray
    angmin: np.ndarray
    angmax: np.ndarray
    # generators [G]
    gbus: np.ndarray  # int32
    c2: np.ndarray  # $/(MW^2 h)
    c1: np.ndarray  # $/MWh
    c0: np.ndarray
    pmin: np.ndarray
    pmax: np.ndarray
    qmin: np.ndarray
    qmax: np.ndarray
    ref_bus: int = 0
    base_mva: float = 100.0
    # generation metadata (not model data)
    seed: int = 0
    load_scale: float = 1.0
    repaired_branches: int = 0

    @property
    def nbus(self) -> int:
        return int(self.pd.shape[0])

    @property
    def nbranch(self) -> int:
        return int(self.f.shape[0])

    @property
    def ngen(self) -> int:
        return int(self.gbus.shape[0])

    def dims(self):
        """(n, m) of the polar model with arc-flow variables: n = 2N+2G+4E, m = 2N+1+7E."""
        N, E, G = self.nbus, self.nbranch, self.ngen
        return 2 * N + 2 * G + 4 * E, 2 * N + 1 + 7 * E


# Named workloads: (buses, branches, generators).
CONFIGS = {
    "cfg0": (30, 41, 6),
    "cfg1": (2000, 2700, 300),
    "cfg2": (10000, 13500, 1000),
    "cfg3": (80000, 105000, 6400),
}
DEFAULT_SEED = {"cfg0": 1, "cfg1": 1, "cfg2": 2, "cfg3": 3}


def make_grid(nbus: int, nbranch: int, ngen: int, seed: int, load_factor: float | None = None,
              repair: bool | str = True) -> Grid:
    """Generate one seeded grid.  ``load_factor`` (if given) multiplies every load before repair;
    ``repair`` is True (AC-certified), ``"dc"`` (DC-flow rating repair only) or False."""
    N, E, G = int(nbus), int(nbranch), int(ngen)
    if N < 1 or E < N - 1 or G < 1 or G > N:
        raise ValueError("need N>=1, E>=N-1, 1<=G<=N")
    if E > N * (N - 1) // 2:
        raise ValueError("too many branches for a simple graph")
    rng = SplitMix64(seed)

    # topology: random recursive tree over a random permutation
    perm = np.argsort(rng.uniform(N), kind="stable")
    fr = np.empty(E, dtype=np.int64)
    to = np.empty(E, dtype=np.int64)
    if N > 1:
        u = rng.uniform(N - 1)
        i = np.arange(1, N)
        par = perm[np.floor(u * i).astype(np.int64)]
        fr[: N - 1] = par
        to[: N - 1] = perm[1:]
    edges = set()
    for a, b in zip(fr[: N - 1].tolist(), to[: N - 1].tolist()):
        edges.add((min(a, b), max(a, b)))
    k = N - 1
    while k < E:
        need = E - k
        batch = rng.uniform(2 * max(need, 16))
        ab = np.floor(batch * N).astype(np.int64).reshape(-1, 2)
        for a, b in ab.tolist():
            if a == b:
                continue
            key = (min(a, b), max(a, b))
            if key in edges:
                continue
            edges.add(key)
            fr[k], to[k] = a, b
            k += 1
            if k == E:
                break

    ub = rng.uniform(4 * E).reshape(E, 4)
    r = 0.001 + (0.05 - 0.001) * ub[:, 0]
    x = 0.01 + (0.3 - 0.01) * ub[:, 1]
    bch = 0.05 * ub[:, 2]
    rate = 0.5 + 1.5 * ub[:, 3]

    gbus = np.argsort(rng.uniform(N), kind="stable")[:G]
    ug = rng.uniform(3 * G).reshape(G, 3)
    c2 = 0.01 + 0.09 * ug[:, 0]
    c1 = 10.0 + 30.0 * ug[:, 1]
    pmax = 0.5 + 2.5 * ug[:, 2]

    pd = 0.5 * rng.uniform(N)
    if load_factor is not None:
        pd = pd * float(load_factor)
    lam = 1.0
    nrep = 0
    bs = None
    if repair:
        tot_pd = float(pd.sum())
        if tot_pd > 0:
            lam = min(1.0, 0.75 * float(pmax.sum()) / tot_pd)
        if repair == "dc":
            bs = np.zeros(N)
            rate, nrep = _dc_rating_repair(N, fr, to, x, gbus, pmax, rate, pd * lam)
        else:
            lam_v, bs, rate, nrep = _feasibility_repair(N, fr, to, r, x, bch, gbus, pmax, np.full(G, -1.0),
                                                        np.ones(G), rate, pd * lam)
            lam *= lam_v
        pd = pd * lam
    else:
        bs = np.zeros(N)
    qd = 0.3 * pd

    return Grid(
        pd=pd, qd=qd, gs=np.zeros(N), bs=bs,
        vmin=np.full(N, 0.94), vmax=np.full(N, 1.06),
        f=fr.astype(np.int32), t=to.astype(np.int32), r=r, x=x, b=bch, rate=rate,
        angmin=np.full(E, -math.pi / 3), angmax=np.full(E, math.pi / 3),
        gbus=gbus.astype(np.int32), c2=c2, c1=c1, c0=np.zeros(G),
        pmin=np.zeros(G), pmax=pmax, qmin=np.full(G, -1.0), qmax=np.full(G, 1.0),
        ref_bus=0, base_mva=100.0, seed=int(seed), load_scale=lam, repaired_branches=nrep,
    )


def _cg(A, b):
    """Jacobi-preconditioned CG for the SPD reduced susceptance systems."""
    import scipy.sparse.linalg as spla

    dinv = 1.0 / A.diagonal()
    pre = spla.LinearOperator(A.shape, matvec=lambda v: dinv * v)
    sol, info = spla.cg(A, b, rtol=1e-10, atol=0.0, maxiter=50000, M=pre)
    return sol if info == 0 else None


DIRECT_MAX = 5000  # reduced susceptance systems up to this size are solved by sparse LU, larger ones by CG


def _solver(A):
    """Solve function for repeated right-hand sides with the SPD matrix A (None where it fails)."""
    if A.shape[0] <= DIRECT_MAX:
        import scipy.sparse.linalg as spla

        try:
            lu = spla.splu(A.tocsc())
        except RuntimeError:
            return lambda b: None

        def solve(b):
            x = lu.solve(np.asarray(b, dtype=np.float64))
            return x if np.all(np.isfinite(x)) else None
        return solve
    return lambda b: _cg(A, b)


def _ac_power_flow(N, fr, to, r, x, bch, bs, gbus, pgen_k, pd, qd, vset, max_iter=400):
    """Fast-decoupled AC power flow (Stott & Alsac, 1974) in complex bus-admittance form.

    Generators hold |V| = vset and inject ``pgen_k``; the bus of the largest
    injection is the slack.  ``bs`` are bus shunt susceptances.  Returns the
    complex bus voltages and bus power injections, or None if the iteration
    does not converge.
    """
    import scipy.sparse as sp

    ys = 1.0 / (r + 1j * x)
    ysh = 0.5j * bch
    Y = sp.csr_matrix((np.concatenate([ys + ysh, ys + ysh, -ys, -ys, 1j * bs]),
                       (np.concatenate([fr, to, fr, to, np.arange(N)]),
                        np.concatenate([fr, to, to, fr, np.arange(N)]))), shape=(N, N))
    slack = int(gbus[int(np.argmax(pgen_k))])
    pv = np.zeros(N, dtype=bool)
    pv[gbus] = True
    pq = ~pv
    pgen = np.zeros(N)
    np.add.at(pgen, gbus, pgen_k)
    psp = pgen - pd
    qsp = -qd
    vm = np.ones(N)
    vm[gbus] = vset
    th = np.zeros(N)
    nsl = np.flatnonzero(np.arange(N) != slack)
    ipq = np.flatnonzero(pq)
    bl = 1.0 / x
    Bp = sp.csr_matrix((np.concatenate([bl, bl, -bl, -bl]),
                        (np.concatenate([fr, to, fr, to]), np.concatenate([fr, to, to, fr]))), shape=(N, N))
    Bp = Bp[nsl][:, nsl].tocsr()
    Bpp = (-Y.imag)[ipq][:, ipq].tocsr()
    solve_p = _solver(Bp)
    solve_q = _solver(Bpp) if len(ipq) else None
    for _ in range(max_iter):
        V = vm * np.exp(1j * th)
        S = V * np.conj(Y @ V)
        dP = psp - S.real
        dQ = qsp - S.imag
        mis = max(np.max(np.abs(dP[nsl])), np.max(np.abs(dQ[ipq])) if len(ipq) else 0.0)
        if mis < 1e-9:
            return V, S
        if not np.isfinite(mis) or mis > 1e3 or np.min(vm) < 0.5:
            return None
        dth = solve_p(dP[nsl] / vm[nsl])
        if dth is None:
            return None
        th[nsl] += dth
        if len(ipq):
            V = vm * np.exp(1j * th)
            S = V * np.conj(Y @ V)
            dQ = qsp - S.imag
            dv = solve_q(dQ[ipq] / vm[ipq])
            if dv is None:
                return None
            vm[ipq] += dv
    return None


def _pf_check(N, fr, to, r, x, bch, bs, gbus, pmax, qmin, qmax, pd, lam, loss, isgen):
    """Power flow at load multiplier ``lam`` plus the certificate quantities (None if it diverges).

    The dispatch covers load plus losses; the loss estimate is iterated until
    the slack generator's output is within 2% of Pmax of its share.
    """
    for _ in range(12):
        pgen_k = pmax * ((lam * pd.sum() + loss) / pmax.sum())
        sol = _ac_power_flow(N, fr, to, r, x, bch, bs, gbus, pgen_k, lam * pd, 0.3 * lam * pd, 1.0)
        if sol is None:
            return None
        V, S = sol
        new_loss = float(S.real.sum())
        if abs(new_loss - loss) <= 0.02 * float(np.max(pmax)):
            break
        loss = new_loss
    vm = np.abs(V)
    pbus = S.real + lam * pd
    qbus = S.imag + 0.3 * lam * pd
    pk = np.zeros(N)
    np.add.at(pk, gbus, pgen_k)
    pg = pgen_k * (pbus[gbus] / pk[gbus])
    qhi = np.zeros(N)
    qlo = np.zeros(N)
    np.add.at(qhi, gbus, qmax)
    np.add.at(qlo, gbus, qmin)
    dth = np.abs(np.angle(V[fr]) - np.angle(V[to]))
    vbad = (~isgen) & ((vm < 0.945) | (vm > 1.055))
    qbad = isgen & ((qbus > 0.95 * qhi) | (qbus < 0.95 * qlo))
    hard = np.any(pg < 0.0) or np.any(pg > pmax) or np.any(dth > 0.9 * math.pi / 3)
    return dict(V=V, vm=vm, qbus=qbus, qhi=qhi, qlo=qlo, loss=loss, vbad=vbad, qbad=qbad, hard=hard)


def _dc_rating_repair(N, fr, to, x, gbus, pmax, rate, pd):
    """DC power flow with generation in proportion to Pmax; ratings raised to 1.25 * 1.044 * |P_DC|."""
    import scipy.sparse as sp

    pg = np.zeros(N)
    np.add.at(pg, gbus, pmax * (pd.sum() / pmax.sum()))
    bl = 1.0 / x
    B = sp.csr_matrix((np.concatenate([bl, bl, -bl, -bl]),
                       (np.concatenate([fr, to, fr, to]), np.concatenate([fr, to, to, fr]))), shape=(N, N))
    th = np.zeros(N)
    if N > 1:
        red = B[1:][:, 1:].tocsr()
        sol = _cg(red, (pg - pd)[1:])
        if sol is None:
            raise RuntimeError("DC power flow did not converge")
        th[1:] = sol
    need = 1.25 * 1.044 * np.abs(bl * (th[fr] - th[to]))
    return np.maximum(rate, need), int(np.count_nonzero(need > rate))


def _feasibility_repair(N, fr, to, r, x, bch, gbus, pmax, qmin, qmax, rate, pd):
    """Load scaling plus small reactive compensation until an AC power flow certifies feasibility.

    The certificate is a fast-decoupled power flow with generators at
    |V| = 1.0 dispatched in proportion to Pmax (scaled to load plus losses)
    whose load-bus voltages lie in [0.945, 1.055], generator reactive outputs
    within 95% of their limits, active outputs within [0, Pmax] and angle
    differences below 0.9 pi/3.  Phase 1 scales the loads by 0.9 until the
    flow converges, the active/angle conditions hold and at most 1% of the
    load buses violate their voltage band.  Phase 2 (at most 60 rounds) adds
    bus shunts: a violating load bus i gets ``0.5 (1 - V_i) / (T_ii V_i^2)``
    with ``T_ii = (B''^-1)_ii`` (capped at 0.05 p.u. per round), a generator
    bus beyond 90% of a reactive limit gets a shunt taking over the excess.
    If phase 2 fails the loads are scaled by 0.9 and the shunts cleared.
    Ratings are then raised to 1.1x the certified apparent power at either
    end of each branch.  Returns (load multiplier, shunts, ratings, raised).
    """
    import scipy.sparse as sp

    isgen = np.zeros(N, dtype=bool)
    isgen[gbus] = True
    ipq = np.flatnonzero(~isgen)
    pos = np.full(N, -1)
    pos[ipq] = np.arange(len(ipq))
    lam = 1.0
    for _ in range(80):
        bs = np.zeros(N)
        st = _pf_check(N, fr, to, r, x, bch, bs, gbus, pmax, qmin, qmax, pd, lam, 0.0, isgen)
        if st is None or st["hard"] or st["vbad"].sum() > 0.01 * max(len(ipq), 1):
            lam *= 0.9
            continue
        for _round in range(60):
            if not st["vbad"].any() and not st["qbad"].any():
                V = st["V"]
                ys = 1.0 / (r + 1j * x)
                ysh = 0.5j * bch
                i_ft = (V[fr] - V[to]) * ys + V[fr] * ysh
                i_tf = (V[to] - V[fr]) * ys + V[to] * ysh
                smax = np.maximum(np.abs(V[fr] * np.conj(i_ft)), np.abs(V[to] * np.conj(i_tf)))
                need = 1.1 * smax
                return lam, bs, np.maximum(rate, need), int(np.count_nonzero(need > rate))
            vm, qbus = st["vm"], st["qbus"]
            Y = sp.csr_matrix((np.concatenate([1.0 / (r + 1j * x) + 0.5j * bch, 1.0 / (r + 1j * x) + 0.5j * bch,
                                               -1.0 / (r + 1j * x), -1.0 / (r + 1j * x), 1j * bs]),
                               (np.concatenate([fr, to, fr, to, np.arange(N)]),
                                np.concatenate([fr, to, to, fr, np.arange(N)]))), shape=(N, N))
            Bpp = (-Y.imag)[ipq][:, ipq].tocsr()
            solve_t = _solver(Bpp)
            nb = bs.copy()
            for i in np.flatnonzero(st["vbad"] | ((~isgen) & ((vm < 0.955) | (vm > 1.045)))):
                e = np.zeros(len(ipq))
                e[pos[i]] = 1.0
                t = solve_t(e)
                if t is None or t[pos[i]] <= 0:
                    continue
                nb[i] += float(np.clip(0.5 * (1.0 - vm[i]) / (t[pos[i]] * vm[i] ** 2), -0.05, 0.05))
            hi = isgen & (qbus > 0.9 * st["qhi"])
            lo = isgen & (qbus < 0.9 * st["qlo"])
            nb[hi] += np.minimum((qbus[hi] - 0.9 * st["qhi"][hi]) / vm[hi] ** 2, 0.05)
            nb[lo] += np.maximum((qbus[lo] - 0.9 * st["qlo"][lo]) / vm[lo] ** 2, -0.05)
            nst = _pf_check(N, fr, to, r, x, bch, nb, gbus, pmax, qmin, qmax, pd, lam, st["loss"], isgen)
            if nst is None or nst["hard"]:
                break
            bs, st = nb, nst
        lam *= 0.9
    raise RuntimeError("feasibility repair failed")


def make_config(name: str, seed: int | None = None) -> Grid:
    N, E, G = CONFIGS[name]
    return make_grid(N, E, G, DEFAULT_SEED[name] if seed is None else seed,
                     repair="dc" if name == "cfg3" else True)


def serving_trace(num_requests: int = 512, seed: int = 4):
    """Request list for the batched serving workload: (seed_k, N_k, E_k, G_k, load_factor_k).

    N_k is log-uniform on [30, 2000]; E_k = round(1.35 N_k); G_k = round(0.2 N_k);
    the load factor is U(0.9, 1.1).  Request k uses grid seed 4,000,000 + k.
    """
    rng = SplitMix64(seed)
    u = rng.uniform(2 * num_requests).reshape(num_requests, 2)
    out = []
    for k in range(num_requests):
        nb = int(round(math.exp(math.log(30) + (math.log(2000) - math.log(30)) * u[k, 0])))
        ne = int(math.floor(1.35 * nb + 0.5))
        ng = max(1, int(math.floor(0.2 * nb + 0.5)))
        out.append((4_000_000 + k, nb, ne, ng, 0.9 + 0.2 * u[k, 1]))
    return out
