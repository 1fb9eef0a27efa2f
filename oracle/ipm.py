"""Oracle: condensed-space interior-point method (Algorithm 1 of the paper), FP64 CPU.

TEST INFRASTRUCTURE ONLY.

The method follows Section IV of the paper: inequality relaxation of every
constraint row into ``c(x) - s = 0`` with slack bounds (equality rows get
``[-eps_tol, +eps_tol]``, Section IV-A), the log-barrier subproblem (IV-B),
Newton steps on its first-order conditions computed through the condensed
positive-definite system (IV-C), inertia correction by a primal
regularization that restores positive definiteness, iterative refinement on
the full system, a filter line search (IV-D) and the scaled convergence test.
The paper defers the line-search, scaling and barrier-update details to
Waechter & Biegler (2006); the constants and rules used here are those of that
reference, fixed in :class:`Options` and restated in the project's design
notes.  The HIP implementation follows the same steps.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

from . import chol as ochol
from . import kkt as okkt
from .model import Model

EPS_MACH = 2.220446049250313e-16


@dataclasses.dataclass
class Options:
    tol: float = 1e-4              # eps_tol: termination and equality-row relaxation
    max_iter: int = 500
    mu_init: float = 0.1
    kappa_eps: float = 10.0
    kappa_mu: float = 0.2
    theta_mu: float = 1.5
    tau_min: float = 0.99
    bound_push: float = 1e-2       # kappa_1
    bound_frac: float = 1e-2       # kappa_2
    bound_relax: float = 1e-8      # relaxation of variable bounds and inequality rows
    s_max: float = 100.0
    kappa_sigma: float = 1e10
    grad_max: float = 100.0        # gradient-based scaling target
    # filter line search
    gamma_theta: float = 1e-5
    gamma_phi: float = 1e-8
    delta: float = 1.0
    s_theta: float = 1.1
    s_phi: float = 2.3
    eta_phi: float = 1e-4
    gamma_alpha: float = 0.05
    # inertia correction
    dw_first: float = 1e-4
    dw_min: float = 1e-20
    dw_max: float = 1e40
    kappa_w_minus: float = 1.0 / 3.0
    kappa_w_plus_first: float = 100.0
    kappa_w_plus: float = 8.0
    # iterative refinement on the full system
    max_ir: int = 10
    ir_tol: float = 1e-10
    ir_stall: float = 0.9
    # a pivot counts as positive only above pivot_tol * |K_jj|: at that size its sign is within
    # rounding noise of the condensed matrix, so regularization is applied instead
    pivot_tol: float = 1e-12
    # second-order correction of a rejected first trial step (filter line search extension); off by default
    soc: bool = False
    soc_max: int = 4               # p_max: corrections per iteration
    kappa_soc: float = 0.99        # a correction must reduce the infeasibility by this factor to continue


class Status:
    OK = 0
    MAXITER = -6
    LINESEARCH = -7
    NUMERIC = -8
    REGULARIZATION = -5


def _relax(b, factor, sign):
    out = b.copy()
    fin = np.isfinite(b)
    out[fin] = b[fin] + sign * factor * np.maximum(1.0, np.abs(b[fin]))
    return out


class IPM:
    """State and steps of the condensed-space IPM on one model instance."""

    def __init__(self, model: Model, opts: Options | None = None, analyze_opts: ochol.AnalyzeOptions | None = None):
        self.model = model
        self.o = opts or Options()
        o = self.o
        L = model.L
        self.n, self.m = L.n, L.m
        n, m = self.n, self.m
        # ---- structure (fixed): Jacobian and Hessian COO patterns, K pattern, ordering
        x0 = model.flat_start()
        jr, jc, jv, _ = model.jacobian(x0)
        hr, hc, _, _ = model.hessian(x0, np.zeros(m), 1.0)
        self.jrow, self.jcol = jr, jc
        self.hrow, self.hcol = hr, hc
        kr, kc = okkt.kkt_pattern(n, jr, jc, hr, hc)
        self.krow, self.kcol = kr, kc  # sorted by (col, row): lower CSC order
        self.kcolptr, self.krowind = ochol.lower_csc(n, kr, kc)
        self.sym = ochol.analyze(n, self.kcolptr, self.krowind, analyze_opts)
        self.chol = ochol.Cholesky(n, self.kcolptr, self.krowind, self.sym.perm)
        # ---- gradient-based scaling at the user starting point
        g0, _ = model.gradient(x0)
        self.sf = min(1.0, o.grad_max / max(np.max(np.abs(g0)), 1e-300)) if np.any(g0) else 1.0
        rowmax = np.zeros(m)
        np.maximum.at(rowmax, jr, np.abs(jv))
        self.sc = np.where(rowmax > 0, np.minimum(1.0, o.grad_max / np.where(rowmax > 0, rowmax, 1.0)), 1.0)
        # ---- bounds of the relaxed, scaled problem
        self.xl = _relax(model.xl, o.bound_relax, -1.0)
        self.xu = _relax(model.xu, o.bound_relax, +1.0)
        gl = self.sc * model.gl
        gu = self.sc * model.gu
        eq = model.gl == model.gu
        sl = _relax(gl, o.bound_relax, -1.0)
        su = _relax(gu, o.bound_relax, +1.0)
        sl[eq] = gl[eq] - o.tol
        su[eq] = gu[eq] + o.tol
        self.sl, self.su = sl, su
        self.fxl = np.isfinite(self.xl)
        self.fxu = np.isfinite(self.xu)
        self.fsl = np.isfinite(self.sl)
        self.fsu = np.isfinite(self.su)
        self.nbounds = int(self.fxl.sum() + self.fxu.sum() + self.fsl.sum() + self.fsu.sum())
        # ---- starting point (bound push), multipliers
        self.x = self._push(x0, self.xl, self.xu, self.fxl, self.fxu)
        c0 = self.cons(self.x)
        self.s = self._push(c0, self.sl, self.su, self.fsl, self.fsu)
        self.y = np.zeros(m)
        self.zl = np.where(self.fxl, 1.0, 0.0)
        self.zu = np.where(self.fxu, 1.0, 0.0)
        self.vl = np.where(self.fsl, 1.0, 0.0)
        self.vu = np.where(self.fsu, 1.0, 0.0)
        self.mu = o.mu_init
        self.dw_last = 0.0
        self.filter: list[tuple[float, float]] = []
        th0 = self.theta(self.x, self.s)
        self.theta_max = 1e4 * max(1.0, th0)
        self.theta_min = 1e-4 * max(1.0, th0)
        self.iter = 0
        self.status = None
        self.log: list[dict] = []

    # ------------------------------------------------------------ scaled model
    def obj(self, x):
        return self.sf * self.model.objective(x)

    def grad(self, x):
        return self.sf * self.model.gradient(x)[0]

    def cons(self, x):
        return self.sc * self.model.constraints(x)[0]

    def jac(self, x):
        jr, jc, jv, _ = self.model.jacobian(x)
        return okkt.jac_matrix(self.m, self.n, jr, jc, self.sc[jr] * jv)

    def hess(self, x, y):
        """Lower COO of the scaled Lagrangian Hessian sf grad^2 f - sum (sc y)_i grad^2 c_i."""
        hr, hc, hv, hm = self.model.hessian(x, self.sc * y, self.sf)
        return hr, hc, hv

    @staticmethod
    def _push(v, lo, hi, flo, fhi):
        o_k1, o_k2 = 1e-2, 1e-2
        v = v.copy()
        both = flo & fhi
        pl = np.where(flo, o_k1 * np.maximum(1.0, np.abs(np.where(flo, lo, 0.0))), 0.0)
        pu = np.where(fhi, o_k1 * np.maximum(1.0, np.abs(np.where(fhi, hi, 0.0))), 0.0)
        width = np.where(both, np.where(both, hi, 0.0) - np.where(both, lo, 0.0), np.inf)
        pl = np.where(both, np.minimum(pl, o_k2 * width), pl)
        pu = np.where(both, np.minimum(pu, o_k2 * width), pu)
        v = np.where(flo, np.maximum(v, np.where(flo, lo, 0.0) + pl), v)
        v = np.where(fhi, np.minimum(v, np.where(fhi, hi, 0.0) - pu), v)
        return v

    # ------------------------------------------------------------ merit quantities
    def theta(self, x, s):
        return float(np.sum(np.abs(self.cons(x) - s)))

    def barrier(self, x, s, mu, fval=None):
        f = self.obj(x) if fval is None else fval
        t = 0.0
        t += np.sum(np.log((x - self.xl)[self.fxl]))
        t += np.sum(np.log((self.xu - x)[self.fxu]))
        t += np.sum(np.log((s - self.sl)[self.fsl]))
        t += np.sum(np.log((self.su - s)[self.fsu]))
        return f - mu * t

    def residuals(self, mu, g=None, Jm=None, c=None):
        """F = (Fx, Fs, Fy, Fzl, Fzu, Fvl, Fvu), the first-order conditions of the barrier problem."""
        x, s, y = self.x, self.s, self.y
        g = self.grad(x) if g is None else g
        Jm = self.jac(x) if Jm is None else Jm
        c = self.cons(x) if c is None else c
        Fx = g - Jm.T @ y - self.zl + self.zu
        Fs = y - self.vl + self.vu
        Fy = c - s
        Fzl = np.where(self.fxl, self.zl * (x - np.where(self.fxl, self.xl, 0.0)) - mu, 0.0)
        Fzu = np.where(self.fxu, self.zu * (np.where(self.fxu, self.xu, 0.0) - x) - mu, 0.0)
        Fvl = np.where(self.fsl, self.vl * (s - np.where(self.fsl, self.sl, 0.0)) - mu, 0.0)
        Fvu = np.where(self.fsu, self.vu * (np.where(self.fsu, self.su, 0.0) - s) - mu, 0.0)
        return Fx, Fs, Fy, Fzl, Fzu, Fvl, Fvu

    def error(self, mu, F=None):
        """Scaled optimality error E_mu (Waechter-Biegler eq. (5))."""
        Fx, Fs, Fy, Fzl, Fzu, Fvl, Fvu = self.residuals(mu) if F is None else F
        o = self.o
        z1 = np.sum(np.abs(self.zl)) + np.sum(np.abs(self.zu)) + np.sum(np.abs(self.vl)) + np.sum(np.abs(self.vu))
        y1 = np.sum(np.abs(self.y))
        nb = max(self.nbounds, 1)
        sd = max(o.s_max, (y1 + z1) / (self.m + nb)) / o.s_max
        scc = max(o.s_max, z1 / nb) / o.s_max
        dual = max(np.max(np.abs(Fx)), np.max(np.abs(Fs)))
        primal = np.max(np.abs(Fy))
        compl = max(np.max(np.abs(Fzl)), np.max(np.abs(Fzu)), np.max(np.abs(Fvl)), np.max(np.abs(Fvu)))
        return max(dual / sd, primal, compl / scc), dual, primal, compl

    # ------------------------------------------------------------ Newton step pieces
    def sigmas(self):
        dxl = np.where(self.fxl, self.x - np.where(self.fxl, self.xl, 0.0), 1.0)
        dxu = np.where(self.fxu, np.where(self.fxu, self.xu, 0.0) - self.x, 1.0)
        dsl = np.where(self.fsl, self.s - np.where(self.fsl, self.sl, 0.0), 1.0)
        dsu = np.where(self.fsu, np.where(self.fsu, self.su, 0.0) - self.s, 1.0)
        Sx = self.zl / dxl + self.zu / dxu
        Ss = self.vl / dsl + self.vu / dsu
        return Sx, Ss, (dxl, dxu, dsl, dsu)

    def reduce_solve(self, R, Jm, Sx, Ss, dist, dw):
        """Solve J_F d = R through the condensed system with the current factor (Section IV-C)."""
        Rx, Rs, Ry, Rzl, Rzu, Rvl, Rvu = R
        dxl, dxu, dsl, dsu = dist
        qx = Rx + np.where(self.fxl, Rzl / dxl, 0.0) - np.where(self.fxu, Rzu / dxu, 0.0)
        qs = Rs + np.where(self.fsl, Rvl / dsl, 0.0) - np.where(self.fsu, Rvu / dsu, 0.0)
        qy = Ry
        D = Ss + dw
        rhs = qx + Jm.T @ (qs + D * qy)
        dx = self.chol.solve(rhs)
        ds = Jm @ dx - qy
        dy = qs - D * ds
        dzl = np.where(self.fxl, (Rzl - self.zl * dx) / dxl, Rzl)
        dzu = np.where(self.fxu, (Rzu + self.zu * dx) / dxu, Rzu)
        dvl = np.where(self.fsl, (Rvl - self.vl * ds) / dsl, Rvl)
        dvu = np.where(self.fsu, (Rvu + self.vu * ds) / dsu, Rvu)
        return [dx, ds, dy, dzl, dzu, dvl, dvu]

    def full_residual(self, R, d, Wm, Jm, dist, dw):
        """R - J_F d for the full (unreduced) Newton system including the regularization."""
        dx, ds, dy, dzl, dzu, dvl, dvu = d
        dxl, dxu, dsl, dsu = dist
        Rx, Rs, Ry, Rzl, Rzu, Rvl, Rvu = R
        rx = Rx - (Wm @ dx + dw * dx - Jm.T @ dy - dzl + dzu)
        rs = Rs - (dw * ds + dy - dvl + dvu)
        ry = Ry - (Jm @ dx - ds)
        rzl = np.where(self.fxl, Rzl - (self.zl * dx + dxl * dzl), 0.0)
        rzu = np.where(self.fxu, Rzu - (-self.zu * dx + dxu * dzu), 0.0)
        rvl = np.where(self.fsl, Rvl - (self.vl * ds + dsl * dvl), 0.0)
        rvu = np.where(self.fsu, Rvu - (-self.vu * ds + dsu * dvu), 0.0)
        return [rx, rs, ry, rzl, rzu, rvl, rvu]

    def factor_with_inertia_correction(self, hr, hc, hv, Jm, Sx, Ss):
        """Factor K(dw), increasing dw until K is positive definite (Algorithm 1, regularization)."""
        o = self.o
        trials = 0

        def kvals(dw):
            v = okkt.condensed_values(self.n, self.krow, self.kcol, hr, hc, hv, Jm, Sx, Ss + dw, dw)
            return v

        dw = 0.0
        bad = self.chol.factor(kvals(dw), o.pivot_tol)
        trials += 1
        if bad < 0:
            return dw, trials
        dw = o.dw_first if self.dw_last == 0.0 else max(o.dw_min, o.kappa_w_minus * self.dw_last)
        while True:
            if dw > o.dw_max:
                return None, trials
            bad = self.chol.factor(kvals(dw), o.pivot_tol)
            trials += 1
            if bad < 0:
                self.dw_last = dw
                return dw, trials
            dw *= o.kappa_w_plus_first if self.dw_last == 0.0 else o.kappa_w_plus

    def direction(self, mu, hr, hc, hv, Jm, F):
        Sx, Ss, dist = self.sigmas()
        out = self.factor_with_inertia_correction(hr, hc, hv, Jm, Sx, Ss)
        dw, trials = out
        if dw is None:
            return None, None, trials, 0
        d, nir = self.refined_solve([-v for v in F], hr, hc, hv, Jm, dw)
        return d, dw, trials, nir

    def refined_solve(self, R0, hr, hc, hv, Jm, dw):
        """J_F d = R0 through the current factor, with iterative refinement on the full system."""
        Sx, Ss, dist = self.sigmas()
        Wm = okkt.sym_from_lower(self.n, hr, hc, hv)
        d = self.reduce_solve(R0, Jm, Sx, Ss, dist, dw)
        nr0 = max(np.max(np.abs(v)) for v in R0)
        nir = 0
        prev = math.inf
        for _ in range(self.o.max_ir):
            res = self.full_residual(R0, d, Wm, Jm, dist, dw)
            rn = max(np.max(np.abs(v)) for v in res)
            if rn <= self.o.ir_tol * max(1.0, nr0) or rn > self.o.ir_stall * prev:
                break
            prev = rn
            corr = self.reduce_solve(res, Jm, Sx, Ss, dist, dw)
            d = [a + b for a, b in zip(d, corr)]
            nir += 1
        return d, nir

    def step_to_boundary(self, tau, d):
        dx, ds, dy, dzl, dzu, dvl, dvu = d

        def amax(v, dv, mask_neg):
            sel = mask_neg & (dv < 0)
            if not np.any(sel):
                return 1.0
            return float(min(1.0, np.min(-tau * v[sel] / dv[sel])))

        a = 1.0
        a = min(a, amax(self.x - np.where(self.fxl, self.xl, 0.0), dx, self.fxl))
        a = min(a, amax(np.where(self.fxu, self.xu, 0.0) - self.x, -dx, self.fxu))
        a = min(a, amax(self.s - np.where(self.fsl, self.sl, 0.0), ds, self.fsl))
        a = min(a, amax(np.where(self.fsu, self.su, 0.0) - self.s, -ds, self.fsu))
        az = 1.0
        az = min(az, amax(self.zl, dzl, self.fxl))
        az = min(az, amax(self.zu, dzu, self.fxu))
        az = min(az, amax(self.vl, dvl, self.fsl))
        az = min(az, amax(self.vu, dvu, self.fsu))
        return a, az

    def barrier_gradient_dot(self, g, mu, dx, ds):
        t = float(g @ dx)
        t -= mu * float(np.sum((dx / np.where(self.fxl, self.x - np.where(self.fxl, self.xl, 0.0), 1.0))[self.fxl]))
        t += mu * float(np.sum((dx / np.where(self.fxu, np.where(self.fxu, self.xu, 0.0) - self.x, 1.0))[self.fxu]))
        t -= mu * float(np.sum((ds / np.where(self.fsl, self.s - np.where(self.fsl, self.sl, 0.0), 1.0))[self.fsl]))
        t += mu * float(np.sum((ds / np.where(self.fsu, np.where(self.fsu, self.su, 0.0) - self.s, 1.0))[self.fsu]))
        return t

    def filter_ok(self, th, ph):
        return all(th < tf or ph < pf for tf, pf in self.filter)

    def acceptable(self, tht, pht, alpha, th0, ph0, gphi):
        """Filter and sufficient-decrease test of a trial point: (accepted, f-type step)."""
        o = self.o
        if not (np.isfinite(tht) and np.isfinite(pht) and tht < self.theta_max and self.filter_ok(tht, pht)):
            return False, False
        switching = gphi < 0 and alpha * (-gphi) ** o.s_phi > o.delta * th0 ** o.s_theta
        if th0 <= self.theta_min and switching:
            return pht <= ph0 + o.eta_phi * alpha * gphi, True
        return tht <= (1.0 - o.gamma_theta) * th0 or pht <= ph0 - o.gamma_phi * th0, False

    def second_order_correction(self, mu, tau, F, hr, hc, hv, Jm, dw, c, alpha0, ct, st_, th0, ph0, gphi):
        """Second-order correction after the first trial point (step alpha0) was rejected with a larger
        infeasibility than the current point (Waechter-Biegler 2006, Section 2.4): the same Newton matrix is
        solved again with the constraint residual replaced by the accumulated
        c_soc = alpha0 (c(x) - s) + (c(x_trial) - s_trial), up to soc_max times while each correction cuts the
        infeasibility by kappa_soc.  Returns (direction, alpha, alpha_z, f-type) of an accepted corrected step,
        or None."""
        o = self.o
        c_soc = alpha0 * (c - self.s) + (ct - st_)
        th_old = float(np.sum(np.abs(ct - st_)))
        for p in range(1, o.soc_max + 1):
            R = [-F[0], -F[1], -c_soc, -F[3], -F[4], -F[5], -F[6]]
            d, _ = self.refined_solve(R, hr, hc, hv, Jm, dw)
            a, az = self.step_to_boundary(tau, d)
            xs = self.x + a * d[0]
            ss = self.s + a * d[1]
            cs = self.cons(xs)
            ths = float(np.sum(np.abs(cs - ss)))
            phs = self.barrier(xs, ss, mu)
            ok, ftype = self.acceptable(ths, phs, alpha0, th0, ph0, gphi)
            if ok:
                return d, a, az, ftype
            if p == o.soc_max or ths > o.kappa_soc * th_old:
                return None
            c_soc = a * c_soc + (cs - ss)
            th_old = ths
        return None

    # ------------------------------------------------------------ one iteration
    def step(self):
        """One iteration of Algorithm 1.  Returns a status code if the run has ended, else None."""
        o = self.o
        g = self.grad(self.x)
        Jm = self.jac(self.x)
        c = self.cons(self.x)
        F0 = self.residuals(0.0, g, Jm, c)
        E0 = self.error(0.0, F0)
        info = {"iter": self.iter, "obj": self.model.objective(self.x), "E0": E0[0], "inf_pr": E0[2],
                "inf_du": E0[1], "mu": self.mu}
        if not np.isfinite(E0[0]):
            self.status = Status.NUMERIC
            return self.status
        if E0[0] <= o.tol:
            self.status = Status.OK
            self.log.append(info)
            return self.status
        if self.iter >= o.max_iter:
            self.status = Status.MAXITER
            return self.status
        # barrier parameter update (monotone, fast decrease allowed)
        mu_min = o.tol / 10.0
        while True:
            Emu = self.error(self.mu, self.residuals(self.mu, g, Jm, c))[0]
            if Emu > o.kappa_eps * self.mu or self.mu <= mu_min:
                break
            new_mu = max(mu_min, min(o.kappa_mu * self.mu, self.mu ** o.theta_mu))
            if new_mu >= self.mu:
                break
            self.mu = new_mu
            self.filter = []
        mu = self.mu
        tau = max(o.tau_min, 1.0 - mu)
        hr, hc, hv = self.hess(self.x, self.y)
        F = self.residuals(mu, g, Jm, c)
        d, dw, trials, nir = self.direction(mu, hr, hc, hv, Jm, F)
        if d is None:
            self.status = Status.REGULARIZATION
            return self.status
        dx, ds, dy, dzl, dzu, dvl, dvu = d
        amax, az = self.step_to_boundary(tau, d)
        # filter line search
        th0 = float(np.sum(np.abs(c - self.s)))
        ph0 = self.barrier(self.x, self.s, mu)
        gphi = self.barrier_gradient_dot(g, mu, dx, ds)
        tiny = max(np.max(np.abs(dx) / (1.0 + np.abs(self.x))), np.max(np.abs(ds) / (1.0 + np.abs(self.s)))) \
            < 10.0 * EPS_MACH
        alpha = amax
        nls = 0
        accepted = False
        augment = False
        if tiny:
            accepted = True
        else:
            if gphi < 0:
                if th0 <= self.theta_min:
                    amin = o.gamma_alpha * min(o.gamma_theta, o.gamma_phi * th0 / (-gphi),
                                               o.delta * th0 ** o.s_theta / (-gphi) ** o.s_phi)
                else:
                    amin = o.gamma_alpha * min(o.gamma_theta, o.gamma_phi * th0 / (-gphi))
            else:
                amin = o.gamma_alpha * o.gamma_theta
            nsoc = 0
            while True:
                nls += 1
                xt = self.x + alpha * dx
                st = self.s + alpha * ds
                ct = self.cons(xt)
                tht = float(np.sum(np.abs(ct - st)))
                pht = self.barrier(xt, st, mu)
                ok, ftype = self.acceptable(tht, pht, alpha, th0, ph0, gphi)
                if ok:
                    accepted = True
                    augment = not ftype
                    break
                if o.soc and nls == 1 and tht >= th0:
                    corr = self.second_order_correction(mu, tau, F, hr, hc, hv, Jm, dw, c, alpha, ct, st, th0, ph0,
                                                        gphi)
                    nsoc += 1
                    if corr is not None:
                        d, alpha, az, ftype = corr
                        dx, ds, dy, dzl, dzu, dvl, dvu = d
                        accepted = True
                        augment = not ftype
                        break
                alpha *= 0.5
                if alpha < amin:
                    break
        if not accepted:
            self.status = Status.LINESEARCH
            info.update({"dw": dw, "ls": nls, "ir": nir})
            self.log.append(info)
            return self.status
        if augment:
            self.filter.append(((1.0 - o.gamma_theta) * th0, ph0 - o.gamma_phi * th0))
        self.x = self.x + alpha * dx
        self.s = self.s + alpha * ds
        self.y = self.y + alpha * dy
        self.zl = self.zl + az * dzl
        self.zu = self.zu + az * dzu
        self.vl = self.vl + az * dvl
        self.vu = self.vu + az * dvu
        self._safeguard(mu)
        info.update({"dw": dw, "alpha": alpha, "alpha_z": az, "ls": nls, "ir": nir, "trials": trials,
                     "soc": 0 if tiny else nsoc})
        self.log.append(info)
        self.iter += 1
        return None

    def _safeguard(self, mu):
        k = self.o.kappa_sigma

        def clip(z, dist, mask):
            d = np.where(mask, dist, 1.0)
            return np.where(mask, np.maximum(np.minimum(z, k * mu / d), mu / (k * d)), z)

        self.zl = clip(self.zl, self.x - np.where(self.fxl, self.xl, 0.0), self.fxl)
        self.zu = clip(self.zu, np.where(self.fxu, self.xu, 0.0) - self.x, self.fxu)
        self.vl = clip(self.vl, self.s - np.where(self.fsl, self.sl, 0.0), self.fsl)
        self.vu = clip(self.vu, np.where(self.fsu, self.su, 0.0) - self.s, self.fsu)

    def solve(self, verbose=False):
        while True:
            st = self.step()
            if verbose and self.log:
                r = self.log[-1]
                print("%4d %.10e %.2e %.2e %.1e dw=%s a=%s ls=%s ir=%s" % (
                    r["iter"], r["obj"], r["inf_pr"], r["inf_du"], r["mu"], r.get("dw"), r.get("alpha"),
                    r.get("ls"), r.get("ir")), flush=True)
            if st is not None:
                return st


def solve(grid, tol=1e-4, verbose=False, **kw):
    m = Model(grid)
    ipm = IPM(m, Options(tol=tol, **kw))
    st = ipm.solve(verbose=verbose)
    return ipm, st
