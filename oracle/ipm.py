"""Oracle interior-point method for the scenario absorber NLP (problem 10).

TEST INFRASTRUCTURE ONLY (see oracle/model.py).

The paper solves problem (10) with MadNLP at tolerance 1e-8 (Numerical
results); MadNLP implements the filter line-search primal-dual interior-point
algorithm of Waechter & Biegler (Math. Program. 106, 2006).  This module takes
that algorithm's steps in that paper's order and notation:

  A-1  initialisation: bound push, slack init, least-squares multipliers
  A-2  overall convergence test on the scaled optimality error E_0
  A-3  monotone barrier update while E_mu <= kappa_eps mu
  A-4  search direction from the primal-dual system with inertia correction
  A-5  fraction-to-boundary and backtracking filter line search
  A-6  acceptance; bound multipliers with their own step, then the safeguard
  A-7  filter augmentation

Readings (where the paper is silent): Ipopt's default constants throughout;
each variable is scaled by the magnitude of its cold-start value (1 where that
value is 0), the way a user scaling of the variables is given to Ipopt; then
gradient-based NLP scaling of the rows (max gradient 100) at the bound-pushed
cold point;
no second-order correction, no restoration phase (a failed line search returns
status LS_FAIL), no watchdog.

Problem form.  Variables w = (z_1..z_S, d) with bounds; the hydraulic rows
g(w) <= 0 become g(w) - s = 0 with a slack s <= 0 (upper bound 0).  With
n_sections = p > 1 the shared design variables are the diameters theta_1..p of
p contiguous column sections (the general design vector of the scenario NLP,
eq. 8): each stage's hydraulic row uses its section's diameter and the design
cost is sum_k (N_k / N) theta_k, N_k the stages of section k.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import model as M
from .kkt import BorderedKKT, scenario_kkt

SUCCESS, MAX_ITER, LS_FAIL, INERTIA_FAIL, NAN_IN_EVAL, DIVERGING = 0, -12, -11, -10, -13, -14
# The backtracking stops below the minimum step of the filter line search
# (Waechter & Biegler 2006, eq. 23); when the directional derivative is huge
# that bound underflows, so a step below double-precision resolution relative
# to a unit step also ends it.
ALPHA_FLOOR = 2.0 ** -52


@dataclass
class IpmOptions:
    tol: float = 1e-8
    max_iter: int = 500
    mu_init: float = 0.1
    bound_push: float = 1e-2
    bound_frac: float = 1e-2
    slack_bound_push: float = 1e-2
    bound_mult_init: float = 1.0
    constr_mult_init_max: float = 1e3
    nlp_scaling_max_gradient: float = 100.0
    kappa_eps: float = 10.0
    kappa_mu: float = 0.2
    theta_mu: float = 1.5
    tau_min: float = 0.99
    kappa_sigma: float = 1e10
    kappa_d: float = 1e-5
    s_max: float = 100.0
    gamma_theta: float = 1e-5
    gamma_phi: float = 1e-8
    delta: float = 1.0
    s_theta: float = 1.1
    s_phi: float = 2.3
    eta_phi: float = 1e-8
    gamma_alpha: float = 0.05
    theta_max_fact: float = 1e4
    theta_min_fact: float = 1e-4
    dw_init: float = 1e-4
    dw_min: float = 1e-20
    dw_max: float = 1e40
    kappa_w_minus: float = 1.0 / 3.0
    kappa_w_plus: float = 8.0
    kappa_w_plus_bar: float = 100.0
    dc_bar: float = 1e-8
    kappa_c: float = 0.25
    mu_min: float = 1e-11
    warm_start: bool = False
    warm_mu_init: float = 1e-6
    warm_bound_push: float = 1e-8


@dataclass
class IpmResult:
    status: int
    iterations: int
    E0: float
    d: float
    x: np.ndarray
    yc: np.ndarray
    yd: np.ndarray
    zL: np.ndarray
    zU: np.ndarray
    s: np.ndarray
    vU: np.ndarray
    seconds: float
    log: list = field(default_factory=list)
    n_inertia_corrections: int = 0
    max_lin_resid: float = 0.0
    theta: np.ndarray | None = None  # the p design variables (theta = [d] for one diameter)


class Problem:
    """Problem (10) for S scenarios and N stages, with the oracle's model."""

    def __init__(self, params: dict, feeds: np.ndarray, n_stages: int, n_sections: int = 1):
        self.P = M.OracleParams(params)
        self.p = params
        self.feeds = np.ascontiguousarray(feeds, dtype=np.float64)
        self.S, self.N = self.feeds.shape[0], int(n_stages)
        self.npar = int(n_sections)
        self.c = M.section_weights(self.N, self.npar)  # design-cost weight of each diameter
        # the expected operating cost sum_k a_k theta_k^-4 (zero weight: the case study's objective)
        self.a = M.operating_coefficients(self.feeds, self.N, self.npar, self.P)
        self.nz = self.S * self.N * M.NV
        self.n = self.nz + self.npar
        self.mI = self.S * self.N
        self.mE = self.S * self.N * (M.NR - 1)
        self._bounds()

    def _bounds(self):
        b = self.p["bounds"]
        lo = np.full(M.NV, -np.inf)
        hi = np.full(M.NV, np.inf)
        lo[0:9], hi[0:9] = b["x"]
        lo[9:13], hi[9:13] = b["y"]
        lo[M.IL], hi[M.IL] = b["L"]
        lo[M.IV], hi[M.IV] = b["V"]
        lo[M.IT], hi[M.IT] = b["T"]
        self.xL = np.concatenate([np.tile(lo, self.S * self.N), np.full(self.npar, b["d"][0])])
        self.xU = np.concatenate([np.tile(hi, self.S * self.N), np.full(self.npar, b["d"][1])])

    def initial_point(self) -> np.ndarray:
        """The cold-start point: every stage starts from the lean-solvent liquid,
        the nominal gas, the inlet flows and temperature, zero extents; d0."""
        ip = self.p["initial_point"]
        z = np.zeros(M.NV)
        z[0:9] = ip["x"]
        z[9:13] = ip["y"]
        z[M.IL], z[M.IV], z[M.IT] = ip["L"], ip["V"], ip["T"]
        z[M.IE:M.IE + 5] = ip["eps"]
        return np.concatenate([np.tile(z, self.S * self.N), np.full(self.npar, ip["d"])])

    # --- model evaluations on the full vector -------------------------------------------
    def split(self, x):
        """States (S, N, 21) and the design: the diameter, or the (p,) section diameters."""
        Z = x[:self.nz].reshape(self.S, self.N, M.NV)
        return Z, (float(x[self.nz]) if self.npar == 1 else np.array(x[self.nz:]))

    def cons(self, x):
        Z, d = self.split(x)
        return M.constraints(Z, d, self.feeds, self.P)  # (S, N, 22)

    def jac_blocks(self, x):
        Z, d = self.split(x)
        return [M.jacobian(Z[w], d, self.feeds[w], self.P) for w in range(self.S)]

    def hess_blocks(self, x, lam):
        """lam: (S, N, 22) weights of the (unscaled) rows."""
        Z, d = self.split(x)
        return [M.lagrangian_hessian(Z[w], d, self.feeds[w], lam[w], self.P) for w in range(self.S)]


class OracleIPM:
    def __init__(self, prob: Problem, opts: IpmOptions | None = None, verbose: bool = False, on_factor=None):
        self.pr = prob
        self.o = opts or IpmOptions()
        self.verbose = verbose
        # optional observer called as on_factor(F, dw, dc) after every factorisation
        # of the inertia-correction loop (A-4), for tests that check each trial
        self.on_factor = on_factor
        pr = prob
        self.hasL = np.isfinite(pr.xL)
        self.hasU = np.isfinite(pr.xU)
        self.onlyL = self.hasL & ~self.hasU
        self.onlyU = self.hasU & ~self.hasL
        self.n_inertia_corr = 0
        self.max_lin_resid = 0.0
        x0 = prob.initial_point()
        self.D = np.where(x0 != 0.0, np.abs(x0), 1.0)  # variable scaling x = D * xt
        self.xL = pr.xL / self.D
        self.xU = pr.xU / self.D

    # ---- scaling (gradient-based, at the cold point) ----
    def compute_scaling(self, x0):
        pr, o = self.pr, self.o
        Js = pr.jac_blocks(self.D * x0)
        cs = np.empty((pr.S, pr.N, M.NR))
        for w, J in enumerate(Js):
            J = J * self.block_scale(w)[None, :]
            g = np.abs(J).max(axis=1).reshape(pr.N, M.NR)
            cs[w] = np.minimum(1.0, o.nlp_scaling_max_gradient / np.maximum(g, 1e-300))
        self.cs = cs
        # gradient-based objective scaling: grad f = c - 4 a theta^-5 in the original
        # design variables (c = 1, a = 0 for problem (10)), at the cold point
        q = pr.npar
        th0 = self.D[-q:] * x0[-q:]
        gmax = float(np.max(np.abs(pr.c - 4.0 * pr.a * th0 ** -5.0) * self.D[-q:]))
        self.sf = min(1.0, o.nlp_scaling_max_gradient / gmax)

    def push_into_bounds(self, x, push, frac):
        """A-1 bound push: move x strictly inside [xL, xU] (Ipopt's kappa_1, kappa_2 rule)."""
        xL, xU = self.xL, self.xU
        both = self.hasL & self.hasU
        x = x.copy()
        with np.errstate(invalid="ignore"):
            pL = push * np.maximum(1.0, np.abs(xL))
            pU = push * np.maximum(1.0, np.abs(xU))
            pL = np.where(both, np.minimum(pL, frac * (xU - xL)), pL)
            pU = np.where(both, np.minimum(pU, frac * (xU - xL)), pU)
            x[self.hasL] = np.maximum(x[self.hasL], (xL + pL)[self.hasL])
            x[self.hasU] = np.minimum(x[self.hasU], (xU - pU)[self.hasU])
        return x

    # ---- scaled quantities ----
    def eval_c(self, x):
        c = self.pr.cons(self.D * x) * self.cs
        return c[:, :, :M.NR - 1], c[:, :, M.NR - 1]  # cE (S,N,21), dI (S,N)

    def grad_f(self, x):
        """Gradient of the scaled objective sf (sum_k c_k theta_k + a_k theta_k^-4)
        with respect to the scaled variables (theta = D x on the design entries)."""
        q = self.pr.npar
        g = np.zeros(self.pr.n)
        th = self.D[-q:] * x[-q:]
        g[-q:] = self.sf * self.D[-q:] * (self.pr.c - 4.0 * self.pr.a * th ** -5.0)
        return g

    def hess_f(self, x):
        """Diagonal of the scaled objective's Hessian on the design entries, (p,)."""
        q = self.pr.npar
        th = self.D[-q:] * x[-q:]
        return self.sf * self.D[-q:] ** 2 * 20.0 * self.pr.a * th ** -6.0

    def f_nonlinear(self, x):
        """The operating-cost part of the scaled objective, sf sum_k a_k theta_k^-4."""
        q = self.pr.npar
        th = self.D[-q:] * x[-q:]
        return self.sf * float(np.sum(self.pr.a * th ** -4.0))

    def block_scale(self, w):
        nzs = self.pr.N * M.NV
        return np.concatenate([self.D[w * nzs:(w + 1) * nzs], self.D[-self.pr.npar:]])

    def jac_scaled(self, x):
        out = []
        for w, J in enumerate(self.pr.jac_blocks(self.D * x)):
            out.append(J * self.cs[w].reshape(-1)[:, None] * self.block_scale(w)[None, :])
        return out

    def JT_times(self, Jb, yc, yd):
        """J^T y for the full vector, from per-scenario blocks."""
        pr = self.pr
        q = pr.npar
        r = np.zeros(pr.n)
        for w, J in enumerate(Jb):
            lam = np.concatenate([yc[w], yd[w][:, None]], axis=1).reshape(-1)
            v = J.T @ lam
            r[w * pr.N * M.NV:(w + 1) * pr.N * M.NV] += v[:-q]
            r[-q:] += v[-q:]
        return r

    def J_times(self, Jb, dx):
        pr = self.pr
        cE = np.empty((pr.S, pr.N, M.NR - 1))
        dI = np.empty((pr.S, pr.N))
        for w, J in enumerate(Jb):
            v = J @ np.concatenate([dx[w * pr.N * M.NV:(w + 1) * pr.N * M.NV], dx[-pr.npar:]])
            v = v.reshape(pr.N, M.NR)
            cE[w], dI[w] = v[:, :M.NR - 1], v[:, M.NR - 1]
        return cE, dI

    # ---- barrier pieces ----
    def slacks(self, x):
        sL = np.where(self.hasL, x - self.xL, 1.0)
        sU = np.where(self.hasU, self.xU - x, 1.0)
        return sL, sU

    def barrier_phi(self, x, s, mu):
        sL, sU = self.slacks(x)
        if np.any(sL[self.hasL] <= 0) or np.any(sU[self.hasU] <= 0) or np.any(s >= 0):
            return np.inf
        q = self.pr.npar
        phi = self.sf * x[-1] if q == 1 else self.sf * float((self.pr.c * self.D[-q:]) @ x[-q:])
        phi += self.f_nonlinear(x)
        phi -= mu * (np.log(sL[self.hasL]).sum() + np.log(sU[self.hasU]).sum() + np.log(-s).sum())
        phi += self.o.kappa_d * mu * (sL[self.onlyL].sum() + sU[self.onlyU].sum() + (-s).sum())
        return phi

    def grad_phi(self, x, s, mu):
        sL, sU = self.slacks(x)
        g = self.grad_f(x)
        g = g - np.where(self.hasL, mu / sL, 0.0) + np.where(self.hasU, mu / sU, 0.0)
        g = g + self.o.kappa_d * mu * (self.onlyL.astype(float) - self.onlyU.astype(float))
        gs = mu / (-s) - self.o.kappa_d * mu
        return g, gs

    @staticmethod
    def theta(cE, dI, s):
        return float(np.abs(cE).sum() + np.abs(dI - s).sum())

    # ---- optimality error ----
    def opt_error(self, x, s, yc, yd, zL, zU, vU, Jb, cE, dI, mu):
        o = self.o
        sL, sU = self.slacks(x)
        gl = self.grad_f(x) + self.JT_times(Jb, yc, yd) - zL + zU
        gls = -yd + vU
        dual = max(np.abs(gl).max(), np.abs(gls).max())
        primal = max(np.abs(cE).max(), np.abs(dI - s).max())
        comp = max(np.abs(np.where(self.hasL, sL * zL - mu, 0.0)).max(),
                   np.abs(np.where(self.hasU, sU * zU - mu, 0.0)).max(),
                   np.abs((-s) * vU - mu).max())
        nmult = yc.size + yd.size + int(self.hasL.sum()) + int(self.hasU.sum()) + vU.size
        sd = max(o.s_max, (np.abs(yc).sum() + np.abs(yd).sum() + np.abs(zL).sum() + np.abs(zU).sum()
                           + np.abs(vU).sum()) / nmult) / o.s_max
        nb = int(self.hasL.sum()) + int(self.hasU.sum()) + vU.size
        sc = max(o.s_max, (np.abs(zL).sum() + np.abs(zU).sum() + np.abs(vU).sum()) / nb) / o.s_max
        return max(dual / sd, primal, comp / sc), dual, primal, comp

    # ---- KKT ----
    def factor(self, x, yc, yd, sig_x, sig_s, dw, dc, Jb, objective=True):
        """The bordered KKT at x; objective=False leaves out the objective's
        curvature (the least-squares multiplier system has the identity block)."""
        pr = self.pr
        lam = np.concatenate([yc, yd[:, :, None]], axis=2) * self.cs  # unscaled-row weights
        Hb = pr.hess_blocks(self.D * x, lam)
        q = pr.npar
        blocks, borders, kdd = [], [], 0.0 if q == 1 else np.zeros((q, q))
        for w in range(pr.S):
            bs = self.block_scale(w)
            Hb[w] = Hb[w] * bs[:, None] * bs[None, :]
            sl = slice(w * pr.N * M.NV, (w + 1) * pr.N * M.NV)
            K, b, hdd = scenario_kkt(Jb[w], Hb[w], sig_x[sl], sig_s[w], dw, dc, pr.N, q)
            blocks.append(K)
            borders.append(b)
            kdd = kdd + hdd
        hf = self.hess_f(x) if objective else np.zeros(q)  # the objective's curvature in the design entries
        if q == 1:
            kdd += sig_x[-1] + dw + float(hf[0])
        else:
            kdd = kdd + np.diag(sig_x[-q:] + dw + hf)
        return BorderedKKT(blocks, borders, kdd)

    def kkt_solve(self, F, rx, rc, rd):
        """Solve K [dx; dyc; dyd] = [rx; rc; rd] (reduced system), returns full vectors."""
        pr = self.pr
        nzs = pr.N * M.NV
        q = pr.npar
        rs = []
        for w in range(pr.S):
            rs.append(np.concatenate([rx[w * nzs:(w + 1) * nzs], rc[w].reshape(-1), rd[w]]))
        rth = rx[-1] if q == 1 else rx[-q:]
        sol, dd = F.solve(rs, rth)
        self.max_lin_resid = max(self.max_lin_resid, F.rel_residual(sol, dd, rs, rth))
        dx = np.empty(pr.n)
        dyc = np.empty((pr.S, pr.N, M.NR - 1))
        dyd = np.empty((pr.S, pr.N))
        nE = pr.N * (M.NR - 1)
        for w in range(pr.S):
            u = sol[w]
            dx[w * nzs:(w + 1) * nzs] = u[:nzs]
            dyc[w] = u[nzs:nzs + nE].reshape(pr.N, M.NR - 1)
            dyd[w] = u[nzs + nE:]
        if q == 1:
            dx[-1] = dd
        else:
            dx[-q:] = dd
        return dx, dyc, dyd

    # ---- fraction to boundary ----
    def ftb_primal(self, x, dx, s, ds, tau):
        a = 1.0
        sL, sU = self.slacks(x)
        m = self.hasL & (dx < 0)
        if m.any():
            a = min(a, float(np.min(-tau * sL[m] / dx[m])))
        m = self.hasU & (dx > 0)
        if m.any():
            a = min(a, float(np.min(tau * sU[m] / dx[m])))
        m = ds > 0
        if m.any():
            a = min(a, float(np.min(tau * (-s[m]) / ds[m])))
        return a

    @staticmethod
    def ftb_dual(zs, dzs, tau):
        a = 1.0
        for z, dz in zip(zs, dzs):
            m = dz < 0
            if m.any():
                a = min(a, float(np.min(-tau * z[m] / dz[m])))
        return a

    # ---- the algorithm ----
    def solve(self, x0=None, yc0=None, yd0=None):
        pr, o = self.pr, self.o
        t0 = time.perf_counter()
        log = []
        xcold = self.push_into_bounds(pr.initial_point() / self.D, o.bound_push, o.bound_frac)
        # scaling factors come from the bound-pushed cold point in every mode, so a
        # warm-started solve converges on the same scaled problem as a cold one
        self.compute_scaling(xcold)
        warm = x0 is not None and o.warm_start
        if x0 is None:
            x = xcold.copy()
        elif warm:
            x = self.push_into_bounds(np.asarray(x0, dtype=np.float64) / self.D, o.warm_bound_push, o.warm_bound_push)
        else:
            x = self.push_into_bounds(np.asarray(x0, dtype=np.float64) / self.D, o.bound_push, o.bound_frac)
        mu = o.warm_mu_init if warm else o.mu_init
        cE, dI = self.eval_c(x)
        spush = o.warm_bound_push if warm else o.slack_bound_push
        s = np.minimum(dI, -spush)
        if warm:
            sL, sU = self.slacks(x)
            zL = np.where(self.hasL, mu / sL, 0.0)
            zU = np.where(self.hasU, mu / sU, 0.0)
            vU = mu / (-s)
        else:
            zL = np.where(self.hasL, o.bound_mult_init, 0.0)
            zU = np.where(self.hasU, o.bound_mult_init, 0.0)
            vU = np.full((pr.S, pr.N), o.bound_mult_init)
        Jb = self.jac_scaled(x)
        if warm and yc0 is not None:
            yc = np.asarray(yc0, dtype=np.float64).reshape(pr.S, pr.N, M.NR - 1).copy()
            yd = np.asarray(yd0, dtype=np.float64).reshape(pr.S, pr.N).copy()
        else:
            # least-squares multipliers: [[I, J^T], [J, 0]] with the slack block eliminated
            sig0x = np.zeros(pr.n)
            sig0s = np.zeros((pr.S, pr.N))
            F = self.factor(x, np.zeros((pr.S, pr.N, M.NR - 1)), np.zeros((pr.S, pr.N)),
                            sig0x, sig0s, 1.0, 0.0, Jb, objective=False)
            rx = -(self.grad_f(x) - zL + zU)
            _, yc, yd = self.kkt_solve(F, rx, np.zeros((pr.S, pr.N, M.NR - 1)), -vU)
            if max(np.abs(yc).max(), np.abs(yd).max()) > o.constr_mult_init_max:
                yc = np.zeros_like(yc)
                yd = np.zeros_like(yd)
        th0 = self.theta(cE, dI, s)
        theta_max = o.theta_max_fact * max(1.0, th0)
        theta_min = o.theta_min_fact * max(1.0, th0)
        filt = []  # list of (theta, phi) corner points
        dw_last = 0.0
        tau = max(o.tau_min, 1.0 - mu)
        status = MAX_ITER
        it = 0
        E0 = np.inf
        while True:
            # A-2: overall convergence
            E0, _, _, _ = self.opt_error(x, s, yc, yd, zL, zU, vU, Jb, cE, dI, 0.0)
            if not np.isfinite(E0):
                status = NAN_IN_EVAL
                break
            if E0 <= o.tol:
                status = SUCCESS
                break
            if it >= o.max_iter:
                status = MAX_ITER
                break
            # A-3: barrier parameter update (fast monotone decrease)
            while True:
                Emu, _, _, _ = self.opt_error(x, s, yc, yd, zL, zU, vU, Jb, cE, dI, mu)
                if Emu > o.kappa_eps * mu:
                    break
                mu_new = max(o.tol / 10.0, min(o.kappa_mu * mu, mu ** o.theta_mu))
                if mu_new >= mu:  # already at its floor tol / 10: the update is done
                    break
                mu = mu_new
                tau = max(o.tau_min, 1.0 - mu)
                filt = []
            # A-4: search direction
            sL, sU = self.slacks(x)
            sig_x = np.where(self.hasL, zL / sL, 0.0) + np.where(self.hasU, zU / sU, 0.0)
            sig_s = (vU / (-s))
            gphi, gphis = self.grad_phi(x, s, mu)
            rx = gphi + self.JT_times(Jb, yc, yd)  # residual of x-stationarity
            rs = gphis - yd                          # residual of s-stationarity
            rc = cE
            rdd = dI - s
            dw, dc = 0.0, 0.0
            ncorr = 0
            dw_trials = []
            while True:
                F = self.factor(x, yc, yd, sig_x, sig_s, dw, dc, Jb)
                dw_trials.append(dw)
                if self.on_factor is not None:
                    self.on_factor(F, dw, dc)
                want = (pr.n, pr.mE + pr.mI, 0)  # n counts the p design variables
                if F.inertia == want:
                    if dw > 0:
                        dw_last = dw
                    break
                ncorr += 1
                if F.inertia[2] > 0:
                    dc = o.dc_bar * mu ** o.kappa_c
                if dw == 0.0:
                    dw = o.dw_init if dw_last == 0.0 else max(o.dw_min, o.kappa_w_minus * dw_last)
                else:
                    dw = (o.kappa_w_plus_bar if dw_last == 0.0 else o.kappa_w_plus) * dw
                if dw > o.dw_max:
                    status = INERTIA_FAIL
                    break
            if status == INERTIA_FAIL:
                break
            self.n_inertia_corr += ncorr
            # reduced right-hand side (slack row eliminated)
            rhs_d = -rdd - rs / (sig_s + dw)
            dx, dyc, dyd = self.kkt_solve(F, -rx, -rc, rhs_d)
            ds = (dyd - rs) / (sig_s + dw)
            # bound multiplier steps
            dzL = np.where(self.hasL, mu / sL - zL - zL / sL * dx, 0.0)
            dzU = np.where(self.hasU, mu / sU - zU + zU / sU * dx, 0.0)
            dvU = mu / (-s) - vU + vU / (-s) * ds
            # A-5: line search
            alpha_max = self.ftb_primal(x, dx, s, ds, tau)
            alpha_z = self.ftb_dual([zL[self.hasL], zU[self.hasU], vU.reshape(-1)],
                                    [dzL[self.hasL], dzU[self.hasU], dvU.reshape(-1)], tau)
            th = self.theta(cE, dI, s)
            phi = self.barrier_phi(x, s, mu)
            gdx = float(gphi @ dx + (gphis * ds).sum())
            if gdx < 0 and th <= theta_min:
                amin = o.gamma_alpha * min(o.gamma_theta, o.gamma_phi * th / (-gdx),
                                           o.delta * th ** o.s_theta / (-gdx) ** o.s_phi)
            elif gdx < 0:
                amin = o.gamma_alpha * min(o.gamma_theta, o.gamma_phi * th / (-gdx))
            else:
                amin = o.gamma_alpha * o.gamma_theta
            alpha = alpha_max
            accepted = False
            nls = 0
            ftype = False
            while True:
                xt = x + alpha * dx
                st = s + alpha * ds
                cEt, dIt = self.eval_c(xt)
                tht = self.theta(cEt, dIt, st)
                phit = self.barrier_phi(xt, st, mu)
                nls += 1
                ok = np.isfinite(phit) and np.isfinite(tht) and tht < theta_max
                if ok:
                    for (ft, fp) in filt:
                        if tht >= ft and phit >= fp:
                            ok = False
                            break
                if ok:
                    m_a = alpha * gdx
                    switching = m_a < 0 and (-m_a) ** o.s_phi * alpha ** (1 - o.s_phi) > o.delta * th ** o.s_theta
                    if th <= theta_min and switching:
                        if phit <= phi + o.eta_phi * m_a:
                            accepted, ftype = True, True
                    else:
                        if tht <= (1 - o.gamma_theta) * th or phit <= phi - o.gamma_phi * th:
                            accepted, ftype = True, False
                if accepted:
                    break
                alpha *= 0.5
                if alpha < max(amin, ALPHA_FLOOR):
                    break
            if not accepted:
                status = LS_FAIL
                break
            # A-7: augment filter for h-type steps
            if not ftype:
                filt.append(((1 - o.gamma_theta) * th, phi - o.gamma_phi * th))
            # A-6: accept
            x, s = xt, st
            yc = yc + alpha * dyc
            yd = yd + alpha * dyd
            zL = zL + alpha_z * dzL
            zU = zU + alpha_z * dzU
            vU = vU + alpha_z * dvU
            cE, dI = cEt, dIt
            sL, sU = self.slacks(x)
            zL = np.where(self.hasL, np.maximum(np.minimum(zL, o.kappa_sigma * mu / sL), mu / (o.kappa_sigma * sL)), 0.0)
            zU = np.where(self.hasU, np.maximum(np.minimum(zU, o.kappa_sigma * mu / sU), mu / (o.kappa_sigma * sU)), 0.0)
            vU = np.maximum(np.minimum(vU, o.kappa_sigma * mu / (-s)), mu / (o.kappa_sigma * (-s)))
            Jb = self.jac_scaled(x)
            it += 1
            rec = dict(it=it, mu=mu, theta=th, phi=phi, alpha=alpha, alpha_z=alpha_z, ls=nls,
                       dw=dw, dc=dc, dw_trials=dw_trials, d=float(self.D[-1] * x[-1]), E0=E0)
            log.append(rec)
            if self.verbose:
                print(f"it {it:4d} mu {mu:9.2e} th {th:9.2e} a {alpha:9.2e} az {alpha_z:9.2e} "
                      f"ls {nls:2d} dw {dw:8.1e} d {self.D[-1] * x[-1]:.10f} E0 {E0:9.2e}", flush=True)
            if np.abs(x[np.isfinite(x)]).max() > 1e20:
                status = DIVERGING
                break
        x = self.D * x
        return IpmResult(status, it, float(E0), float(x[-1]), x, yc, yd, zL / self.D, zU / self.D, s, vU,
                         time.perf_counter() - t0, log, self.n_inertia_corr, self.max_lin_resid,
                         np.array(x[-pr.npar:]))


def solve(params, feeds, n_stages, opts=None, verbose=False, x0=None, yc0=None, yd0=None, on_factor=None,
          n_sections=1):
    torch.set_num_threads(1)
    prob = Problem(params, feeds, n_stages, n_sections)
    return OracleIPM(prob, opts, verbose, on_factor).solve(x0, yc0, yd0)
