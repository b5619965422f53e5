"""Oracle model: the equilibrium absorber constraints of one scenario, in plain
PyTorch CPU float64.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.

The residuals follow the paper's equations directly:

* material balance, eq. (1), with zero side feeds;
* reaction equilibrium in activities, eq. (3a), with ideal-liquid activities
  a_i = x_i (Case study, thermodynamics paragraph) and the Kent-Eisenberg form
  of ln K_r(T);
* summations, eq. (4);
* Raoult's law for water, eq. (9a), and Henry's law for CO2, eq. (9b);
* stage energy balance, eq. (6), with Q_n = 0 and the ideal-mixture enthalpies
  of the case study (component enthalpy from a reference value plus the heat
  capacity integral);
* the hydraulic superficial-velocity constraint, eq. (10b).

Exact first and second derivatives come from the autograd library
(``torch.func.jacfwd`` and ``torch.func.hessian``) applied to these residuals,
so the oracle carries no hand-derived derivative.

Local layout of one stage (21 free variables):
  0-8   x of MEA, MEAH+, H+, MEACOO-, HCO3-, OH-, CO3--, CO2, H2O
  9-12  y of CO2, H2O, N2, O2
  13 L, 14 V, 15 T, 16-20 reaction extents eps_1..eps_5
The 9 fixed variables (y of the 7 non-volatile species, x of N2 and O2) are
zero and do not appear.

Row layout of one stage (22 rows):
  0-10  material balances of the 11 species, eq. (1)
  11-15 reaction equilibria R1..R5, eq. (3a)
  16    liquid summation, 17 vapour summation, eq. (4)
  18    water VLE (9a), 19 CO2 VLE (9b)
  20    energy balance (6)
  21    hydraulic inequality (10b), g <= 0
"""

from __future__ import annotations

import math

import numpy as np
import torch

NV = 21  # free variables per stage
NR = 22  # rows per stage (21 MESH equalities + 1 hydraulic inequality)
NLIQ = 9
NVAP = 4
IL, IV, IT, IE = 13, 14, 15, 16


class OracleParams:
    """Constants of params.json as float64 tensors."""

    def __init__(self, p: dict):
        f = lambda a: torch.tensor(a, dtype=torch.float64)  # noqa: E731
        self.nu = f(p["nu"])  # (11, 5)
        self.A, self.B = f(p["lnK_A"]), f(p["lnK_B"])
        self.C, self.D = f(p["lnK_C"]), f(p["lnK_D"])
        self.psat_a, self.psat_b = float(p["psat_a"]), float(p["psat_b"])
        self.lnH298 = float(p["henry_lnH298"])
        self.kH = float(p["henry_kappa"])
        self.TH = float(p["henry_Tref"])
        self.lnrMEA = float(p["henry_ln_ratio_MEA"])
        self.Tref = float(p["Tref"])
        self.hL_ref, self.cpL_a, self.cpL_b = f(p["hL_ref"]), f(p["cpL_a"]), f(p["cpL_b"])
        self.hV_ref, self.cpV_a, self.cpV_b = f(p["hV_ref"]), f(p["cpV_a"]), f(p["cpV_b"])
        self.R = float(p["R"])
        self.u_max = float(p["u_max"])
        # specified pressure drop per stage of the pressure relations (eq. 7); 0 in the case study
        self.dp = float(p.get("dp_stage", 0.0))
        # expected blower cost of the scenario NLP's operating term (eq. 8a); weight 0 in the case study
        op = p.get("operating_cost", {})
        self.op_weight = float(op.get("weight", 0.0))
        self.op_loss = float(op.get("loss_coef", 0.0))
        self.op_M = np.asarray(op.get("molar_mass", [0.0, 0.0, 0.0, 0.0]), dtype=np.float64)
        self.raw = p


def sections(n_stages: int, n_sections: int) -> np.ndarray:
    """Section of every stage (0 = bottom) for a column cut into n_sections
    contiguous sections of near-equal height: stage n is in section n p // N."""
    return np.array([(n * n_sections) // n_stages for n in range(n_stages)], dtype=np.int64)


def section_weights(n_stages: int, n_sections: int) -> np.ndarray:
    """Weight of each section diameter in the design cost: its share of the stages
    (the shell of a section scales with its height times its diameter)."""
    return np.bincount(sections(n_stages, n_sections), minlength=n_sections) / float(n_stages)


def stage_pressures(p_top, n_stages: int, P: OracleParams):
    """Stage pressures of the pressure relations (7) with a specified drop per
    stage: the top stage (index N-1) is at p_top (the feed table's absorber
    pressure) and each stage below is dp higher, P_n = P_{n+1} + dp.  Returns
    (N,) bottom to top (a tensor when p_top is one, else an array)."""
    k = np.arange(n_stages - 1, -1, -1, dtype=np.float64)  # stages above stage n
    if isinstance(p_top, torch.Tensor):
        return p_top + torch.from_numpy(k) * P.dp
    return float(p_top) + k * P.dp


def operating_coefficients(feeds: np.ndarray, n_stages: int, n_sections: int, P: OracleParams) -> np.ndarray:
    """Coefficients a_k of the expected operating cost sum_w p_w C^op_w = sum_k a_k theta_k^-4 (eq. 8a).

    C^op_w is the weight times the blower power of scenario w: the inlet gas (flow
    V_0, temperature T_gas, molar mass M_w of its composition) enters at the
    bottom stage's pressure P_in (eq. 7), with volume flow Q = V_0 R T_gas / P_in
    and density rho = P_in M_w / (R T_gas); each stage of section k loses
    loss_coef rho u^2 / 2 at the superficial velocity u = Q / (pi theta_k^2 / 4),
    so the power is sum_k N_k (8 loss_coef / pi^2) rho Q^3 / theta_k^4.  The
    scenarios are equally likely (p_w = 1 / S).  Returns (p,)."""
    feeds = np.asarray(feeds, dtype=np.float64)
    Nk = np.bincount(sections(n_stages, n_sections), minlength=n_sections).astype(np.float64)
    p_in = np.array([stage_pressures(f[17], n_stages, P)[0] for f in feeds])
    Q = feeds[:, 0] * P.R * feeds[:, 5] / p_in
    rho = p_in * (feeds[:, 1:5] @ P.op_M) / (P.R * feeds[:, 5])
    return P.op_weight * 8.0 * P.op_loss * Nk / math.pi ** 2 * float(np.mean(rho * Q ** 3))


def _h(T, href, a, b, Tref):
    """Component molar enthalpy h(T) = href + int_Tref^T (a + b t) dt, for T (...,)."""
    T = T[..., None]
    return href + a * (T - Tref) + 0.5 * b * (T * T - Tref * Tref)


def scenario_constraints(Z: torch.Tensor, d: torch.Tensor, feed: torch.Tensor, P: OracleParams,
                         sec: torch.Tensor | None = None) -> torch.Tensor:
    """All 22 rows of every stage of one scenario.

    Z: (N, 21) free variables, stages bottom (index 0) to top; d: scalar tensor
    (the diameter), or with sec the (p,) section diameters theta and sec (N,)
    the section of each stage (general design vector of the scenario NLP);
    feed: (18,) feed-table row.  Returns (N, 22).
    """
    x, y = Z[:, 0:NLIQ], Z[:, NLIQ:NLIQ + NVAP]
    L, V, T, eps = Z[:, IL], Z[:, IV], Z[:, IT], Z[:, IE:IE + 5]
    Pabs = stage_pressures(feed[17], Z.shape[0], P)

    # stream entering each stage from above (liquid) and from below (vapour)
    L_up = torch.cat([L[1:], feed[6:7]])
    x_up = torch.cat([x[1:], feed[7:16][None, :]], dim=0)
    T_up = torch.cat([T[1:], feed[16:17]])
    V_dn = torch.cat([feed[0:1], V[:-1]])
    y_dn = torch.cat([feed[1:5][None, :], y[:-1]], dim=0)
    T_dn = torch.cat([feed[5:6], T[:-1]])

    n = Z.shape[0]
    zero2 = torch.zeros((n, 2), dtype=Z.dtype)
    zero7 = torch.zeros((n, 7), dtype=Z.dtype)
    X = torch.cat([x, zero2], dim=1)  # 11 species, N2 and O2 fixed to 0
    Xup = torch.cat([x_up, zero2], dim=1)
    Y = torch.cat([zero7, y], dim=1)  # 11 species, non-volatiles fixed to 0
    Ydn = torch.cat([zero7, y_dn], dim=1)

    # (1) material balance: out - in - generation
    mb = L[:, None] * X + V[:, None] * Y - L_up[:, None] * Xup - V_dn[:, None] * Ydn - eps @ P.nu.T

    # (3a) ideal activities a_i = x_i, Kent-Eisenberg ln K_r(T)
    lnK = P.A + P.B / T[:, None] + P.C * torch.log(T)[:, None] + P.D * T[:, None]
    rx = torch.log(x) @ P.nu[:NLIQ, :] - lnK

    # (4) summations
    sl = x.sum(dim=1) - 1.0
    sv = y.sum(dim=1) - 1.0

    # (9a) Raoult's law for water, (9b) Henry's law for CO2 (c_CO2 read as x_CO2)
    psat = torch.exp(P.psat_a - P.psat_b / T)
    vle_w = Pabs * y[:, 1] - x[:, 8] * psat
    amine = x[:, 0] + x[:, 1] + x[:, 3]
    xapp_mea = amine / (amine + x[:, 8])
    lnH = P.lnH298 + P.kH * (1.0 / P.TH - 1.0 / T) + xapp_mea * P.lnrMEA
    vle_c = Pabs * y[:, 0] - x[:, 7] * torch.exp(lnH)

    # (6) energy balance with ideal-mixture enthalpies, Q = 0
    hL = lambda xx, TT: (xx * _h(TT, P.hL_ref, P.cpL_a, P.cpL_b, P.Tref)).sum(dim=-1)  # noqa: E731
    hV = lambda yy, TT: (yy * _h(TT, P.hV_ref, P.cpV_a, P.cpV_b, P.Tref)).sum(dim=-1)  # noqa: E731
    eb = L * hL(x, T) + V * hV(y, T) - L_up * hL(x_up, T_up) - V_dn * hV(y_dn, T_dn)

    # (10b) hydraulic: volumetric gas flow against the velocity limit of the
    # stage's own diameter
    dn = d if sec is None else d[sec]
    hyd = V * P.R * T / Pabs - P.u_max * math.pi * dn * dn / 4.0

    return torch.cat([mb, rx, sl[:, None], sv[:, None], vle_w[:, None], vle_c[:, None],
                      eb[:, None], hyd[:, None]], dim=1)


def _design(d):
    """Design variables as a 1-D float64 array: (1,) for a scalar diameter, (p,) for sections."""
    return np.atleast_1d(np.asarray(d, dtype=np.float64))


def _flat(P, feed, N, p=1):
    """Rows of one scenario as a function of w = (Z flat, design variables (p))."""
    sec = None if p == 1 else torch.from_numpy(sections(N, p))

    def fn(w):
        Z = w[:-p].reshape(N, NV)
        d = w[-1] if p == 1 else w[-p:]
        return scenario_constraints(Z, d, feed, P, sec).reshape(-1)
    return fn


def constraints(Zall: np.ndarray, d, feeds: np.ndarray, P: OracleParams) -> np.ndarray:
    """c for all scenarios: Zall (S, N, 21), d the diameter or the (p,) section
    diameters, feeds (S, 18) -> (S, N, 22)."""
    S, N, _ = Zall.shape
    th = _design(d)
    p = th.size
    out = np.empty((S, N, NR))
    dt = torch.tensor(float(th[0]), dtype=torch.float64) if p == 1 else torch.from_numpy(th)
    sec = None if p == 1 else torch.from_numpy(sections(N, p))
    for w in range(S):
        out[w] = scenario_constraints(torch.from_numpy(np.ascontiguousarray(Zall[w])), dt,
                                      torch.from_numpy(feeds[w]), P, sec).numpy()
    return out


def _wvec(Zs, d):
    return torch.cat([torch.from_numpy(np.ascontiguousarray(Zs)).reshape(-1), torch.from_numpy(_design(d))])


def jacobian(Zs: np.ndarray, d, feed: np.ndarray, P: OracleParams) -> np.ndarray:
    """Dense Jacobian of one scenario's 22N rows w.r.t. its 21N variables and the
    design variables (d, or the p section diameters).

    Returns (22N, 21N + p); the last p columns are the design derivatives.
    """
    N = Zs.shape[0]
    p = _design(d).size
    return torch.func.jacfwd(_flat(P, torch.from_numpy(feed), N, p))(_wvec(Zs, d)).numpy()


def lagrangian_hessian(Zs: np.ndarray, d, feed: np.ndarray, lam: np.ndarray, P: OracleParams) -> np.ndarray:
    """Dense Hessian of sum_j lam_j c_j (one scenario) w.r.t. (Z, design): (21N+p, 21N+p)."""
    N = Zs.shape[0]
    p = _design(d).size
    f = _flat(P, torch.from_numpy(feed), N, p)
    lt = torch.from_numpy(np.ascontiguousarray(lam).reshape(-1))
    H = torch.func.hessian(lambda v: (lt * f(v)).sum())(_wvec(Zs, d)).numpy()
    return 0.5 * (H + H.T)  # forward-over-reverse AD is symmetric up to rounding


def row_hessian(Zs: np.ndarray, d: float, feed: np.ndarray, row: int, P: OracleParams) -> np.ndarray:
    """Hessian of a single flattened row index of one scenario."""
    lam = np.zeros(Zs.shape[0] * NR)
    lam[row] = 1.0
    return lagrangian_hessian(Zs, d, feed, lam, P)
