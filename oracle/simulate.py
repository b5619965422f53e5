"""Oracle process simulation and the closed-form optimal diameter.

TEST INFRASTRUCTURE ONLY (see oracle/model.py).

Once the feeds, heat duty and pressure are fixed, the MESH equations of a
scenario form a square system (Equilibrium process model, degrees of freedom).
Problem (10) fixes every inlet stream per scenario (Case study, problem setup),
so each scenario's states are determined by its own MESH solve and do not
depend on d.  The hydraulic rows (10b) then only bound d from below and the
objective (10a) pushes d down, so the optimum has the plain definition

    d* = max over scenarios w and stages n of sqrt(4 V R T / (pi u_max P)),

with (V, T) taken from each scenario's MESH solution.  This module computes it
by a damped Newton method on each scenario's square MESH system, with the
Jacobian from the autograd library.  It is independent of the interior-point
code: it solves F_w = 0 directly and never touches d, multipliers or barriers.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from . import model as M


def _log_mask(N):
    """Mole fractions (locals 0-12) are solved for in log form, the rest as is."""
    m = np.zeros(M.NV, dtype=bool)
    m[0:13] = True
    return np.tile(m, N)


def simulate_scenario(Z0: np.ndarray, feed: np.ndarray, P: M.OracleParams, tol: float = 1e-13,
                      max_iter: int = 100):
    """Solve the square MESH system of one scenario from Z0 (N, 21).

    Newton's method on F(Z) = 0 with the mole fractions carried as their
    logarithms (this keeps them positive and leaves the solution unchanged), the
    rows scaled by their Jacobian row maxima at the start, log-steps capped at 5
    and backtracking on the scaled residual inf-norm (stopping when even a step
    of 1e-10 gives no decrease).
    Returns (Z, converged, iterations, final scaled residual inf-norm).
    """
    N = Z0.shape[0]
    ft = torch.from_numpy(np.ascontiguousarray(feed, dtype=np.float64))
    lm = torch.from_numpy(_log_mask(N))
    one = torch.tensor(1.0, dtype=torch.float64)

    def to_z(u):
        return torch.where(lm, torch.exp(u), u)

    def F(u):
        c = M.scenario_constraints(to_z(u).reshape(N, M.NV), one, ft, P)
        return c[:, :M.NR - 1].reshape(-1)

    z0 = np.ascontiguousarray(Z0, dtype=np.float64).reshape(-1)
    u = torch.from_numpy(np.where(_log_mask(N), np.log(np.maximum(z0, 1e-300)), z0))
    jac = torch.func.jacfwd(F)
    rs = 1.0 / jac(u).abs().max(dim=1).values
    r = F(u) * rs
    nr = float(r.abs().max())
    it = 0
    for it in range(max_iter):
        if nr <= tol:
            break
        du = torch.linalg.solve(jac(u) * rs[:, None], -r)
        a = 1.0
        big = float(du[lm].abs().max())
        if big > 5.0:
            a = 5.0 / big
        stalled = False
        while True:
            ut = u + a * du
            rt = F(ut) * rs
            nt = float(rt.abs().max())
            if math.isfinite(nt) and nt < (1.0 - 1e-4 * a) * nr:
                break
            if a < 1e-10:  # no decrease even for a tiny step: give up
                stalled = True
                break
            a *= 0.5
        u, r, nr = ut, rt, nt
        if stalled:
            break
    return to_z(u).reshape(N, M.NV).numpy(), nr <= tol, it, nr


def hydraulic_diameter(Z: np.ndarray, feed: np.ndarray, P: M.OracleParams) -> float:
    """Smallest d meeting (10b) on every stage of one simulated scenario."""
    V, T = Z[:, M.IV], Z[:, M.IT]
    Pn = M.stage_pressures(feed[17], Z.shape[0], P)
    return float(np.sqrt(4.0 * V * P.R * T / (math.pi * P.u_max * Pn)).max())


def closed_form_diameter(feeds: np.ndarray, n_stages: int, params: dict, Z0=None):
    """d* = max_w d_w over independently simulated scenarios.

    Z0 may hold per-scenario starting points (S, N, 21); by default every
    scenario starts from the cold point.  Returns (d*, per-scenario d, states,
    converged flags).
    """
    P = M.OracleParams(params)
    S = feeds.shape[0]
    if Z0 is None:
        ip = params["initial_point"]
        z = np.zeros(M.NV)
        z[0:9] = ip["x"]
        z[9:13] = ip["y"]
        z[M.IL], z[M.IV], z[M.IT] = ip["L"], ip["V"], ip["T"]
        Z0 = np.broadcast_to(z, (S, n_stages, M.NV))
    ds, Zs, ok = np.empty(S), np.empty((S, n_stages, M.NV)), np.empty(S, dtype=bool)
    for w in range(S):
        Z, conv, _, _ = simulate_scenario(Z0[w], feeds[w], P)
        Zs[w], ok[w] = Z, conv
        ds[w] = hydraulic_diameter(Z, feeds[w], P)
    return float(ds.max()), ds, Zs, ok


def closed_form_sections(feeds: np.ndarray, n_stages: int, n_sections: int, params: dict, Z0=None):
    """theta_k* = the largest hydraulic diameter over the stages of section k of
    every independently simulated scenario (the optimum of the section-diameter
    design problem: each section's diameter is bounded below only by its own
    stages' hydraulic rows, and the design cost increases in each of them).
    Returns (theta* (p,), states, converged flags)."""
    P = M.OracleParams(params)
    _, _, Zs, ok = closed_form_diameter(feeds, n_stages, params, Z0)
    V, T = Zs[:, :, M.IV], Zs[:, :, M.IT]
    Pn = np.stack([M.stage_pressures(f[17], n_stages, P) for f in feeds])  # (S, N)
    dh = np.sqrt(4.0 * V * P.R * T / (math.pi * P.u_max * Pn))  # (S, N)
    sec = M.sections(n_stages, n_sections)
    theta = np.array([dh[:, sec == k].max() for k in range(n_sections)])
    return theta, Zs, ok


def closed_form_design(feeds: np.ndarray, n_stages: int, n_sections: int, params: dict, Z0=None):
    """Optimum of the design problem with the operating cost of eq. (8a): each
    section's objective term c_k theta_k + a_k theta_k^-4 is convex and its
    only lower bound is the section's hydraulic minimum, so theta_k* =
    max(theta_hyd,k, (4 a_k / c_k)^(1/5)), clipped to the diameter bounds.
    Returns (theta* (p,), states, converged flags)."""
    P = M.OracleParams(params)
    th_h, Zs, ok = closed_form_sections(feeds, n_stages, n_sections, params, Z0)
    a = M.operating_coefficients(feeds, n_stages, n_sections, P)
    c = M.section_weights(n_stages, n_sections)
    th = np.maximum(th_h, (4.0 * a / c) ** 0.2)
    lo, hi = params["bounds"]["d"]
    return np.clip(th, lo, hi), Zs, ok
