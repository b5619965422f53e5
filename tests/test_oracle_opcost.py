"""The operating-cost term of the scenario NLP (eq. 8a), pinned in the oracle.

The expected blower cost sum_w p_w C^op_w falls with the diameter as theta^-4
while the design cost rises linearly, so the optimum of each section diameter is
max(theta_hyd, (4 a_k / c_k)^(1/5)): the hydraulic bound when the blower is
cheap, an interior point (all hydraulic rows inactive) when it is dear.  The pins
rebuild the blower power stage by stage from its definition, check the oracle's
scaled objective derivatives against differences, and solve both regimes.
"""

import copy
import math

import numpy as np
import pytest

from absorber_inputs import CONFIGS
from oracle import ipm, simulate
from oracle import model as M


def _with_weight(params, weight, dp=None):
    p = copy.deepcopy(params)
    p["operating_cost"]["weight"] = weight
    if dp is not None:
        p["dp_stage"] = dp
    return p


def test_blower_power_from_its_definition(params):
    # stage by stage: volume flow at the inlet pressure, density of the inlet gas,
    # superficial velocity in the stage's section, loss K rho u^2 / 2 times the flow
    p = _with_weight(params, 0.37, dp=500.0)
    P = M.OracleParams(p)
    F = CONFIGS["C2"].feeds(p)[:9]
    N, q = 7, 3
    th = np.array([0.55, 0.8, 1.1])
    sec = M.sections(N, q)
    Mg = np.array(p["operating_cost"]["molar_mass"])
    K = p["operating_cost"]["loss_coef"]
    total = 0.0
    for f in F:
        p_in = f[17] + (N - 1) * 500.0
        Q = f[0] * P.R * f[5] / p_in
        rho = p_in * float(f[1:5] @ Mg) / (P.R * f[5])
        W = 0.0
        for n in range(N):
            u = Q / (math.pi * th[sec[n]] ** 2 / 4.0)
            W += Q * K * rho * u * u / 2.0
        total += 0.37 * W / F.shape[0]
    a = M.operating_coefficients(F, N, q, P)
    assert float(np.sum(a * th ** -4.0)) == pytest.approx(total, rel=1e-13)
    # the case study has no operating cost
    assert np.all(M.operating_coefficients(F, N, q, M.OracleParams(params)) == 0.0)


def test_scaled_objective_derivatives(params):
    p = _with_weight(params, 0.5)
    F = CONFIGS["C1"].feeds(p)
    prob = ipm.Problem(p, F, 8, 2)
    o = ipm.OracleIPM(prob)
    x = o.push_into_bounds(prob.initial_point() / o.D, 1e-2, 1e-2)
    o.compute_scaling(x)
    x[-2:] = [0.7, 0.9]

    def f(xx):
        th = o.D[-2:] * xx[-2:]
        return o.sf * float(prob.c @ th + np.sum(prob.a * th ** -4.0))

    g, hf = o.grad_f(x), o.hess_f(x)
    assert np.all(g[:-2] == 0.0)
    for k in (1, 2):
        h = 1e-5
        e = np.zeros_like(x)
        e[-k] = h
        assert g[-k] == pytest.approx((f(x + e) - f(x - e)) / (2 * h), rel=1e-7)
        assert hf[-k] == pytest.approx((f(x + e) - 2 * f(x) + f(x - e)) / h ** 2, rel=1e-4)
        assert f(x) - o.sf * float(prob.c @ (o.D[-2:] * x[-2:])) == pytest.approx(o.f_nonlinear(x), rel=1e-13)


@pytest.fixture(scope="module")
def c1_hydraulic(params):
    w = CONFIGS["C1"]
    F = w.feeds(params)
    dstar, _, Zs, ok = simulate.closed_form_diameter(F, w.n_stages, params)
    a1 = M.operating_coefficients(F, w.n_stages, 1, M.OracleParams(_with_weight(params, 1.0)))[0]
    return w, F, dstar, Zs, ok, a1


def test_dear_blower_moves_the_optimum_inside(params, c1_hydraulic):
    w, F, dstar, Zs, ok, a1 = c1_hydraulic
    # the weight that puts the blower optimum 30% above the hydraulic bound
    weight = (1.3 * dstar) ** 5 / (4.0 * a1)
    p = _with_weight(params, weight)
    th, _, _ = simulate.closed_form_design(F, w.n_stages, 1, p)
    assert th[0] == pytest.approx(1.3 * dstar, rel=1e-12)
    r = ipm.solve(p, F, w.n_stages)
    assert r.status == ipm.SUCCESS and r.E0 <= 1e-8 and r.max_lin_resid <= 1e-10
    assert abs(r.d - th[0]) / th[0] <= 1e-6
    # every hydraulic row is slack, so its multiplier vanishes (up to the barrier)
    prob = ipm.Problem(p, F, w.n_stages)
    o = ipm.OracleIPM(prob)
    o.compute_scaling(o.push_into_bounds(prob.initial_point() / o.D, 1e-2, 1e-2))
    lam = r.yd * o.cs[:, :, -1]
    assert np.abs(lam).sum() <= 1e-6 * 2.0 / (math.pi * params["u_max"] * dstar)
    Z = r.x[:-1].reshape(F.shape[0], w.n_stages, M.NV)
    assert np.abs(Z - Zs).max() / np.abs(Zs).max() < 1e-8


def test_cheap_blower_keeps_the_hydraulic_optimum(params, c1_hydraulic):
    w, F, dstar, Zs, ok, a1 = c1_hydraulic
    weight = 0.5 * dstar ** 5 / (4.0 * a1)  # blower optimum below the hydraulic bound
    p = _with_weight(params, weight)
    r = ipm.solve(p, F, w.n_stages)
    assert r.status == ipm.SUCCESS and abs(r.d - dstar) / dstar <= 1e-6
    # dL/dd = 0: the hydraulic multipliers now balance c - 4 a d^-5 instead of c
    prob = ipm.Problem(p, F, w.n_stages)
    o = ipm.OracleIPM(prob)
    o.compute_scaling(o.push_into_bounds(prob.initial_point() / o.D, 1e-2, 1e-2))
    lam = r.yd * o.cs[:, :, -1]
    a = prob.a[0]
    want = 2.0 * (1.0 - 4.0 * a * r.d ** -5.0) / (math.pi * params["u_max"] * r.d)
    assert 0.0 < want < 2.0 / (math.pi * params["u_max"] * r.d)
    assert lam.sum() == pytest.approx(want, rel=1e-6)


def test_sections_with_operating_cost(params, c1_hydraulic):
    w, F, dstar, Zs, ok, a1 = c1_hydraulic
    th_h, _, _ = simulate.closed_form_sections(F, w.n_stages, 2, params)
    # a weight between the two sections' thresholds: one section interior, one on its bound
    c = M.section_weights(w.n_stages, 2)
    a_unit = M.operating_coefficients(F, w.n_stages, 2, M.OracleParams(_with_weight(params, 1.0)))
    thr = c * th_h ** 5 / (4.0 * a_unit)  # weight at which each section's blower optimum meets its bound
    weight = float(np.sqrt(thr.min() * thr.max())) if thr.max() > 1.05 * thr.min() else 2.0 * thr.max()
    p = _with_weight(params, weight)
    th, _, _ = simulate.closed_form_design(F, w.n_stages, 2, p)
    r = ipm.solve(p, F, w.n_stages, n_sections=2)
    assert r.status == ipm.SUCCESS and r.E0 <= 1e-8
    assert np.abs(r.theta - th).max() / th.max() <= 1e-6
    assert np.any(th > th_h * (1 + 1e-3))
