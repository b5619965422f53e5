"""Oracle interior-point solutions against closed forms, invariants and
invariances (the optimum of problem (10) is pinned without the oracle IPM)."""

import math

import numpy as np
import pytest

from absorber_inputs import CONFIGS, feed_table
from oracle import ipm
from oracle import model as M
from oracle import simulate


@pytest.fixture(scope="module")
def c1(params):
    w = CONFIGS["C1"]
    F = w.feeds(params)
    res = ipm.solve(params, F, w.n_stages)
    dstar, dw, Zs, ok = simulate.closed_form_diameter(F, w.n_stages, params)
    return w, F, res, dstar, dw, Zs, ok


def test_c1_converges_to_tolerance(c1):
    w, F, res, *_ = c1
    assert res.status == ipm.SUCCESS
    assert res.E0 <= 1e-8
    assert res.max_lin_resid <= 1e-10


def test_c1_diameter_equals_closed_form(c1):
    # d* = max_{n,w} sqrt(4 V R T / (pi u_max P)) from independent MESH solves
    w, F, res, dstar, dw, Zs, ok = c1
    assert ok.all()
    assert abs(res.d - dstar) / dstar <= 1e-6


def test_c1_states_equal_simulation(c1):
    w, F, res, dstar, dw, Zs, ok = c1
    Z = res.x[:-1].reshape(F.shape[0], w.n_stages, M.NV)
    assert np.abs(Z - Zs).max() / np.abs(Zs).max() < 1e-9


def test_c1_min_hydraulic_margin_is_zero(c1, params):
    # sanity check of the numerical results: the hydraulic constraint is active
    w, F, res, *_ = c1
    P = M.OracleParams(params)
    Z = res.x[:-1].reshape(F.shape[0], w.n_stages, M.NV)
    g = Z[:, :, M.IV] * P.R * Z[:, :, M.IT] / F[:, 17][:, None] - P.u_max * math.pi * res.d ** 2 / 4
    area = P.u_max * math.pi * res.d ** 2 / 4
    assert abs(g.max()) / area < 1e-7


def test_c1_column_closure(c1, params):
    # summing (1) over stages telescopes to in = out for every reaction
    # invariant a (a^T nu = 0); the enthalpy closure of (6) is pinned in
    # test_oracle_rows.py (test_column_enthalpy_closure)
    w, F, res, *_ = c1
    P = M.OracleParams(params)
    nu = P.nu.numpy()
    Z = res.x[:-1].reshape(F.shape[0], w.n_stages, M.NV)
    basis = np.linalg.svd(nu.T)[2][np.linalg.matrix_rank(nu):]  # null space of nu^T
    for s in range(F.shape[0]):
        f = F[s]
        liq_in = np.r_[f[7:16], 0, 0] * f[6]
        gas_in = np.r_[np.zeros(7), f[1:5]] * f[0]
        liq_out = np.r_[Z[s, 0, 0:9], 0, 0] * Z[s, 0, M.IL]
        gas_out = np.r_[np.zeros(7), Z[s, -1, 9:13]] * Z[s, -1, M.IV]
        flow_in, flow_out = basis @ (liq_in + gas_in), basis @ (liq_out + gas_out)
        assert np.abs(flow_in - flow_out).max() < 1e-9 * np.abs(flow_in).max()
        # summations (4)
        assert np.abs(Z[s, :, 0:9].sum(axis=1) - 1).max() < 1e-12
        assert np.abs(Z[s, :, 9:13].sum(axis=1) - 1).max() < 1e-12


def test_c1_diameter_multiplier_closed_form(c1):
    # dL/dd = 0 with inactive diameter bounds: sum of the hydraulic multipliers
    # (of the unscaled rows) equals 2 / (pi u_max d*)
    w, F, res, *_ = c1
    prob = ipm.Problem(__import__("absorber_inputs").load_params(), F, w.n_stages)
    o = ipm.OracleIPM(prob)
    o.compute_scaling(o.push_into_bounds(prob.initial_point() / o.D, 1e-2, 1e-2))
    lam = (res.yd * o.cs[:, :, -1]).sum()
    assert lam == pytest.approx(2.0 / (math.pi * o.pr.P.u_max * res.d), rel=1e-6)


def test_identical_scenarios_give_single_scenario_diameter(params):
    pert = np.array([[0.05, -0.03, 0.02]])
    F1 = feed_table(pert, params)
    F3 = feed_table(np.repeat(pert, 3, axis=0), params)
    r1 = ipm.solve(params, F1, 4)
    r3 = ipm.solve(params, F3, 4)
    assert r1.status == ipm.SUCCESS and r3.status == ipm.SUCCESS
    d1 = simulate.closed_form_diameter(F1, 4, params)[0]
    assert abs(r1.d - d1) / d1 < 1e-6
    assert abs(r3.d - r1.d) / r1.d < 1e-6


def test_scenario_permutation_leaves_diameter(params):
    pert = np.array([[0.08, -0.05, 0.10], [-0.1, 0.1, -0.05]])
    Fa = feed_table(pert, params)
    Fb = feed_table(pert[::-1], params)
    ra = ipm.solve(params, Fa, 3)
    rb = ipm.solve(params, Fb, 3)
    assert ra.status == ipm.SUCCESS and rb.status == ipm.SUCCESS
    assert abs(ra.d - rb.d) / ra.d < 1e-9
    Za = ra.x[:-1].reshape(2, 3, M.NV)
    Zb = rb.x[:-1].reshape(2, 3, M.NV)
    assert np.abs(Za - Zb[::-1]).max() / np.abs(Za).max() < 1e-9
