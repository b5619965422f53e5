"""Pressure relations (eq. 7) with a specified pressure drop per stage, pinned
in the oracle.

The top stage is at the feed table's absorber pressure and every stage below
is dp higher (P_n = P_{n+1} + dp, P_N = P_top); the pressure enters the water
and CO2 equilibria (9a, 9b) and the hydraulic row (10b).  The pins recover the
pressure of every stage from the residual of its (9a) row, check that the
mass and energy rows do not see it, and check the closed-form optimum and the
IPM against each other with a drop: a higher pressure lower in the column
shrinks the gas volume flow there, so the diameter falls.
"""

import copy
import math

import numpy as np
import pytest
import torch

from absorber_inputs import CONFIGS
from oracle import ipm, simulate
from oracle import model as M


def _with_dp(params, dp):
    p = copy.deepcopy(params)
    p["dp_stage"] = dp
    return p


def _random_point(N, seed):
    rng = np.random.default_rng(seed)
    Z = np.empty((N, M.NV))
    Z[:, 0:9] = rng.uniform(0.01, 0.3, (N, 9))
    Z[:, 9:13] = rng.uniform(0.05, 0.5, (N, 4))
    Z[:, M.IL] = rng.uniform(30, 60, N)
    Z[:, M.IV] = rng.uniform(5, 15, N)
    Z[:, M.IT] = rng.uniform(300, 350, N)
    Z[:, M.IE:] = rng.uniform(-1, 1, (N, 5))
    return Z


def test_zero_drop_is_the_case_study(params):
    P0, P1 = M.OracleParams(params), M.OracleParams(_with_dp(params, 0.0))
    feed = CONFIGS["C1"].feeds(params)[2]
    Z = _random_point(6, 1)
    assert np.array_equal(M.constraints(Z[None], 0.8, feed[None], P0), M.constraints(Z[None], 0.8, feed[None], P1))


def test_stage_pressures_recovered_from_the_water_equilibrium(params):
    # (9a): P_n y_H2O - x_H2O Psat(T) = c  =>  P_n = (c + x_H2O Psat(T)) / y_H2O
    dp = 750.0
    P = M.OracleParams(_with_dp(params, dp))
    N = 7
    feed = CONFIGS["C1"].feeds(params)[1]
    Z = _random_point(N, 2)
    c = M.constraints(Z[None], 0.9, feed[None], P)[0]
    psat = np.exp(P.psat_a - P.psat_b / Z[:, M.IT])
    Pn = (c[:, 18] + Z[:, 8] * psat) / Z[:, M.NLIQ + 1]
    assert Pn[-1] == pytest.approx(feed[17], rel=1e-12)          # P_N = P_top
    assert np.allclose(Pn[:-1] - Pn[1:], dp, rtol=1e-9, atol=0.0)  # P_n = P_{n+1} + dp
    # the material, reaction, summation and energy rows do not depend on the pressure
    c0 = M.constraints(Z[None], 0.9, feed[None], M.OracleParams(params))[0]
    keep = [r for r in range(M.NR) if r not in (18, 19, 21)]
    assert np.array_equal(c[:, keep], c0[:, keep])
    # the hydraulic row sees V R T / P_n
    hyd = Z[:, M.IV] * P.R * Z[:, M.IT] / Pn - P.u_max * math.pi * 0.81 / 4.0
    assert np.allclose(c[:, 21], hyd, rtol=1e-12, atol=1e-14)


def test_pressure_derivatives_against_central_differences(params):
    P = M.OracleParams(_with_dp(params, 900.0))
    N = 4
    feed = CONFIGS["C1"].feeds(params)[0]
    Z = _random_point(N, 3)
    d = 0.7
    J = M.jacobian(Z, d, feed, P)
    w = np.r_[Z.reshape(-1), d]
    h = 1e-6 * np.maximum(np.abs(w), 1.0)
    for j in np.random.default_rng(4).choice(w.size, 12, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[j] += h[j]
        wm[j] -= h[j]
        cp = M.constraints(wp[:-1].reshape(1, N, M.NV), wp[-1], feed[None], P)[0].reshape(-1)
        cm = M.constraints(wm[:-1].reshape(1, N, M.NV), wm[-1], feed[None], P)[0].reshape(-1)
        fd = (cp - cm) / (2 * h[j])
        scale = np.abs(J).max(axis=1) + 1e-300
        assert np.all(np.abs(fd - J[:, j]) <= 1e-6 * scale), j


@pytest.fixture(scope="module")
def c1_with_drop(params):
    w = CONFIGS["C1"]
    F = w.feeds(params)
    p = _with_dp(params, 2000.0)
    d_dp, _, Zs_dp, ok_dp = simulate.closed_form_diameter(F, w.n_stages, p)
    d_0, _, _, ok_0 = simulate.closed_form_diameter(F, w.n_stages, params)
    r = ipm.solve(p, F, w.n_stages)
    return w, F, p, d_dp, Zs_dp, ok_dp, d_0, ok_0, r


def test_drop_shrinks_the_closed_form_diameter(c1_with_drop):
    w, F, p, d_dp, Zs, ok_dp, d_0, ok_0, r = c1_with_drop
    assert ok_dp.all() and ok_0.all()
    # the largest hydraulic diameter sits low in the column, where the pressure
    # is now up to (N-1) dp higher: a smaller volume flow, a smaller diameter
    assert d_dp < d_0
    assert d_dp > d_0 * math.sqrt(F[:, 17].min() / (F[:, 17].max() + (w.n_stages - 1) * 2000.0)) * 0.9


def test_ipm_with_drop_reaches_the_closed_form(c1_with_drop):
    w, F, p, d_dp, Zs, ok_dp, d_0, ok_0, r = c1_with_drop
    assert r.status == ipm.SUCCESS and r.E0 <= 1e-8 and r.max_lin_resid <= 1e-10
    assert abs(r.d - d_dp) / d_dp <= 1e-6
    Z = r.x[:-1].reshape(F.shape[0], w.n_stages, M.NV)
    assert np.abs(Z - Zs).max() / np.abs(Zs).max() < 1e-8
