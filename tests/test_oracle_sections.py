"""The general design vector of the scenario NLP (eq. 8: shared design variables
theta in R^p, replicated scenario blocks), built as one diameter per column
section, pinned in the oracle.

With p sections every stage's hydraulic row (10b) uses its section's diameter
and the design cost is sum_k (N_k / N) theta_k.  The scenario states do not
depend on theta (square MESH blocks), so the optimum has a closed form: theta_k*
is the largest hydraulic diameter over the stages of section k of all
independently simulated scenarios.  The KKT system gains a p-column border and
a dense p x p Schur complement, checked against dense linear algebra.
"""

import math

import numpy as np
import pytest

from absorber_inputs import CONFIGS, feed_table, perturbations
from oracle import ipm, simulate
from oracle import model as M
from oracle.kkt import BorderedKKT, scenario_kkt


def test_sections_split_the_column_evenly():
    for N, p in ((8, 2), (10, 3), (60, 4), (9, 1)):
        sec = M.sections(N, p)
        counts = np.bincount(sec, minlength=p)
        assert sec[0] == 0 and sec[-1] == p - 1 and np.all(np.diff(sec) >= 0)
        assert counts.max() - counts.min() <= 1
        assert M.section_weights(N, p).sum() == pytest.approx(1.0)


def test_one_section_is_the_paper_problem(params):
    # p = 1 reproduces the rows and derivatives of the single-diameter model exactly
    P = M.OracleParams(params)
    rng = np.random.default_rng(3)
    Z = np.abs(rng.normal(0.2, 0.05, (3, M.NV))) + 0.01
    Z[:, M.IL], Z[:, M.IV], Z[:, M.IT] = 40.0, 10.0, 320.0
    feed = CONFIGS["C1"].feeds(params)[0]
    J1 = M.jacobian(Z, 0.7, feed, P)
    J2 = M.jacobian(Z, np.array([0.7]), feed, P)
    assert np.array_equal(J1, J2)


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


def test_section_rows_use_their_own_diameter(params):
    # the hydraulic row of stage n changes only with theta of its own section,
    # by -u_max pi theta / 2 per unit of theta
    P = M.OracleParams(params)
    N, p = 6, 3
    Z = _random_point(N, 4)
    th = np.array([0.6, 0.8, 1.1])
    J = M.jacobian(Z, th, CONFIGS["C1"].feeds(params)[1], P)
    sec = M.sections(N, p)
    for n in range(N):
        row = J[n * M.NR + M.NR - 1, -p:]
        want = np.zeros(p)
        want[sec[n]] = -P.u_max * math.pi * th[sec[n]] / 2.0
        assert np.allclose(row, want, rtol=1e-14, atol=0.0)
    # no other row depends on theta
    other = np.delete(J[:, -p:], [n * M.NR + M.NR - 1 for n in range(N)], axis=0)
    assert np.all(other == 0.0)


def test_p_column_bordered_kkt_against_dense_brute_force(params):
    P = M.OracleParams(params)
    rng = np.random.default_rng(11)
    N, S, p = 3, 2, 3
    feeds = CONFIGS["C1"].feeds(params)[:S]
    th = np.array([0.7, 0.9, 1.2])
    blocks, borders, kdd = [], [], np.zeros((p, p))
    for w in range(S):
        Z = _random_point(N, 20 + w)
        J = M.jacobian(Z, th, feeds[w], P)
        cs = 1.0 / np.abs(J).max(axis=1)
        J = J * cs[:, None]
        H = M.lagrangian_hessian(Z, th, feeds[w], rng.normal(size=(N, M.NR)) * cs.reshape(N, M.NR), P)
        K, B, Hdd = scenario_kkt(J, H, rng.uniform(0.1, 5, N * M.NV), rng.uniform(0.1, 5, N), 0.3, 1e-6, N, p)
        assert B.shape == (K.shape[0], p) and Hdd.shape == (p, p)
        blocks.append(K)
        borders.append(B)
        kdd = kdd + Hdd
    kdd = kdd + np.diag([2.0, 0.5, 1.5])
    F = BorderedKKT(blocks, borders, kdd)
    n = sum(K.shape[0] for K in blocks) + p
    A = np.zeros((n, n))
    o = 0
    for K, B in zip(blocks, borders):
        m = K.shape[0]
        A[o:o + m, o:o + m] = K
        A[o:o + m, -p:] = B
        A[-p:, o:o + m] = B.T
        o += m
    A[-p:, -p:] = kdd
    ev = np.linalg.eigvalsh(A)
    assert F.inertia == (int((ev > 0).sum()), int((ev < 0).sum()), 0)
    r = rng.normal(size=n)
    rs, o = [], 0
    for K in blocks:
        rs.append(r[o:o + K.shape[0]])
        o += K.shape[0]
    xs, xd = F.solve(rs, r[-p:])
    x = np.concatenate(xs + [xd])
    xr = np.linalg.solve(A, r)
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-9
    # the design block of the inverse is the inverse of the Schur complement
    E = np.zeros((n, p))
    E[-p:, :] = np.eye(p)
    assert np.allclose(np.linalg.solve(A, E)[-p:, :], np.linalg.inv(F.sd), rtol=1e-8, atol=1e-12)


@pytest.fixture(scope="module")
def two_sections(params):
    w = CONFIGS["C1"]
    F = w.feeds(params)
    r = ipm.solve(params, F, w.n_stages, n_sections=2)
    th, Zs, ok = simulate.closed_form_sections(F, w.n_stages, 2, params)
    return w, F, r, th, Zs, ok


def test_section_diameters_equal_closed_form(two_sections):
    w, F, r, th, Zs, ok = two_sections
    assert r.status == ipm.SUCCESS and r.E0 <= 1e-8 and r.max_lin_resid <= 1e-10
    assert ok.all()
    assert np.abs(r.theta - th).max() / th.max() <= 1e-6
    # the bottom section carries the larger gas volume flow here: distinct diameters
    assert abs(th[0] - th[1]) / th.max() > 1e-3
    Z = r.x[:-2].reshape(F.shape[0], w.n_stages, M.NV)
    assert np.abs(Z - Zs).max() / np.abs(Zs).max() < 1e-9


def test_section_multipliers_close_dL_dtheta(two_sections, params):
    # dL/dtheta_k = 0 with inactive bounds: the hydraulic multipliers (unscaled
    # rows) of section k sum to 2 c_k / (pi u_max theta_k)
    w, F, r, th, _, _ = two_sections
    prob = ipm.Problem(params, F, w.n_stages, 2)
    o = ipm.OracleIPM(prob)
    o.compute_scaling(o.push_into_bounds(prob.initial_point() / o.D, 1e-2, 1e-2))
    lam = r.yd * o.cs[:, :, -1]
    sec = M.sections(w.n_stages, 2)
    for k in range(2):
        got = lam[:, sec == k].sum()
        assert got == pytest.approx(2.0 * prob.c[k] / (math.pi * params["u_max"] * r.theta[k]), rel=1e-6)


def test_section_solution_is_permutation_invariant(params):
    pert = np.array([[0.08, -0.05, 0.10], [-0.1, 0.1, -0.05], [0.02, 0.0, 0.04]])
    ra = ipm.solve(params, feed_table(pert, params), 4, n_sections=2)
    rb = ipm.solve(params, feed_table(pert[::-1], params), 4, n_sections=2)
    assert ra.status == ipm.SUCCESS and rb.status == ipm.SUCCESS
    assert np.abs(ra.theta - rb.theta).max() / ra.theta.max() < 1e-9
