"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these tests retypes an oracle formula: each checks a property that a
plausible mistake in the oracle (a dropped term, a wrong sign or index, a
transposed operand, a mis-transcribed constant) would break.
"""

import math

import numpy as np
import pytest
import torch

from absorber_inputs import CONFIGS, dims, feed_table, perturbations
from oracle import model as M
from oracle.kkt import BorderedKKT, scenario_kkt


# ---------------------------------------------------------------- problem data
def test_problem_size_matches_paper():
    # Numerical results: |Omega| = 5000 gives 1,500,001 variables, 1,050,000 MESH
    # equalities, 450,000 variable-fixing constraints, 50,000 hydraulic rows.
    d = dims(10, 5000)
    assert d["n_var_total"] == 1_500_001
    assert d["n_eq"] == 1_050_000
    assert d["n_fixed"] == 450_000
    assert d["n_ineq"] == 50_000
    assert d["n_var_free"] + d["n_fixed"] == d["n_var_total"]


def test_stoichiometry_conserves_atoms_and_charge(params):
    # R1-R5 (Case study) must conserve the amine backbone, carbon, H and O
    # atoms and charge; a mis-transcribed coefficient breaks one of these.
    nu = np.array(params["nu"], dtype=float)
    groups = {
        "amine": [1, 1, 0, 1, 0, 0, 0, 0, 0, 0, 0],
        "carbon": [0, 0, 0, 1, 1, 0, 1, 1, 0, 0, 0],
        "charge": [0, 1, 1, -1, -1, -1, -2, 0, 0, 0, 0],
        "H": [7, 8, 1, 6, 1, 1, 0, 0, 2, 0, 0],
        "O": [1, 1, 0, 3, 3, 1, 3, 2, 1, 0, 0],
        "N2": [0] * 9 + [1, 0],
        "O2": [0] * 10 + [1],
    }
    for name, a in groups.items():
        assert np.allclose(np.array(a, dtype=float) @ nu, 0.0), name
    assert np.linalg.matrix_rank(nu) == 5


def test_equilibrium_constants_reproduce_textbook_pk(params):
    # 298.15 K anchors: pKa(MEAH+) 9.50, pKa2(CO2) 10.33, pKw 14.0 (pure water),
    # carbamate reversion 0.033 mol/L, pKa1(CO2) 6.35, converted to mole fractions.
    A, B = np.array(params["lnK_A"]), np.array(params["lnK_B"])
    lnK = A + B / 298.15
    ln10, c = math.log(10.0), 43.0
    expect = [-9.50 * ln10 - math.log(c), -10.33 * ln10 - math.log(c),
              math.log(1e-14) - 2 * math.log(55.5), math.log(0.033 / (c * 0.87)),
              -6.35 * ln10 - math.log(c * 0.87)]
    assert np.allclose(lnK, expect, atol=1e-9)


def test_enthalpies_consistent_with_van_t_hoff(params):
    # the reference enthalpies must carry the reaction enthalpies dH_r = -R B_r
    nu = np.array(params["nu"], dtype=float)[:9]
    href = np.array(params["hL_ref"])
    dH = -params["R"] * np.array(params["lnK_B"])
    assert np.allclose(href @ nu, dH, rtol=1e-9, atol=1e-6)


def test_saturation_pressure_matches_steam_table(params):
    # normal boiling point and 40 C vapour pressure of water
    ps = lambda T: math.exp(params["psat_a"] - params["psat_b"] / T)  # noqa: E731
    assert abs(ps(373.15) - 101325.0) / 101325.0 < 1e-9
    assert abs(ps(313.15) - 7380.0) / 7380.0 < 1e-9


def test_feed_table_rows(params):
    u = perturbations(3, 0.2, 7)
    F = feed_table(u, params)
    assert np.allclose(F[:, 1:5].sum(axis=1), 1.0)
    assert np.allclose(F[:, 0], 10.0 * (1 + u[:, 0]))
    assert np.allclose(F[:, 5], 313.15 * (1 + u[:, 2]))


# ---------------------------------------------------------------- derivatives
def _random_point(N, seed):
    rng = np.random.default_rng(seed)
    Z = np.empty((N, M.NV))
    Z[:, 0:9] = rng.uniform(0.01, 0.3, (N, 9))
    Z[:, 9:13] = rng.uniform(0.05, 0.5, (N, 4))
    Z[:, M.IL] = rng.uniform(30, 60, N)
    Z[:, M.IV] = rng.uniform(5, 15, N)
    Z[:, M.IT] = rng.uniform(300, 350, N)
    Z[:, M.IE:] = rng.uniform(-1, 1, (N, 5))
    return Z, float(rng.uniform(0.3, 2.0))


def _fd_jac(f, w, h):
    cols = []
    for j in range(w.numel()):
        e = torch.zeros_like(w)
        e[j] = h * max(1.0, abs(float(w[j])))
        cols.append((f(w + e) - f(w - e)) / (2 * e[j]))
    return torch.stack(cols, dim=1)


def test_jacobian_matches_central_differences(params):
    P = M.OracleParams(params)
    N = 3
    Z, d = _random_point(N, 1)
    feed = CONFIGS["C1"].feeds(params)[0]
    J = M.jacobian(Z, d, feed, P)
    f = M._flat(P, torch.from_numpy(feed), N)
    w = torch.cat([torch.from_numpy(Z.reshape(-1)), torch.tensor([d], dtype=torch.float64)])
    Jfd = _fd_jac(f, w, 1e-6).numpy()
    scale = np.abs(J).max(axis=1, keepdims=True) + 1e-30
    assert np.abs((J - Jfd) / scale).max() < 1e-6


def test_hessian_matches_differences_of_gradient(params):
    P = M.OracleParams(params)
    N = 3
    Z, d = _random_point(N, 2)
    feed = CONFIGS["C1"].feeds(params)[1]
    lam = np.random.default_rng(3).normal(size=(N, M.NR))
    H = M.lagrangian_hessian(Z, d, feed, lam, P)
    assert np.allclose(H, H.T, atol=0, rtol=0)
    f = M._flat(P, torch.from_numpy(feed), N)
    lt = torch.from_numpy(lam.reshape(-1))

    def grad(w):
        return torch.func.jacrev(lambda v: (lt * f(v)).sum())(w)

    w = torch.cat([torch.from_numpy(Z.reshape(-1)), torch.tensor([d], dtype=torch.float64)])
    Hfd = _fd_jac(grad, w, 1e-6).numpy()
    scale = np.abs(H).max() + 1e-30
    assert np.abs(H - Hfd).max() / scale < 1e-6


def test_hessian_is_block_diagonal_by_stage(params):
    # every nonlinear term of (1)-(10b) involves one stage's variables (or d alone)
    P = M.OracleParams(params)
    N = 4
    Z, d = _random_point(N, 4)
    feed = CONFIGS["C1"].feeds(params)[2]
    lam = np.random.default_rng(5).normal(size=(N, M.NR))
    H = M.lagrangian_hessian(Z, d, feed, lam, P)
    for a in range(N):
        for b in range(N):
            if a != b:
                blk = H[a * M.NV:(a + 1) * M.NV, b * M.NV:(b + 1) * M.NV]
                assert np.all(blk == 0.0)
    assert np.all(H[:-1, -1] == 0.0)
    assert H[-1, -1] == pytest.approx(-lam[:, -1].sum() * P.u_max * math.pi / 2, rel=1e-14)


def test_jacobian_columns_depend_on_own_stage_only(params):
    # d c / d z_n depends on z_n alone: coupling terms are products L x, V y, L h, V h
    P = M.OracleParams(params)
    N = 4
    Z, d = _random_point(N, 6)
    feed = CONFIGS["C1"].feeds(params)[3]
    J1 = M.jacobian(Z, d, feed, P)
    Z2 = _random_point(N, 7)[0]
    Z2[1] = Z[1]
    J2 = M.jacobian(Z2, d, feed, P)
    cols = slice(1 * M.NV, 2 * M.NV)
    assert np.array_equal(J1[:, cols], J2[:, cols])


# ---------------------------------------------------------------- KKT algebra
def test_bordered_kkt_against_dense_brute_force(params):
    P = M.OracleParams(params)
    rng = np.random.default_rng(8)
    N, S = 2, 2
    feeds = CONFIGS["C1"].feeds(params)[:S]
    blocks, borders, kdd = [], [], 0.0
    for w in range(S):
        Z, d = _random_point(N, 10 + w)
        J = M.jacobian(Z, d, feeds[w], P)
        cs = 1.0 / np.abs(J).max(axis=1)  # row scaling as in the NLP scaling step
        J = J * cs[:, None]
        H = M.lagrangian_hessian(Z, d, feeds[w], rng.normal(size=(N, M.NR)) * cs.reshape(N, M.NR), P)
        K, b, hdd = scenario_kkt(J, H, rng.uniform(0.1, 5, N * M.NV), rng.uniform(0.1, 5, N), 0.3, 1e-6, N)
        blocks.append(K)
        borders.append(b)
        kdd += hdd
    kdd += 2.0
    F = BorderedKKT(blocks, borders, kdd)
    # dense assembly of the full bordered matrix
    n = sum(K.shape[0] for K in blocks) + 1
    A = np.zeros((n, n))
    o = 0
    for K, b in zip(blocks, borders):
        m = K.shape[0]
        A[o:o + m, o:o + m] = K
        A[o:o + m, -1] = b
        A[-1, o:o + m] = b
        o += m
    A[-1, -1] = kdd
    ev = np.linalg.eigvalsh(A)
    assert F.inertia == (int((ev > 0).sum()), int((ev < 0).sum()), 0)
    r = rng.normal(size=n)
    rs, o = [], 0
    for K in blocks:
        rs.append(r[o:o + K.shape[0]])
        o += K.shape[0]
    xs, xd = F.solve(rs, r[-1])
    x = np.concatenate(xs + [np.array([xd])])
    xr = np.linalg.solve(A, r)
    assert np.abs(A @ x - r).max() <= 1e-13 * np.abs(A).max() * np.abs(x).max()
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-9
    # Schur scalar: the d-d entry of the inverse is 1 / S_d
    e = np.zeros(n)
    e[-1] = 1.0
    assert np.linalg.solve(A, e)[-1] == pytest.approx(1.0 / F.sd, rel=1e-9)
