"""The oracle's inertia-correction loop (interior-point search direction step:
the Ipopt rule for delta_w and delta_c) pinned against dense linear algebra.

Problem (10) has square MESH blocks, so a scenario block K_w always has the
inertia (21 N, 22 N, 0) and only the sign of the Schur complement S_d on the
diameter can be wrong.  A warm start at the simulated states with d above its
optimum and large hydraulic multipliers makes the (d, d) Hessian entry
-(u_max pi / 2) sum lambda_hyd dominate, so S_d < 0 and the loop has to raise
delta_w until the matrix has n positive and m negative eigenvalues.
"""

import math

import numpy as np
import pytest

from absorber_inputs import feed_table
from oracle import ipm, simulate
from oracle import model as M

N_STAGES = 3
PERT = np.array([[0.05, -0.1, 0.02]])
D_FACTOR = 1.5        # start d at 1.5 x its optimum
LAMBDA_FACTOR = 10.0  # hydraulic multipliers 10 x their optimal sum, spread over the stages


def inertia_case(params):
    """Feeds, warm-start point (original units) and multipliers of the scaled rows."""
    F = feed_table(PERT, params)
    dstar, _, Zs, ok = simulate.closed_form_diameter(F, N_STAGES, params)
    assert ok.all()
    x0 = np.concatenate([Zs.reshape(-1), [D_FACTOR * dstar]])
    prob = ipm.Problem(params, F, N_STAGES)
    o = ipm.OracleIPM(prob)
    o.compute_scaling(o.push_into_bounds(prob.initial_point() / o.D, 1e-2, 1e-2))
    lam_h = LAMBDA_FACTOR * 2.0 / (math.pi * params["u_max"] * dstar * N_STAGES)
    lam = np.zeros((1, N_STAGES, M.NR))
    lam[:, :, -1] = lam_h                     # multipliers of the unscaled rows
    lam_scaled = lam / o.cs                   # the same multipliers for the scaled rows
    return F, dstar, x0, lam, lam_scaled


def dense_bordered(Fk):
    """Assemble the whole bordered KKT matrix from the oracle's blocks."""
    n = sum(B.K.shape[0] for B in Fk.blocks) + 1
    A = np.zeros((n, n))
    o = 0
    for B, b in zip(Fk.blocks, Fk.borders):
        m = B.K.shape[0]
        A[o:o + m, o:o + m] = B.K
        A[o:o + m, -1] = b
        A[-1, o:o + m] = b
        o += m
    A[-1, -1] = Fk.kdd
    return A


@pytest.fixture(scope="module")
def corrected(params):
    F, dstar, x0, lam, lam_s = inertia_case(params)
    trials = []

    def observe(Fk, dw, dc):
        A = dense_bordered(Fk)
        ev = np.linalg.eigvalsh(A)
        tiny = 1e-12 * np.abs(ev).max()
        trials.append(dict(dw=dw, dc=dc, inertia=Fk.inertia, sd=Fk.sd,
                           eig=(int((ev > tiny).sum()), int((ev < -tiny).sum()), int((np.abs(ev) <= tiny).sum()))))

    r = ipm.solve(params, F, N_STAGES, ipm.IpmOptions(warm_start=True), x0=x0,
                  yc0=lam_s[:, :, :-1], yd0=lam_s[:, :, -1], on_factor=observe)
    return r, trials, dstar


def test_warm_start_takes_inertia_corrections(corrected):
    r, trials, dstar = corrected
    assert r.status == ipm.SUCCESS
    assert r.n_inertia_corrections >= 1
    assert any(t["sd"] < 0 for t in trials)
    # the corrected run still reaches the closed-form optimum
    assert abs(r.d - dstar) / dstar <= 1e-6


def test_every_trial_inertia_equals_dense_eigenvalue_count(corrected):
    r, trials, _ = corrected
    n = N_STAGES * M.NV + 1
    m = N_STAGES * M.NR
    for t in trials:
        assert t["inertia"] == t["eig"], t
        # Haynsworth: the blocks are always (21N, 22N, 0); S_d decides the rest
        assert t["inertia"] == ((n, m, 0) if t["sd"] > 0 else (n - 1, m + 1, 0))


def test_delta_w_sequence_follows_the_correction_rule(corrected):
    # first correction of the solve: delta_w^0 = 1e-4, then x 100 until the
    # inertia is right; later iterations start from delta_w_last / 3 and grow x 8
    r, trials, _ = corrected
    o = ipm.IpmOptions()
    last = 0.0
    for rec in r.log:
        seq = rec["dw_trials"]
        assert seq[0] == 0.0
        for k in range(1, len(seq)):
            if k == 1:
                want = o.dw_init if last == 0.0 else max(o.dw_min, o.kappa_w_minus * last)
            else:
                want = seq[k - 1] * (o.kappa_w_plus_bar if last == 0.0 else o.kappa_w_plus)
            assert seq[k] == pytest.approx(want, rel=1e-15)
        if seq[-1] > 0.0:
            last = seq[-1]
    assert sum(len(rec["dw_trials"]) - 1 for rec in r.log) == r.n_inertia_corrections


def test_delta_w_above_its_maximum_is_an_inertia_failure(params):
    F, dstar, x0, lam, lam_s = inertia_case(params)
    opts = ipm.IpmOptions(warm_start=True, dw_max=1e-3)
    r = ipm.solve(params, F, N_STAGES, opts, x0=x0, yc0=lam_s[:, :, :-1], yd0=lam_s[:, :, -1])
    assert r.status == ipm.INERTIA_FAIL
    assert r.iterations == 0
