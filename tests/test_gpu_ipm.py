"""The GPU interior-point solve against the oracle (C1) and against the
closed-form optimum checked scenario by scenario (C2 and C3, full size).

Tolerances: diameter relative error <= 1e-6, final scaled optimality error
E_0 <= 1e-8, largest per-solve linear relative residual <= 1e-10.
"""

import math

import numpy as np
import pytest
import torch

from absorber_inputs import CONFIGS
from oracle import ipm as oipm
from oracle import model as M
from oracle import simulate

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def gpu_solve(params, feeds, N, **opts):
    from paper_2607_15420_amd import Absorber
    h = Absorber(params, N, feeds)
    x = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    lam = torch.empty(h.nc, dtype=torch.float64, device=DEV)
    r = h.ipm_solve(Absorber.default_options(**opts), x_out=x, lam_out=lam)
    torch.cuda.synchronize()
    out = (r, x.cpu().numpy(), lam.cpu().numpy())
    h.close()
    return out


def test_c1_matches_oracle(params):
    w = CONFIGS["C1"]
    F = w.feeds(params)
    r, x, lam = gpu_solve(params, F, w.n_stages)
    assert r.status == 0, r.as_dict()
    assert r.E0 <= 1e-8
    assert r.max_lin_resid <= 1e-10
    dstar, dw, Zs, ok = simulate.closed_form_diameter(F, w.n_stages, params)
    assert ok.all()
    assert abs(r.d - dstar) / dstar <= 1e-6
    Z = x[:-1].reshape(F.shape[0], w.n_stages, M.NV)
    assert np.abs(Z - Zs).max() / np.abs(Zs).max() <= 1e-8
    ro = oipm.solve(params, F, w.n_stages)
    assert ro.status == 0
    assert abs(r.d - ro.d) / ro.d <= 1e-6
    # the hydraulic multipliers of the unscaled rows sum to 2 / (pi u_max d*) (dL/dd = 0)
    s = lam.reshape(F.shape[0], w.n_stages, M.NR)[:, :, -1].sum()
    assert s == pytest.approx(2.0 / (math.pi * params["u_max"] * r.d), rel=1e-6)


def check_full_size(params, w, n_sample, seed, mesh_sample=None):
    F = w.feeds(params)
    S, N = F.shape[0], w.n_stages
    r, x, lam = gpu_solve(params, F, N)
    assert r.status == 0, r.as_dict()
    assert r.E0 <= 1e-8
    assert r.max_lin_resid <= 1e-10
    P = M.OracleParams(params)
    Z = x[:-1].reshape(S, N, M.NV)
    # the MESH rows vanish at the GPU states (oracle residuals), relative to the
    # row's magnitude |J| |z|: every scenario, or a seeded sample of them
    c = M.constraints(Z, r.d, F, P)
    rows = range(S) if mesh_sample is None else sorted(
        np.random.default_rng(seed + 100).choice(S, mesh_sample, replace=False).tolist())
    for s in rows:
        J = M.jacobian(Z[s], r.d, F[s], P)
        mag = np.abs(J) @ np.abs(np.r_[Z[s].reshape(-1), r.d])
        assert (np.abs(c[s, :, :-1].reshape(-1)) <= 1e-9 * mag.reshape(N, M.NR)[:, :-1].reshape(-1)).all(), s
    # d equals the largest hydraulic diameter over all scenarios' states
    dmax = max(simulate.hydraulic_diameter(Z[s], F[s], P) for s in range(S))
    assert abs(r.d - dmax) / dmax <= 1e-6
    # sampled scenarios, and the one that sets d, simulated independently by the oracle
    ds = np.array([simulate.hydraulic_diameter(Z[s], F[s], P) for s in range(S)])
    rng = np.random.default_rng(seed)
    sample = set(rng.choice(S, n_sample, replace=False).tolist()) | {int(ds.argmax())}
    ip = params["initial_point"]
    z0 = np.r_[ip["x"], ip["y"], ip["L"], ip["V"], ip["T"], [0.0] * 5]
    for s in sorted(sample):
        Zs, ok, _, _ = simulate.simulate_scenario(np.tile(z0, (N, 1)), F[s], P)
        assert ok
        assert np.abs(Zs - Z[s]).max() / np.abs(Zs).max() <= 1e-8
    s_star = int(ds.argmax())
    Zs, ok, _, _ = simulate.simulate_scenario(np.tile(z0, (N, 1)), F[s_star], P)
    dstar = simulate.hydraulic_diameter(Zs, F[s_star], P)
    assert abs(r.d - dstar) / dstar <= 1e-6
    return r


def test_c2_full_size(params):
    check_full_size(params, CONFIGS["C2"], 6, 1)


def test_c3_full_size(params):
    """The benchmarked workload (10 stages x 5000 scenarios, default options as
    timed): d against the largest hydraulic diameter over all 5000 scenarios'
    states, MESH residuals on 40 sampled scenarios, and 12 sampled scenarios plus
    the one that sets d simulated independently by the oracle."""
    r = check_full_size(params, CONFIGS["C3"], 12, 2, mesh_sample=40)
    assert r.iterations <= 60


def test_c6_convex_combination_scenarios_full_size(params):
    """10 stages x 5000 scenarios drawn as convex combinations of seven base
    cases (the paper's sampling scheme on synthetic cases): the same checks as
    the benchmarked workload."""
    r = check_full_size(params, CONFIGS["C6"], 8, 6, mesh_sample=20)
    assert r.iterations <= 60


def test_autotune_keeps_the_result(params):
    """Launch shapes chosen by measurement change the speed, not the arithmetic:
    the solve with the tuned shapes is bit-identical to the default shapes."""
    from paper_2607_15420_amd import Absorber
    w = CONFIGS["C1"]
    F = w.feeds(params)
    h0 = Absorber(params, w.n_stages, F)
    r0 = h0.ipm_solve(Absorber.default_options(autotune=0))
    assert not h0.tuning()["tuned"]
    h0.close()
    h1 = Absorber(params, w.n_stages, F)
    r1 = h1.ipm_solve(Absorber.default_options(autotune=1))
    t = h1.tuning()
    h1.close()
    assert t["tuned"] and t["factor_waves_per_simd"] in (2, 3) and t["eval_block"] in (64, 128, 256)
    assert t["factor_row_split"] in (0, 1, 2)
    assert min(min(r) for r in t["factor_ms"]) > 0 and min(t["solve_ms"]) > 0
    assert r1.status == 0 and r1.iterations == r0.iterations and r1.d == r0.d


@pytest.mark.parametrize("wpe", [2, 3])
@pytest.mark.parametrize("split", [0, 1, 2])
def test_every_factor_tile_shape_gives_the_same_solve(params, wpe, split):
    """Each block-LDL^T launch shape the autotuner chooses among (occupancy x row
    split of the trailing update) takes the same pivots and gives a
    bit-identical solve on C1 and on a ragged 10-stage x 23-scenario instance."""
    from paper_2607_15420_amd import Absorber
    from absorber_inputs import feed_table, perturbations
    for N, F in ((CONFIGS["C1"].n_stages, CONFIGS["C1"].feeds(params)),
                 (10, feed_table(perturbations(23, 0.2, 9), params))):
        out = []
        for shape in ((3, 0), (wpe, split)):
            h = Absorber(params, N, F)
            h.set_tuning(factor_waves_per_simd=shape[0], factor_row_split=shape[1])
            x = torch.empty(h.nx, dtype=torch.float64, device=DEV)
            r = h.ipm_solve(Absorber.default_options(), x_out=x)
            torch.cuda.synchronize()
            out.append((r, x.cpu().numpy()))
            h.close()
        (ra, xa), (rb, xb) = out
        assert ra.status == 0 and rb.status == 0
        assert rb.iterations == ra.iterations and rb.d == ra.d and np.array_equal(xa, xb)
