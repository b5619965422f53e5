"""Graph-replayed iterations with the per-problem decisions on the device
(absorber_ipm_options.use_graph = 1) against the host-driven loop (use_graph
= 0), the oracle and the closed-form optimum.

The device control kernels take the host loop's decisions with the same
arithmetic, so both modes must take the same iterations, factorisations,
delta_w and line-search trials; every solve replays the captured graphs many
times with host reads in between, and repeated solves on one handle reuse
them.
"""

import numpy as np
import pytest
import torch

from absorber_inputs import CONFIGS, feed_table, perturbations
from oracle import ipm as oipm
from oracle import model as M
from oracle import simulate
from test_oracle_inertia import N_STAGES, inertia_case

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def solve(h, **opts):
    from paper_2607_15420_amd import Absorber
    x = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    lam = torch.empty(h.nc, dtype=torch.float64, device=DEV)
    r = h.ipm_solve(Absorber.default_options(**opts), x_out=x, lam_out=lam)
    torch.cuda.synchronize()
    return r, x.cpu().numpy(), lam.cpu().numpy(), h.ipm_log()


def same_logs(a, b, rel_mu=1e-13):
    assert len(a) == len(b)
    for u, v in zip(a, b):
        assert u["n_factorizations"] == v["n_factorizations"], (u, v)
        assert u["n_trials"] == v["n_trials"], (u, v)
        assert u["delta_w"] == pytest.approx(v["delta_w"], rel=1e-12, abs=0.0)
        assert u["mu"] == pytest.approx(v["mu"], rel=rel_mu)
        assert u["d"] == pytest.approx(v["d"], rel=1e-9)


def test_c1_graph_matches_host_loop_and_closed_form(params):
    from paper_2607_15420_amd import Absorber
    w = CONFIGS["C1"]
    F = w.feeds(params)
    h = Absorber(params, w.n_stages, F)
    rh, xh, lh, logh = solve(h, use_graph=0)
    rg, xg, lg, logg = solve(h, use_graph=1)
    assert rh.status == 0 and rg.status == 0, rg.as_dict()
    assert rg.iterations == rh.iterations
    assert rg.E0 <= 1e-8 and rg.max_lin_resid <= 1e-10
    assert abs(rg.d - rh.d) / rh.d <= 1e-10
    assert np.abs(xg - xh).max() / np.abs(xh).max() <= 1e-9
    same_logs(logg, logh)
    dstar, _, Zs, ok = simulate.closed_form_diameter(F, w.n_stages, params)
    assert abs(rg.d - dstar) / dstar <= 1e-6
    # repeated solves reuse the captured graphs and give the same result
    for _ in range(2):
        r2, x2, _, log2 = solve(h, use_graph=1)
        assert r2.iterations == rg.iterations and np.array_equal(x2, xg)
        same_logs(log2, logg, rel_mu=0.0)
    h.close()


def test_inertia_corrections_in_graph_mode(params):
    from paper_2607_15420_amd import Absorber
    F, dstar, x0, lam, lam_s = inertia_case(params)
    ro = oipm.solve(params, F, N_STAGES, oipm.IpmOptions(warm_start=True), x0=x0,
                    yc0=lam_s[:, :, :-1], yd0=lam_s[:, :, -1])
    h = Absorber(params, N_STAGES, F)
    x0d = torch.tensor(x0, dtype=torch.float64, device=DEV)
    l0d = torch.tensor(lam.reshape(-1), dtype=torch.float64, device=DEV)
    r = h.ipm_solve(Absorber.default_options(warm_start=1, feasibility_restart=0, use_graph=1), x0=x0d, lam0=l0d)
    log = h.ipm_log()
    assert r.status == 0, r.as_dict()
    assert r.n_inertia_corrections == ro.n_inertia_corrections >= 1
    assert r.iterations == ro.iterations
    for dev, ora in zip(log, ro.log):
        assert dev["n_factorizations"] == len(ora["dw_trials"])
        assert dev["delta_w"] == pytest.approx(ora["dw"], rel=1e-12, abs=0.0)
    assert abs(r.d - dstar) / dstar <= 1e-6
    # a delta_w bound below the first correction: inertia failure
    r = h.ipm_solve(Absorber.default_options(warm_start=1, feasibility_restart=0, use_graph=1, delta_w_max=1e-3),
                    x0=x0d, lam0=l0d)
    assert r.status == -10 and r.iterations == 0
    h.close()


def test_uneven_batch_in_graph_mode(params):
    from paper_2607_15420_amd import Absorber
    Ns, Ss = [8, 10, 13, 6, 20], [3, 7, 1, 12, 4]
    problems = [(N, feed_table(perturbations(S, 0.15, 100 + p), params)) for p, (N, S) in enumerate(zip(Ns, Ss))]
    h = Absorber.batch(params, problems)
    o0 = Absorber.default_options(use_graph=0)
    o1 = Absorber.default_options(use_graph=1)
    x0 = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    x1 = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    rc0, res0 = h.batch_solve(o0, x_out=x0)
    logs0 = [h.ipm_log(p) for p in range(h.P)]
    rc1, res1 = h.batch_solve(o1, x_out=x1)
    logs1 = [h.ipm_log(p) for p in range(h.P)]
    torch.cuda.synchronize()
    assert rc1 == 0, [r.as_dict() for r in res1]
    for p, ((N, F), a, b) in enumerate(zip(problems, res0, res1)):
        assert b.status == 0 and b.E0 <= 1e-8 and b.max_lin_resid <= 1e-10, (p, b.as_dict())
        assert b.iterations == a.iterations and b.feasibility_restarts == a.feasibility_restarts, p
        assert abs(b.d - a.d) / a.d <= 1e-10, p
        dstar = simulate.closed_form_diameter(F, N, params)[0]
        assert abs(b.d - dstar) / dstar <= 1e-6, p
        same_logs(logs1[p], logs0[p])
    h.close()


def test_c2_full_size_graph_matches_host_loop(params):
    from paper_2607_15420_amd import Absorber
    w = CONFIGS["C2"]
    F = w.feeds(params)
    h = Absorber(params, w.n_stages, F)
    rh, xh, _, logh = solve(h, use_graph=0)
    rg, xg, _, logg = solve(h, use_graph=1)
    assert rg.status == 0 and rg.E0 <= 1e-8 and rg.max_lin_resid <= 1e-10, rg.as_dict()
    assert rg.iterations == rh.iterations
    assert abs(rg.d - rh.d) / rh.d <= 1e-10
    same_logs(logg, logh)
    h.close()


def test_tall_column_fails_cold_in_graph_mode_like_the_oracle(params):
    from paper_2607_15420_amd import Absorber
    F = feed_table(perturbations(4, 0.15, 104), params)[1:2]
    N = 20
    ro = oipm.solve(params, F, N)
    h = Absorber(params, N, F)
    r = h.ipm_solve(Absorber.default_options(feasibility_restart=0, use_graph=1))
    assert ro.status == -11 and r.status == -11 and r.iterations == ro.iterations
    assert r.d == pytest.approx(ro.d, rel=1e-8)
    r1 = h.ipm_solve(Absorber.default_options(use_graph=1))
    assert r1.status == 0 and r1.feasibility_restarts == 1
    h.close()
