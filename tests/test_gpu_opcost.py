"""The expected operating cost of eq. (8a) (a blower cost falling as theta^-4)
on the GPU, through the C ABI, against the oracle: the interior optimum where
every hydraulic row is slack, the hydraulic optimum with multipliers that
balance c - 4 a d^-5, section diameters with one section of each kind, in host
and graph control (1e-6 on the design, as for problem (10)); the objective
and its gradient; a batch handle rejects the term.
"""

import copy
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


def _with_weight(params, weight):
    p = copy.deepcopy(params)
    p["operating_cost"]["weight"] = weight
    return p


@pytest.fixture(scope="module")
def c1(params):
    w = CONFIGS["C1"]
    F = w.feeds(params)
    dstar, _, Zs, ok = simulate.closed_form_diameter(F, w.n_stages, params)
    a1 = M.operating_coefficients(F, w.n_stages, 1, M.OracleParams(_with_weight(params, 1.0)))[0]
    return w, F, dstar, Zs, a1


def _solve(h, **opts):
    from paper_2607_15420_amd import Absorber
    x = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    lam = torch.empty(h.nc, dtype=torch.float64, device=DEV)
    r = h.ipm_solve(Absorber.default_options(**opts), x_out=x, lam_out=lam)
    torch.cuda.synchronize()
    return r, x.cpu().numpy(), lam.cpu().numpy()


def test_interior_optimum_host_and_graph(params, c1):
    from paper_2607_15420_amd import Absorber
    w, F, dstar, Zs, a1 = c1
    p = _with_weight(params, (1.3 * dstar) ** 5 / (4.0 * a1))
    th, _, _ = simulate.closed_form_design(F, w.n_stages, 1, p)
    ro = oipm.solve(p, F, w.n_stages)
    assert ro.status == oipm.SUCCESS
    h = Absorber(p, w.n_stages, F)
    try:
        for graph in (0, 1):
            r, x, lam = _solve(h, use_graph=graph)
            assert r.status == 0, (graph, r.as_dict())
            assert r.E0 <= 1e-8 and r.max_lin_resid <= 1e-10
            assert abs(x[-1] - th[0]) / th[0] <= 1e-6
            assert abs(x[-1] - ro.d) / ro.d <= 1e-6
            assert r.d == pytest.approx(x[-1], rel=1e-12)  # the design cost of one diameter is d
            Z = x[:-1].reshape(F.shape[0], w.n_stages, M.NV)
            assert np.abs(Z - Zs).max() / np.abs(Zs).max() <= 1e-8
            yh = lam.reshape(F.shape[0], w.n_stages, M.NR)[:, :, -1]
            assert np.abs(yh).sum() <= 1e-6 * 2.0 / (math.pi * params["u_max"] * dstar)
        # the objective and its gradient at the solution: stationary in d
        xt = torch.tensor(x, dtype=torch.float64, device=DEV)
        g = torch.empty_like(xt)
        f = h.eval_obj(xt, g)
        a = a1 * p["operating_cost"]["weight"]
        assert f == pytest.approx(x[-1] + a / x[-1] ** 4, rel=1e-13)
        assert float(g[-1]) == pytest.approx(1.0 - 4.0 * a / x[-1] ** 5, abs=1e-6)
    finally:
        h.close()


def test_hydraulic_optimum_with_cheap_blower(params, c1):
    from paper_2607_15420_amd import Absorber
    w, F, dstar, Zs, a1 = c1
    weight = 0.5 * dstar ** 5 / (4.0 * a1)
    p = _with_weight(params, weight)
    h = Absorber(p, w.n_stages, F)
    try:
        r, x, lam = _solve(h)
    finally:
        h.close()
    assert r.status == 0 and abs(r.d - dstar) / dstar <= 1e-6
    a = a1 * weight
    yh = lam.reshape(F.shape[0], w.n_stages, M.NR)[:, :, -1]
    want = 2.0 * (1.0 - 4.0 * a * r.d ** -5.0) / (math.pi * params["u_max"] * r.d)
    assert yh.sum() == pytest.approx(want, rel=1e-6)


def test_sections_with_operating_cost(params, c1):
    from paper_2607_15420_amd import Absorber
    w, F, dstar, Zs, a1 = c1
    th_h, _, _ = simulate.closed_form_sections(F, w.n_stages, 2, params)
    c = M.section_weights(w.n_stages, 2)
    a_unit = M.operating_coefficients(F, w.n_stages, 2, M.OracleParams(_with_weight(params, 1.0)))
    thr = c * th_h ** 5 / (4.0 * a_unit)
    weight = float(np.sqrt(thr.min() * thr.max())) if thr.max() > 1.05 * thr.min() else 2.0 * thr.max()
    p = _with_weight(params, weight)
    th, _, _ = simulate.closed_form_design(F, w.n_stages, 2, p)
    h = Absorber.sections(p, w.n_stages, F, 2)
    try:
        for graph in (0, 1):
            r, x, _ = _solve(h, use_graph=graph)
            assert r.status == 0, (graph, r.as_dict())
            assert r.E0 <= 1e-8 and r.max_lin_resid <= 1e-10
            assert np.abs(x[-2:] - th).max() / th.max() <= 1e-6
    finally:
        h.close()


def test_batch_rejects_operating_cost(params):
    from paper_2607_15420_amd import Absorber, AbsorberError
    p = _with_weight(params, 0.1)
    F = CONFIGS["C1"].feeds(params)
    with pytest.raises(AbsorberError):
        Absorber.batch(p, [(4, F[:2]), (5, F[2:])])
