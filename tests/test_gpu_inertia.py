"""The inertia correction on the GPU against the oracle (interior-point search
direction step: delta_w / delta_c rule), on the warm-started instance whose
Schur complement on d starts negative (see tests/test_oracle_inertia.py).

Both solvers must take the same number of factorisations in every iteration
with the same accepted delta_w, the same iteration count and reach the same
diameter; a delta_w bound below the first correction must end the solve with
the inertia failure status.
"""

import numpy as np
import pytest
import torch

from oracle import ipm as oipm
from test_oracle_inertia import N_STAGES, inertia_case

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ABS_ERR_INERTIA = -10


def device_solve(params, F, x0, lam, **opts):
    from paper_2607_15420_amd import Absorber
    h = Absorber(params, N_STAGES, F)
    x0d = torch.tensor(x0, dtype=torch.float64, device=DEV)
    l0d = torch.tensor(lam.reshape(-1), dtype=torch.float64, device=DEV)
    xo = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    o = Absorber.default_options(warm_start=1, feasibility_restart=0, **opts)
    r = h.ipm_solve(o, x0=x0d, lam0=l0d, x_out=xo)
    torch.cuda.synchronize()
    log = h.ipm_log()
    h.close()
    return r, log


@pytest.fixture(scope="module")
def both(params):
    F, dstar, x0, lam, lam_s = inertia_case(params)
    ro = oipm.solve(params, F, N_STAGES, oipm.IpmOptions(warm_start=True), x0=x0,
                    yc0=lam_s[:, :, :-1], yd0=lam_s[:, :, -1])
    rg, log = device_solve(params, F, x0, lam)
    return ro, rg, log, dstar


def test_device_takes_the_oracle_corrections(both):
    ro, rg, log, dstar = both
    assert ro.status == oipm.SUCCESS and rg.status == 0, rg.as_dict()
    assert rg.n_inertia_corrections == ro.n_inertia_corrections >= 1
    assert rg.iterations == ro.iterations
    assert len(log) == len(ro.log)
    for dev, ora in zip(log, ro.log):
        assert dev["n_factorizations"] == len(ora["dw_trials"]), (dev, ora)
        assert dev["delta_w"] == pytest.approx(ora["dw"], rel=1e-12, abs=0.0), (dev, ora)
        assert dev["delta_c"] == ora["dc"]
        assert dev["mu"] == pytest.approx(ora["mu"], rel=1e-12)
        assert dev["n_trials"] == ora["ls"]
    assert abs(rg.d - ro.d) / ro.d <= 1e-6
    assert abs(rg.d - dstar) / dstar <= 1e-6
    assert rg.E0 <= 1e-8
    assert rg.max_lin_resid <= 1e-10


def test_first_iterations_follow_the_oracle(both):
    # the early trajectory (steps, constraint violation, diameter) to 1e-8 relative
    ro, rg, log, _ = both
    for dev, ora in list(zip(log, ro.log))[:5]:
        assert dev["alpha"] == pytest.approx(ora["alpha"], rel=1e-8)
        assert dev["alpha_z"] == pytest.approx(ora["alpha_z"], rel=1e-8)
        # theta starts at the rounding level of the simulated states' residuals
        assert dev["theta"] == pytest.approx(ora["theta"], rel=1e-8, abs=1e-11)
        assert dev["d"] == pytest.approx(ora["d"], rel=1e-10)


def test_delta_w_bound_gives_inertia_failure(params):
    F, dstar, x0, lam, lam_s = inertia_case(params)
    r, log = device_solve(params, F, x0, lam, delta_w_max=1e-3)
    assert r.status == ABS_ERR_INERTIA, r.as_dict()
    assert r.iterations == 0 and len(log) == 0
    # the oracle stops the same way with the same bound
    ro = oipm.solve(params, F, N_STAGES, oipm.IpmOptions(warm_start=True, dw_max=1e-3), x0=x0,
                    yc0=lam_s[:, :, :-1], yd0=lam_s[:, :, -1])
    assert ro.status == oipm.INERTIA_FAIL
