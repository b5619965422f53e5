"""Edge cases of the single-diameter solve on the GPU, through the C ABI:
columns of one and two stages (a stage that is both the top and the bottom of
its column; no coupling to pass up), one scenario, a scenario count that is not
a multiple of anything the kernels tile by, and handles that cannot exist
(no stages, no scenarios, too many stages) rejected as argument errors.

The solves are checked against the closed form (independent per-scenario
Newton simulations of the oracle) and against the oracle IPM, to the same
tolerances as C1: d within 1e-6, E_0 <= 1e-8, linear residual <= 1e-10.
"""

import numpy as np
import pytest
import torch

from absorber_inputs import CONFIGS
from oracle import ipm as oipm
from oracle import model as M
from oracle import simulate

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _solve(h):
    from paper_2607_15420_amd import Absorber
    x = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    r = h.ipm_solve(Absorber.default_options(), x_out=x)
    torch.cuda.synchronize()
    return r, x.cpu().numpy()


@pytest.mark.parametrize("N,S", [(1, 3), (2, 1), (2, 5), (3, 7)], ids=["1x3", "2x1", "2x5", "3x7"])
def test_short_columns_match_closed_form_and_oracle(params, N, S):
    from paper_2607_15420_amd import Absorber
    F = CONFIGS["C2"].feeds(params)[:S]
    dstar, _, Zs, ok = simulate.closed_form_diameter(F, N, params)
    assert np.all(ok)
    ro = oipm.solve(params, F, N)
    assert ro.status == oipm.SUCCESS
    h = Absorber(params, N, F)
    try:
        r, x = _solve(h)
    finally:
        h.close()
    assert r.status == 0 and r.E0 <= 1e-8 and r.max_lin_resid <= 1e-10, r.as_dict()
    assert abs(r.d - dstar) / dstar <= 1e-6
    assert abs(r.d - ro.d) / ro.d <= 1e-6
    Z = x[:-1].reshape(S, N, M.NV)
    assert np.abs(Z - Zs).max() / np.abs(Zs).max() <= 1e-6


@pytest.mark.parametrize("N,S", [(0, 3), (4, 0), (4097, 1)], ids=["no-stages", "no-scenarios", "too-many-stages"])
def test_impossible_handles_are_argument_errors(params, N, S):
    from paper_2607_15420_amd import Absorber, AbsorberError
    F = CONFIGS["C1"].feeds(params)
    F = np.repeat(F, max(1, -(-S // F.shape[0])), axis=0)[:S]
    with pytest.raises(AbsorberError) as e:
        Absorber(params, N, F)
    assert "ARG" in str(e.value)


def test_batch_with_an_impossible_problem_is_an_argument_error(params):
    from paper_2607_15420_amd import Absorber, AbsorberError
    F = CONFIGS["C1"].feeds(params)
    with pytest.raises(AbsorberError) as e:
        Absorber.batch(params, [(4, F), (0, F)])
    assert "ARG" in str(e.value)
