"""absorber_warm_start_noalloc (the warm start for callers that cannot
allocate device memory) against absorber_warm_start, the same computation with
caller workspaces: identical decoded points, on two calls in a row with the
second on a smaller input, for a primal-dual and a primal network; sizes past
the static workspace are rejected."""

import numpy as np
import pytest
import torch

from absorber_inputs import feed_table, perturbations

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N = 4


def _compare(params, net, S, seed, dual):
    from paper_2607_15420_amd import Absorber
    h = Absorber(params, N, feed_table(perturbations(S, 0.2, seed), params))
    no = net.cfg.n_out
    X = torch.empty((S, 3), dtype=torch.float32, device=DEV)
    Y = torch.empty((S, no), dtype=torch.float32, device=DEV)
    x_ref = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    l_ref = torch.empty(h.nc, dtype=torch.float64, device=DEV) if dual else None
    h.warm_start(net, X, Y, x_ref, l_ref)
    x1 = torch.full((h.nx,), float("nan"), dtype=torch.float64, device=DEV)
    l1 = torch.full((h.nc,), float("nan"), dtype=torch.float64, device=DEV) if dual else None
    h.warm_start_noalloc(net, x1, l1)
    torch.cuda.synchronize()
    assert torch.isfinite(x_ref).all()
    assert torch.equal(x1, x_ref)
    if dual:
        assert torch.equal(l1, l_ref)
        # the multipliers of exactly one scenario (the worst) are set
        nz = (l1.view(S, N * 22) != 0).any(dim=1)
        assert int(nz.sum()) == 1
    h.close()


@pytest.mark.parametrize("dual", [True, False])
def test_noalloc_warm_start_matches_warm_start(params, dual):
    from paper_2607_15420_amd import Mlp
    net = Mlp(3, 64, 2, (43 if dual else 21) * N, max_batch=64, seed=11)
    rng = np.random.default_rng(5)
    # a random network whose outputs decode to moderate states
    net.set_params(0.05 * rng.standard_normal(net.n_params).astype(np.float32))
    _compare(params, net, 37, 7, dual)   # several forward chunks and a ragged tail
    _compare(params, net, 5, 8, dual)    # then a smaller input on the same workspace
    net.close()


def test_noalloc_rejects_sizes_past_its_workspace(params):
    from paper_2607_15420_amd import Absorber, Mlp
    from paper_2607_15420_amd.binding import AbsorberError
    S, n = 20000, 10   # the training set as one problem: 20000 x 430 outputs take 34.7 MB
    h = Absorber(params, n, feed_table(perturbations(S, 0.2, 4), params))
    net = Mlp(3, 64, 1, 43 * n, max_batch=64, seed=1)
    x0 = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    with pytest.raises(AbsorberError) as e:
        h.warm_start_noalloc(net, x0)
    assert e.value.code == -1 and "maximum" in str(e.value)
    net.close()
    h.close()
