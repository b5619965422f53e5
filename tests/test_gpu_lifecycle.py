"""Handle lifecycle: creating, using and closing handles of every kind (single
problem, sections, batch, network) again and again returns the device memory
it took, and a closed handle's solve is not reachable through the binding.
"""

import pytest
import torch

from absorber_inputs import CONFIGS

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def _cycle(params):
    from paper_2607_15420_amd import Absorber, Mlp
    F = CONFIGS["C2"].feeds(params)[:40]
    h = Absorber(params, 10, F)
    r = h.ipm_solve()
    assert r.status == 0
    h.close()
    h = Absorber.sections(params, 10, F, 2)
    r = h.ipm_solve()
    assert r.status == 0
    h.close()
    h = Absorber.batch(params, [(6, F[:5]), (10, F[5:20])])
    rc, res = h.batch_solve()
    assert rc == 0 and all(q.status == 0 for q in res)
    h.close()
    net = Mlp(3, 64, 2, 40, max_batch=256, seed=1)
    X = torch.randn((300, 3), dtype=torch.float32, device=DEV)
    Y = torch.empty((300, 40), dtype=torch.float32, device=DEV)
    net.forward(X, Y)
    net.close()


def test_repeated_handles_return_their_device_memory(params):
    _cycle(params)  # first use: library and runtime set-up
    before = _free()
    for _ in range(5):
        _cycle(params)
    after = _free()
    # the runtime may keep a few MiB of its own; five cycles leaking one handle's
    # work vectors (several MiB each) would show
    assert before - after <= 8 * 2 ** 20, (before - after) / 2 ** 20


def test_closed_handle_is_an_argument_error(params):
    from paper_2607_15420_amd import Absorber, AbsorberError
    h = Absorber(params, 4, CONFIGS["C1"].feeds(params))
    h.close()
    h.close()  # closing twice is harmless
    with pytest.raises(AbsorberError) as e:
        h.ipm_solve()
    assert "ARG" in str(e.value)
