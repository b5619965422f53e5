"""The warm-start network (bf16 MFMA GEMMs, hand-written backward, Adam)
against the float64 NumPy oracle with the same bf16 rounding points, through
the C ABI; and the warm-start encoding and solve.

Tolerances: forward outputs within 5e-3 of max|Y| (bf16 operands, float32
accumulation, and a float32 value that falls on the other side of a bf16
rounding boundary than the float64 one moves one operand by 2^-8); gradients
within 2e-2 relative per parameter array (norm and elementwise against the
array's largest entry); Adam within float32 rounding.
"""

import numpy as np
import pytest
import torch

from absorber_inputs import CONFIGS, feed_table, perturbations
from oracle import mlp as O
from oracle import model as M
from oracle import simulate

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _f32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=DEV)


def _flat(ps):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in ps]).astype(np.float32)


def _unflat(v, ps):
    out, o = [], 0
    for W, b in ps:
        nW = W.size
        out.append([v[o:o + nW].reshape(W.shape).astype(np.float64), v[o + nW:o + nW + b.size].astype(np.float64)])
        o += nW + b.size
    return out


def _net(n_in, n_hidden, n_layers, n_out, seed, max_batch=128):
    from paper_2607_15420_amd import Mlp
    ps = O.init_params(n_in, n_hidden, n_layers, n_out, seed)
    rng = np.random.default_rng(seed + 1)
    for W, b in ps:
        b[:] = (rng.standard_normal(b.shape) * 0.1).astype(np.float32)
    net = Mlp(n_in, n_hidden, n_layers, n_out, max_batch=max_batch, seed=seed)
    net.set_params(_flat(ps))
    ps = _unflat(_flat(ps), ps)  # the float32 values the device holds
    return net, ps


@pytest.mark.parametrize("B", [96, 70, 300])
def test_forward_matches_oracle(B):
    # 300 rows > max_batch: three chunks, the last one ragged
    net, ps = _net(3, 64, 3, 40, seed=21)
    X = np.random.default_rng(B).standard_normal((B, 3))
    Y = torch.empty((B, 40), dtype=torch.float32, device=DEV)
    net.forward(_f32(X), Y)
    torch.cuda.synchronize()
    Yo, _ = O.forward(ps, X.astype(np.float32).astype(np.float64), quantize=True)
    err = np.abs(Y.cpu().numpy() - Yo).max()
    assert err <= 5e-3 * np.abs(Yo).max(), err
    net.close()


def test_forward_standardisation():
    net, ps = _net(3, 32, 1, 5, seed=3)
    im, isd = np.array([1.0, -2.0, 0.5]), np.array([2.0, 0.5, 4.0])
    om, osd = np.arange(5) * 0.1, np.arange(1, 6) * 0.3
    net.set_normalization(im, isd, om, osd)
    X = np.random.default_rng(0).standard_normal((40, 3)) * 3
    Y = torch.empty((40, 5), dtype=torch.float32, device=DEV)
    net.forward(_f32(X), Y)
    Yo, _ = O.forward(ps, ((X - im) / isd).astype(np.float32).astype(np.float64), quantize=True)
    Yo = Yo * osd + om
    assert np.abs(Y.cpu().numpy() - Yo).max() <= 5e-3 * np.abs(Yo).max()
    net.close()


def test_loss_grad_matches_oracle():
    net, ps = _net(3, 64, 3, 40, seed=5)
    rng = np.random.default_rng(6)
    B = 64
    X = rng.standard_normal((B, 3)).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((B, 40)).astype(np.float32).astype(np.float64)
    g = torch.empty(net.n_params, dtype=torch.float32, device=DEV)
    loss = net.loss_grad(_f32(X), _f32(T), g)
    lo, go = O.loss_and_grads(ps, X, T, quantize=True)
    assert loss == pytest.approx(lo, rel=2e-3)
    gg = _unflat(g.cpu().numpy(), ps)
    for l, ((gW, gb), (oW, ob)) in enumerate(zip(gg, go)):
        for a, b_ in ((gW, oW), (gb, ob)):
            assert np.linalg.norm(a - b_) <= 2e-2 * np.linalg.norm(b_), l
            assert np.abs(a - b_).max() <= 2e-2 * np.abs(b_).max(), l
    net.close()


def test_loss_grad_rejects_ragged_batch():
    from paper_2607_15420_amd import AbsorberError
    net, _ = _net(3, 32, 1, 8, seed=1)
    X = _f32(np.zeros((40, 3)))
    T = _f32(np.zeros((40, 8)))
    g = torch.empty(net.n_params, dtype=torch.float32, device=DEV)
    with pytest.raises(AbsorberError):
        net.loss_grad(X, T, g)
    net.close()


def test_adam_steps_match_oracle():
    net, ps = _net(3, 32, 2, 7, seed=8)
    rng = np.random.default_rng(9)
    opt = O.Adam(ps)
    o = net.default_train_options()
    for k, lr in enumerate((1e-2, 5e-3, 2e-3)):
        gr = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in ps]
        gflat = _flat([[a.astype(np.float32), b.astype(np.float32)] for a, b in gr])
        gr = _unflat(gflat, ps)
        net.adam_step(_f32(gflat), lr, o)
        opt.step(ps, gr, lr)
        got = net.get_params()
        want = _flat([[W, b] for W, b in ps])
        assert np.abs(got - want).max() <= 1e-6 * max(1.0, np.abs(want).max()), k
    net.close()


def test_training_fits_a_smooth_map():
    from paper_2607_15420_amd import Mlp
    rng = np.random.default_rng(5)
    n = 4096
    X = rng.uniform(-1, 1, (n, 3))
    T = np.stack([np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2], np.exp(0.5 * X[:, 2]) - X[:, 0],
                  X[:, 0] * X[:, 1] * 10 + 3], axis=1)
    net = Mlp(3, 64, 2, 3, max_batch=256, seed=1)
    Xd, Td = _f32(X), _f32(T)
    Y = torch.empty((n, 3), dtype=torch.float32, device=DEV)
    r = net.train(Xd, Td, net.default_train_options(epochs=150, batch=256, lr=3e-3))
    net.forward(Xd, Y)
    err = ((Y.cpu().numpy() - T) ** 2).mean(0) / T.var(0)
    assert r.steps == 150 * (n // 256)
    assert np.all(err < 1e-2), (err, r.final_loss)
    # the fitted standardisation is the data's
    im, isd, om, osd = net.get_normalization()
    assert np.allclose(im, X.mean(0), atol=1e-5) and np.allclose(osd, T.std(0), rtol=1e-4)
    net.close()


def test_warm_encoding_roundtrip(params):
    from paper_2607_15420_amd import Absorber
    w = CONFIGS["C1"]
    F = w.feeds(params)
    N, S = w.n_stages, F.shape[0]
    dstar, ds, Zs, ok = simulate.closed_form_diameter(F, N, params)
    h = Absorber(params, N, F)
    x = torch.as_tensor(np.concatenate([Zs.reshape(-1), [dstar]]), device=DEV)
    T = torch.empty((S, 21 * N), dtype=torch.float32, device=DEV)
    X = torch.empty((S, 3), dtype=torch.float32, device=DEV)
    h.warm_targets(x, T)
    h.warm_features(X)
    x0 = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    h.warm_point(T, x0, d_margin=1e-3)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    assert np.allclose(Xh, F[:, [0, 1, 5]].astype(np.float32))
    Th = T.cpu().numpy().reshape(S, N, 21)
    assert np.allclose(Th[..., :13], np.log(Zs[..., :13]).astype(np.float32))
    x0h = x0.cpu().numpy()
    Z0 = x0h[:-1].reshape(S, N, 21)
    assert np.allclose(Z0, Zs, rtol=1e-6, atol=1e-6)
    # the decoded diameter is the hydraulic diameter of the decoded states times (1 + margin)
    P = M.OracleParams(params)
    dz = max(simulate.hydraulic_diameter(Z0[s], F[s], P) for s in range(S))
    assert x0h[-1] == pytest.approx(1.001 * dz, rel=1e-12)
    assert x0h[-1] == pytest.approx(1.001 * dstar, rel=1e-6)
    h.close()


def test_warm_start_solve(params):
    """Train on the states of one solve of 2000 scenarios, warm-start 300 new
    ones: same optimum as the closed form, fewer iterations than cold."""
    from paper_2607_15420_amd import Absorber, Mlp
    N = 10
    Ftr = feed_table(perturbations(2000, 0.2, 4), params)
    htr = Absorber(params, N, Ftr)
    xtr = torch.empty(htr.nx, dtype=torch.float64, device=DEV)
    r = htr.ipm_solve(x_out=xtr)
    assert r.status == 0
    Xtr = torch.empty((2000, 3), dtype=torch.float32, device=DEV)
    Ttr = torch.empty((2000, 21 * N), dtype=torch.float32, device=DEV)
    htr.warm_features(Xtr)
    htr.warm_targets(xtr, Ttr)
    net = Mlp(3, 256, 3, 21 * N, max_batch=512, seed=0)
    tr = net.train(Xtr, Ttr, net.default_train_options(epochs=150, batch=256, lr=2e-3))
    htr.close()
    Fte = feed_table(perturbations(300, 0.2, 3), params)
    h = Absorber(params, N, Fte)
    Xw = torch.empty((300, 3), dtype=torch.float32, device=DEV)
    Yw = torch.empty((300, 21 * N), dtype=torch.float32, device=DEV)
    x0 = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    h.warm_start(net, Xw, Yw, x0)
    xw = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    rw = h.ipm_solve(Absorber.default_options(warm_start=1), x0=x0, x_out=xw)
    rc = h.ipm_solve(Absorber.default_options())
    rs, used = h.warm_solve(net)  # library entry: warm start with cold fallback
    dstar, _, _, ok = simulate.closed_form_diameter(Fte, N, params)
    assert ok.all()
    assert rw.status == 0 and rw.E0 <= 1e-8, (rw.as_dict(), tr.final_loss)
    assert abs(rw.d - dstar) / dstar <= 1e-6
    assert rw.iterations < rc.iterations, (rw.iterations, rc.iterations)
    assert used and rs.status == 0 and rs.iterations == rw.iterations
    assert abs(rs.d - dstar) / dstar <= 1e-6
    print(f"warm {rw.iterations} iterations, cold {rc.iterations}; train loss {tr.final_loss:.2e}")
    h.close()
    net.close()


def test_primal_dual_encoding_roundtrip(params):
    """Multipliers are encoded as asinh(lambda / 1e-6); decoding gives them back for
    the worst scenario (largest hydraulic diameter) and zero for the others."""
    from paper_2607_15420_amd import Absorber
    w = CONFIGS["C1"]
    F = w.feeds(params)
    N, S = w.n_stages, F.shape[0]
    h = Absorber(params, N, F)
    x = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    lam = torch.empty(h.nc, dtype=torch.float64, device=DEV)
    r = h.ipm_solve(x_out=x, lam_out=lam)
    assert r.status == 0
    T = torch.empty((S, 43 * N), dtype=torch.float32, device=DEV)
    h.warm_targets(x, T, lam)
    x0 = torch.empty(h.nx, dtype=torch.float64, device=DEV)
    l0 = torch.empty(h.nc, dtype=torch.float64, device=DEV)
    h.warm_point(T, x0, l0, d_margin=0.0)
    torch.cuda.synchronize()
    lh, l0h = lam.cpu().numpy().reshape(S, N, 22), l0.cpu().numpy().reshape(S, N, 22)
    Z = x.cpu().numpy()[:-1].reshape(S, N, 21)
    P = M.OracleParams(params)
    dh = [simulate.hydraulic_diameter(Z[s], F[s], P) for s in range(S)]
    worst = int(np.argmax(dh))
    assert np.allclose(l0h[worst], lh[worst], rtol=1e-5, atol=1e-10)
    assert np.all(l0h[np.arange(S) != worst] == 0.0)
    assert x0.cpu().numpy()[-1] == pytest.approx(max(dh), rel=1e-6)
    h.close()


def test_primal_dual_network_from_batched_single_scenario_solves(params):
    """Training data from the batched solver (one single-scenario problem per
    training scenario, primal and dual solutions), a 43 N-output network, and the
    warm start with predicted multipliers reaches the closed form faster than cold."""
    from paper_2607_15420_amd import Absorber, Mlp
    N, n_train = 10, 2048
    Ftr = feed_table(perturbations(n_train, 0.2, 4), params)
    hb = Absorber.batch(params, [(N, Ftr[i:i + 1]) for i in range(n_train)])
    x = torch.empty(hb.nx, dtype=torch.float64, device=DEV)
    lam = torch.empty(hb.nc, dtype=torch.float64, device=DEV)
    rc, res = hb.batch_solve(x_out=x, lam_out=lam)
    assert rc == 0
    X = torch.empty((n_train, 3), dtype=torch.float32, device=DEV)
    T = torch.empty((n_train, 43 * N), dtype=torch.float32, device=DEV)
    hb.warm_features(X)
    hb.warm_targets(x, T, lam)
    hb.close()
    net = Mlp(3, 256, 3, 43 * N, max_batch=512, seed=0)
    tr = net.train(X, T, net.default_train_options(epochs=150, batch=256, lr=2e-3))
    Fte = feed_table(perturbations(300, 0.2, 3), params)
    h = Absorber(params, N, Fte)
    rc_ = h.ipm_solve()
    rw, used = h.warm_solve(net)
    dstar, _, _, ok = simulate.closed_form_diameter(Fte, N, params)
    assert ok.all() and used, (tr.final_loss, rw.as_dict())
    assert rw.status == 0 and rw.E0 <= 1e-8 and abs(rw.d - dstar) / dstar <= 1e-6
    assert rw.iterations < rc_.iterations, (rw.iterations, rc_.iterations)
    print(f"primal-dual warm {rw.iterations} iterations, cold {rc_.iterations}; train loss {tr.final_loss:.2e}")
    h.close()
    net.close()


# ---------------------------------------------------------------- the deployed shape
# the benchmarked warm-start network: 3 inputs, 3 hidden layers of 256, 430 outputs
# (43 per stage at 10 stages, padded to 448 columns on the device), 512-row chunks
DEPLOYED = dict(n_in=3, n_hidden=256, n_layers=3, n_out=430)


def test_forward_matches_oracle_at_the_deployed_shape():
    net, ps = _net(**DEPLOYED, seed=31, max_batch=512)
    rng = np.random.default_rng(32)
    im, isd = np.array([10.0, 0.12, 313.0]), np.array([1.2, 0.014, 36.0])
    om, osd = rng.standard_normal(430) * 2, rng.uniform(0.1, 3.0, 430)
    net.set_normalization(im, isd, om, osd)
    B = 1100  # three chunks of 512, the last one ragged
    X = im + isd * rng.standard_normal((B, 3))
    Y = torch.empty((B, 430), dtype=torch.float32, device=DEV)
    net.forward(_f32(X), Y)
    torch.cuda.synchronize()
    Xs = ((X - im.astype(np.float32)) / isd.astype(np.float32)).astype(np.float32).astype(np.float64)
    Yo, _ = O.forward(ps, Xs, quantize=True)
    Yo = Yo * osd.astype(np.float32) + om.astype(np.float32)
    Yd = Y.cpu().numpy()
    assert np.isfinite(Yd).all()
    assert np.abs(Yd - Yo).max() <= 5e-3 * np.abs(Yo).max()
    net.close()


def test_loss_grad_matches_oracle_at_the_deployed_shape():
    net, ps = _net(**DEPLOYED, seed=33, max_batch=512)
    rng = np.random.default_rng(34)
    B = 512
    X = rng.standard_normal((B, 3)).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((B, 430)).astype(np.float32).astype(np.float64)
    g = torch.empty(net.n_params, dtype=torch.float32, device=DEV)
    loss = net.loss_grad(_f32(X), _f32(T), g)
    lo, go = O.loss_and_grads(ps, X, T, quantize=True)
    assert loss == pytest.approx(lo, rel=2e-3)
    gg = _unflat(g.cpu().numpy(), ps)
    for l, ((gW, gb), (oW, ob)) in enumerate(zip(gg, go)):
        for a, b_ in ((gW, oW), (gb, ob)):
            assert np.linalg.norm(a - b_) <= 2e-2 * np.linalg.norm(b_), l
            assert np.abs(a - b_).max() <= 2e-2 * np.abs(b_).max(), l
    net.close()
