"""GPU path against the CPU oracle, through the C ABI.

Evaluation: hand-derived residuals and derivatives (HIP) against the oracle's
residuals and autograd derivatives.  Linear algebra: the GPU block LDL^T with
the Schur complement on d against the oracle's dense Bunch-Kaufman per
scenario.  Tolerances: see each test.
"""

import math

import numpy as np
import pytest
import torch

from absorber_inputs import CONFIGS, feed_table
from oracle import model as M
from oracle.kkt import BorderedKKT, scenario_kkt

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _random_states(S, N, seed):
    rng = np.random.default_rng(seed)
    Z = np.empty((S, N, M.NV))
    Z[..., 0:9] = rng.uniform(0.01, 0.3, (S, N, 9))
    Z[..., 9:13] = rng.uniform(0.05, 0.5, (S, N, 4))
    Z[..., M.IL] = rng.uniform(30, 60, (S, N))
    Z[..., M.IV] = rng.uniform(5, 15, (S, N))
    Z[..., M.IT] = rng.uniform(300, 350, (S, N))
    Z[..., M.IE:] = rng.uniform(-1, 1, (S, N, 5))
    return Z, float(rng.uniform(0.3, 2.0))


# (stages, scenarios, feed table): 4 x 3 (two segments of 11 stages, the second
# ragged), and 10 x 23 (23 chains, 21 segments with a ragged last one, several
# evaluation blocks with a ragged tail)
@pytest.fixture(scope="module", params=[(4, 3, "C1"), (10, 23, "C2")], ids=["4x3", "10x23"])
def small(params, request):
    from paper_2607_15420_amd import Absorber
    N, S, cfg = request.param
    feeds = CONFIGS[cfg].feeds(params)[:S]
    h = Absorber(params, N, feeds)
    Z, d = _random_states(S, N, 11)
    x = np.concatenate([Z.reshape(-1), [d]])
    yield h, params, feeds, N, S, Z, d, x
    h.close()


def test_eval_cons(small):
    h, params, feeds, N, S, Z, d, x = small
    P = M.OracleParams(params)
    c = torch.empty(h.nc, dtype=torch.float64, device=DEV)
    h.eval_cons(_t(x), c)
    torch.cuda.synchronize()
    cg = c.cpu().numpy().reshape(S, N, M.NR)
    co = M.constraints(Z, d, feeds, P)
    # magnitude of the terms of each row: |J| |x| + |c|
    for w in range(S):
        J = M.jacobian(Z[w], d, feeds[w], P)
        mag = np.abs(J) @ np.abs(np.r_[Z[w].reshape(-1), d]) + np.abs(co[w].reshape(-1))
        err = np.abs(cg[w].reshape(-1) - co[w].reshape(-1))
        assert (err <= 1e-13 * mag + 1e-300).all(), err.max()


def test_eval_jac(small):
    h, params, feeds, N, S, Z, d, x = small
    P = M.OracleParams(params)
    rows, cols = h.jac_structure()
    vals = torch.empty(rows.size, dtype=torch.float64, device=DEV)
    h.eval_jac(_t(x), vals)
    torch.cuda.synchronize()
    v = vals.cpu().numpy()
    nzs = N * M.NV
    for w in range(S):
        Jo = M.jacobian(Z[w], d, feeds[w], P)  # (22N, 21N+1)
        Jg = np.zeros_like(Jo)
        sel = (rows >= w * N * M.NR) & (rows < (w + 1) * N * M.NR)
        r = rows[sel] - w * N * M.NR
        cc = cols[sel]
        cl = np.where(cc == h.nx - 1, nzs, cc - w * nzs)
        assert ((cl >= 0) & (cl <= nzs)).all()
        np.add.at(Jg, (r, cl), v[sel])
        scale = np.abs(Jo).max(axis=1, keepdims=True)
        assert np.abs(Jg - Jo).max() <= 1e-13 * scale.max()
        assert (np.abs(Jg - Jo) <= 1e-13 * scale).all()
        # nothing of the oracle's Jacobian lies outside the structure
        mask = np.zeros_like(Jo, dtype=bool)
        mask[r, cl] = True
        assert np.all(Jo[~mask] == 0.0)


def test_eval_hess(small):
    h, params, feeds, N, S, Z, d, x = small
    P = M.OracleParams(params)
    lam = np.random.default_rng(5).normal(size=(S, N, M.NR))
    rows, cols = h.hess_structure()
    vals = torch.empty(rows.size, dtype=torch.float64, device=DEV)
    h.eval_hess(_t(x), _t(lam.reshape(-1)), vals)
    torch.cuda.synchronize()
    v = vals.cpu().numpy()
    nzs = N * M.NV
    hdd = 0.0
    for w in range(S):
        Ho = M.lagrangian_hessian(Z[w], d, feeds[w], lam[w], P)
        hdd += Ho[-1, -1]
        Hg = np.zeros((nzs, nzs))
        sel = (rows < h.nx - 1) & (rows >= w * nzs) & (rows < (w + 1) * nzs)
        r, cc = rows[sel] - w * nzs, cols[sel] - w * nzs
        assert (r >= cc).all()
        Hg[r, cc] = v[sel]
        Hg = Hg + np.tril(Hg, -1).T
        scale = np.abs(Ho[:-1, :-1]).max()
        assert np.abs(Hg - Ho[:-1, :-1]).max() <= 1e-13 * scale
    assert v[-1] == pytest.approx(hdd, rel=1e-13)


def _oracle_bordered(params, feeds, N, Z, d, lam_s, cs, D, sig_x, sig_s, dw, dc):
    """The oracle's bordered KKT with the same scaling the GPU handle applies."""
    P = M.OracleParams(params)
    S = feeds.shape[0]
    blocks, borders, kdd = [], [], 0.0
    for w in range(S):
        bs = np.r_[np.tile(D[:M.NV], N), D[M.NV]]
        J = M.jacobian(Z[w], d, feeds[w], P) * cs[w].reshape(-1)[:, None] * bs[None, :]
        H = M.lagrangian_hessian(Z[w], d, feeds[w], lam_s[w] * cs[w], P) * bs[:, None] * bs[None, :]
        K, b, hdd = scenario_kkt(J, H, sig_x[w * N * M.NV:(w + 1) * N * M.NV], sig_s[w], dw, dc, N)
        blocks.append(K)
        borders.append(b)
        kdd += hdd
    kdd += sig_x[-1] + dw
    return BorderedKKT(blocks, borders, kdd)


def _to_oracle_order(v, S, N):
    """KKT vector [S][N][43] + d  ->  per-scenario [x (21N), yc (21N), yd (N)] lists and d."""
    a = v[:-1].reshape(S, N, M.NK if hasattr(M, "NK") else 43)
    out = []
    for w in range(S):
        out.append(np.concatenate([a[w, :, :21].reshape(-1), a[w, :, 21:42].reshape(-1), a[w, :, 42]]))
    return out, v[-1]


@pytest.mark.parametrize("dw,dc", [(0.0, 0.0), (1e-3, 1e-8)])
def test_kkt_factor_and_solve(small, dw, dc):
    h, params, feeds, N, S, Z, d, x = small
    rng = np.random.default_rng(17)
    P = M.OracleParams(params)
    # scaling like the interior-point method: variables by magnitude, rows by gradient
    D = np.r_[np.abs(Z[0, 0]) + 0.1, 1.0]
    cs = np.empty((S, N, M.NR))
    for w in range(S):
        bs = np.r_[np.tile(D[:M.NV], N), D[M.NV]]
        J = M.jacobian(Z[w], d, feeds[w], P) * bs[None, :]
        cs[w] = np.minimum(1.0, 100.0 / np.abs(J).max(axis=1)).reshape(N, M.NR)
    lam_s = rng.normal(scale=0.1, size=(S, N, M.NR))
    sig_x = rng.uniform(0.1, 10.0, S * N * M.NV + 1)
    sig_s = rng.uniform(0.5, 5.0, (S, N))
    h.set_scaling(D, _t(cs.reshape(-1)))
    inert = h.kkt_factor(_t(x), _t(lam_s.reshape(-1)), _t(sig_x), _t(sig_s.reshape(-1)), dw, dc)
    F = _oracle_bordered(params, feeds, N, Z, d, lam_s, cs, D, sig_x, sig_s, dw, dc)
    assert inert == F.inertia
    rhs = rng.normal(size=h.nkkt)
    sol = torch.empty(h.nkkt, dtype=torch.float64, device=DEV)
    rel = h.kkt_solve(_t(rhs), sol)
    assert rel <= 1e-10
    rs, rd = _to_oracle_order(rhs, S, N)
    xs, xd = F.solve(rs, rd)
    gs, gd = _to_oracle_order(sol.cpu().numpy(), S, N)
    # the relative residual the device reports is that of the returned solution (oracle's K),
    # up to the rounding of evaluating a residual: a few eps times max_i (|K||x|)_i / ||r||
    mag = max(float((np.abs(B.K) @ np.abs(xb) + np.abs(bb) * abs(gd)).max())
              for B, bb, xb in zip(F.blocks, F.borders, gs))
    bound = 64 * np.finfo(float).eps * mag / np.abs(rhs).max()
    assert abs(rel - F.rel_residual(gs, gd, rs, rd)) <= bound, (rel, bound)
    ref = max(np.abs(np.concatenate(xs)).max(), abs(xd))
    assert abs(gd - xd) <= 1e-9 * ref
    for a, b in zip(gs, xs):
        assert np.abs(a - b).max() <= 1e-9 * ref
    h.set_scaling(None, None)


def test_kkt_solve_before_factor_is_an_error(params):
    from paper_2607_15420_amd import Absorber, AbsorberError
    h = Absorber(params, 2, CONFIGS["C1"].feeds(params)[:1])
    rhs = torch.zeros(h.nkkt, dtype=torch.float64, device=DEV)
    with pytest.raises(AbsorberError):
        h.kkt_solve(rhs, torch.empty_like(rhs))
    h.close()


def test_profile_counts_timed_launches(small):
    """Event timing per kernel class: launches of the enabled classes are counted
    and timed; times are read when the profile is fetched."""
    h, params, feeds, N, S, Z, d, x = small
    lam = torch.zeros(S * N * M.NR, dtype=torch.float64, device=DEV)
    sig_x = torch.ones(h.nx, dtype=torch.float64, device=DEV)
    sig_s = torch.ones(S * N, dtype=torch.float64, device=DEV)
    h.profile_enable(True, mask=0b11)
    for _ in range(3):
        h.kkt_factor(_t(x), lam, sig_x, sig_s, 1e-2, 0.0)
    rhs = torch.ones(h.nkkt, dtype=torch.float64, device=DEV)
    h.kkt_solve(rhs, torch.empty_like(rhs))
    p = h.profile()
    assert p["factor"]["calls"] == 3 and p["factor"]["ms"] > 0.0
    assert p["solve"]["calls"] >= 1 and p["solve"]["ms"] > 0.0
    h.profile_enable(True, mask=0b01)  # resets; only the factorisation is timed now
    h.kkt_factor(_t(x), lam, sig_x, sig_s, 1e-2, 0.0)
    h.kkt_solve(rhs, torch.empty_like(rhs))
    p = h.profile()
    assert p["factor"]["calls"] == 1 and p["solve"]["calls"] == 0
    h.profile_enable(False)


def test_kkt_full_size_inertia_and_sampled_rows(params):
    """The benchmarked size (10 stages x 5000 scenarios, random states, variables
    scaled by magnitude).  With zero multipliers the Lagrangian Hessian vanishes,
    so the (1,1) block is Sigma_x + delta_w > 0 and the dual block is negative
    definite (-delta_c, slack terms): by Sylvester's law the inertia is exactly
    (nx, nc, 0).  The rows of sampled scenarios, rebuilt by the oracle from its
    own Jacobian, hold at the returned solution to the relative residual the
    device reports (its maximum over all rows bounds theirs).  Random states are
    not an interior-point iterate, so the refinement may stop above its 1e-10
    target; it must still stay well below 1e-6."""
    from paper_2607_15420_amd import Absorber
    w = CONFIGS["C3"]
    N, feeds = w.n_stages, w.feeds(params)
    S = feeds.shape[0]
    h = Absorber(params, N, feeds)
    Z, d = _random_states(S, N, 23)
    x = np.concatenate([Z.reshape(-1), [d]])
    D = np.r_[np.abs(Z[0, 0]) + 0.1, 1.0]
    h.set_scaling(D, None)
    rng = np.random.default_rng(29)
    lam = np.zeros(S * N * M.NR)
    sig_x = rng.uniform(0.1, 10.0, h.nx)
    sig_s = rng.uniform(0.5, 5.0, S * N)
    dw, dc = 1e-4, 1e-8
    inert = h.kkt_factor(_t(x), _t(lam), _t(sig_x), _t(sig_s), dw, dc)
    assert inert == (h.nx, h.nc, 0)
    rhs = rng.normal(size=h.nkkt)
    sol = torch.empty(h.nkkt, dtype=torch.float64, device=DEV)
    rel = h.kkt_solve(_t(rhs), sol)
    assert rel < 1e-6
    gs, gd = _to_oracle_order(sol.cpu().numpy(), S, N)
    rs, rd = _to_oracle_order(rhs, S, N)
    P = M.OracleParams(params)
    bs = np.r_[np.tile(D[:M.NV], N), D[M.NV]]
    eps = np.finfo(float).eps
    for s in sorted(rng.choice(S, 5, replace=False).tolist()):
        J = M.jacobian(Z[s], d, feeds[s], P) * bs[None, :]
        H = np.zeros((N * M.NV + 1, N * M.NV + 1))
        K, b, _ = scenario_kkt(J, H, sig_x[s * N * M.NV:(s + 1) * N * M.NV], sig_s[s * N:(s + 1) * N], dw, dc, N)
        res = rs[s] - K @ gs[s] - b * gd
        mag = np.abs(K) @ np.abs(gs[s]) + np.abs(b) * abs(gd)
        bound = 1.01 * rel * np.abs(rhs).max() + 64 * eps * mag.max()
        assert np.abs(res).max() <= bound, (s, np.abs(res).max(), bound)
    h.set_scaling(None, None)
    h.close()
