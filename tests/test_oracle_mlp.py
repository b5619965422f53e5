"""Pins of the warm-start network oracle (oracle/mlp.py) against facts fixed by
the number format, the mathematics of GELU and Adam, and finite differences."""

import math

import numpy as np
import pytest

from oracle import mlp as O


# ----------------------------------------------------------------- bfloat16
def test_bf16_round_known_values():
    # bfloat16 has 7 stored mantissa bits: spacing 2^-7 just above 1
    e = 2.0 ** -7
    cases = {
        1.0: 1.0,
        1.0 + e: 1.0 + e,                 # representable
        1.0 + e / 2: 1.0,                 # tie, 1.0 has an even mantissa
        1.0 + 3 * e / 2: 1.0 + 2 * e,     # tie, rounds up to the even neighbour
        1.0 + e / 2 + 2.0 ** -20: 1.0 + e,  # just above the tie
        -(1.0 + 3 * e / 2): -(1.0 + 2 * e),
        3.0: 3.0,
        1.0 / 3.0: 0.333984375,           # 0x3EAB: 1.0101011b x 2^-2
        0.0: 0.0,
        65504.0: 65536.0,                 # float16 max is not a bfloat16 value
    }
    for x, want in cases.items():
        assert O.bf16_round(np.array([x]))[0] == want, x


def test_bf16_round_error_bound_and_idempotence():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(10000) * 10.0 ** rng.uniform(-10, 10, 10000)
    r = O.bf16_round(x)
    # relative error at most half a unit in the 8th significant bit
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))
    assert np.array_equal(O.bf16_round(r), r)


# ---------------------------------------------------------------------- GELU
def test_gelu_special_values():
    assert O.gelu(np.array([0.0]))[0] == 0.0
    # GELU(1) = Phi(1), textbook value of the normal CDF
    assert abs(O.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    x = np.linspace(-6, 6, 101)
    # Phi(x) + Phi(-x) = 1  =>  GELU(x) - GELU(-x) = x
    assert np.allclose(O.gelu(x) - O.gelu(-x), x, atol=1e-14)
    # tails: GELU -> x for large x, -> 0 for very negative x
    assert abs(O.gelu(np.array([40.0]))[0] - 40.0) < 1e-12
    assert abs(O.gelu(np.array([-40.0]))[0]) < 1e-12


def test_gelu_prime_matches_central_differences():
    x = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (O.gelu(x + h) - O.gelu(x - h)) / (2 * h)
    assert np.allclose(O.gelu_prime(x), fd, atol=1e-9)
    # GELU'(0) = Phi(0) = 1/2
    assert O.gelu_prime(np.array([0.0]))[0] == 0.5


# ------------------------------------------------------------------ backward
def _tiny():
    p = O.init_params(3, 7, 2, 5, seed=11)
    rng = np.random.default_rng(12)
    for W, b in p:
        b[:] = rng.standard_normal(b.shape) * 0.1
    X = rng.standard_normal((6, 3))
    T = rng.standard_normal((6, 5))
    return p, X, T


def test_gradients_match_central_differences():
    p, X, T = _tiny()
    _, grads = O.loss_and_grads(p, X, T, quantize=False)
    h = 1e-4
    worst = 0.0

    def loss_at(A, idx, v):
        old = A[idx]
        A[idx] = v
        r = O.mse(O.forward(p, X, False)[0], T)
        A[idx] = old
        return r

    for l in range(len(p)):
        for j in range(2):
            A = p[l][j]
            G = grads[l][j]
            for idx in np.ndindex(A.shape):
                x0 = A[idx]
                # fourth-order central difference
                fd = (-loss_at(A, idx, x0 + 2 * h) + 8 * loss_at(A, idx, x0 + h) - 8 * loss_at(A, idx, x0 - h)
                      + loss_at(A, idx, x0 - 2 * h)) / (12 * h)
                worst = max(worst, abs(fd - G[idx]) / max(1e-3, abs(fd)))
    assert worst <= 1e-7, worst


def test_single_linear_layer_gradient_closed_form():
    # no hidden layer: Y = X W^T + b, dL/dW = 2/(B n) (Y - T)^T X, dL/db = 2/(B n) sum (Y - T)
    rng = np.random.default_rng(3)
    W = rng.standard_normal((4, 3))
    b = rng.standard_normal(4)
    X = rng.standard_normal((9, 3))
    T = rng.standard_normal((9, 4))
    _, g = O.loss_and_grads([[W, b]], X, T, quantize=False)
    R = X @ W.T + b - T
    assert np.allclose(g[0][0], 2.0 / 36 * R.T @ X, rtol=1e-13, atol=1e-15)
    assert np.allclose(g[0][1], 2.0 / 36 * R.sum(0), rtol=1e-13, atol=1e-15)


def test_quantized_forward_is_close_to_exact():
    p, X, T = _tiny()
    Yq, _ = O.forward(p, X, True)
    Y, _ = O.forward(p, X, False)
    assert np.max(np.abs(Yq - Y)) <= 3e-2 * max(1.0, np.max(np.abs(Y)))
    assert not np.array_equal(Yq, Y)


# ---------------------------------------------------------------------- Adam
def test_adam_first_steps_closed_form():
    # with a constant gradient g, m_hat = g and v_hat = g^2 at every step, so each
    # step moves a weight by -lr * g / (|g| + eps)
    p = [[np.array([[1.0, -2.0]]), np.array([0.5])]]
    g = [(np.array([[0.3, -4.0]]), np.array([1e-3]))]
    opt = O.Adam(p)
    lr = 1e-2
    for k in range(1, 4):
        opt.step(p, g, lr)
        want_W = np.array([[1.0, -2.0]]) - k * lr * np.array([[0.3 / (0.3 + 1e-8), -4.0 / (4.0 + 1e-8)]])
        want_b = 0.5 - k * lr * 1e-3 / (1e-3 + 1e-8)
        assert np.allclose(p[0][0], want_W, rtol=0, atol=1e-15)
        assert abs(p[0][1][0] - want_b) < 1e-15


def test_cosine_schedule_endpoints():
    assert O.cosine_lr(1e-3, 0, 100) == 1e-3
    assert abs(O.cosine_lr(1e-3, 50, 100) - 5e-4) < 1e-18
    assert abs(O.cosine_lr(1e-3, 100, 100)) < 1e-18


def test_training_fits_a_smooth_map():
    # sanity of the whole loop: a smooth 3 -> 2 map is learned well below its variance
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (256, 3))
    T = np.stack([np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2], np.exp(0.5 * X[:, 2]) - X[:, 0]], axis=1)
    p = O.init_params(3, 32, 2, 2, seed=6)
    opt = O.Adam(p)
    l0 = O.mse(O.forward(p, X, False)[0], T)
    steps = 600
    for s in range(steps):
        idx = rng.choice(256, 64, replace=False)
        _, g = O.loss_and_grads(p, X[idx], T[idx], quantize=False)
        opt.step(p, g, O.cosine_lr(1e-2, s, steps))
    l1 = O.mse(O.forward(p, X, False)[0], T)
    assert l1 < 0.01 * l0, (l0, l1)
