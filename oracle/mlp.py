"""Oracle of the warm-start network: a plain NumPy float64 multilayer perceptron
with exact (erf) GELU, mean-squared-error loss, hand-written backward pass and
Adam, plus the bfloat16 rounding that the device network applies to its GEMM
operands.

TEST INFRASTRUCTURE ONLY (see oracle/model.py).

Network: inputs (n_in) -> [Linear -> GELU] x n_hidden_layers -> Linear ->
outputs (n_out).  Weights are stored as W[out][in] with bias b[out].

Precision model (quantize=True), mirroring where the device rounds: every GEMM
operand is a bfloat16 value -- the weights (rounded from their float32 master
copy), the layer inputs (features and GELU outputs) and the back-propagated
gradients dL/dZ -- while sums, biases, pre-activations, GELU and its derivative
are exact here (float32 on the device).  With quantize=False the network is
the plain float64 function, which is what the finite-difference pins check.

GELU(z) = z * Phi(z) with Phi the standard normal CDF (Hendrycks & Gimpel
2016, the erf form); Adam as in Kingma & Ba 2015, Algorithm 1.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def bf16_round(a) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), returned as float64.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 mantissa bits of
    an IEEE float32; the value is first rounded to float32 (as the device holds
    it) and then its low 16 bits are rounded away to nearest, ties to even.
    """
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def gelu(z: np.ndarray) -> np.ndarray:
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z: np.ndarray) -> np.ndarray:
    """d/dz z Phi(z) = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def layer_sizes(n_in: int, n_hidden: int, n_layers: int, n_out: int) -> list[tuple[int, int]]:
    """(out, in) of every linear layer."""
    dims = [n_in] + [n_hidden] * n_layers + [n_out]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def init_params(n_in: int, n_hidden: int, n_layers: int, n_out: int, seed: int):
    """He-normal weights, zero biases (float32 master values held as float64)."""
    rng = np.random.default_rng(seed)
    ps = []
    for o, i in layer_sizes(n_in, n_hidden, n_layers, n_out):
        W = rng.standard_normal((o, i)) * math.sqrt(2.0 / i)
        ps.append([W.astype(np.float32).astype(np.float64), np.zeros(o)])
    return ps


def forward(params, X: np.ndarray, quantize: bool):
    """Outputs Y (B, n_out) and the cache for backward."""
    q = bf16_round if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    H = q(X)
    cache = []
    L = len(params)
    for l, (W, b) in enumerate(params):
        Wq = q(W)
        Z = H @ Wq.T + b
        cache.append((H, Wq, Z))
        H = q(gelu(Z)) if l < L - 1 else Z
    return H, cache


def mse(Y: np.ndarray, T: np.ndarray) -> float:
    return float(np.mean((Y - T) ** 2))


def backward(params, cache, Y: np.ndarray, T: np.ndarray, quantize: bool):
    """Gradients [(dW, db)] of mse(Y, T) by the chain rule, layer by layer:
    G_L = 2 (Y - T) / (B n_out); dW_l = G_l^T H_{l-1}; db_l = sum_batch G_l;
    G_{l-1} = (G_l W_l) * GELU'(Z_{l-1})."""
    q = bf16_round if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    B, n_out = Y.shape
    G = q(2.0 * (Y - T) / (B * n_out))
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        H, Wq, _ = cache[l]
        grads[l] = (G.T @ H, G.sum(axis=0))
        if l > 0:
            Zp = cache[l - 1][2]
            G = q((G @ Wq) * gelu_prime(Zp))
    return grads


def loss_and_grads(params, X, T, quantize: bool):
    Y, cache = forward(params, X, quantize)
    return mse(Y, T), backward(params, cache, Y, T, quantize)


class Adam:
    """Adam with bias correction; one moment pair per parameter array."""

    def __init__(self, params, beta1=0.9, beta2=0.999, eps=1e-8):
        self.b1, self.b2, self.eps = beta1, beta2, eps
        self.m = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
        self.v = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
        self.t = 0

    def step(self, params, grads, lr: float):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for l, (gW, gb) in enumerate(grads):
            for j, g in enumerate((gW, gb)):
                self.m[l][j] = self.b1 * self.m[l][j] + (1.0 - self.b1) * g
                self.v[l][j] = self.b2 * self.v[l][j] + (1.0 - self.b2) * g * g
                mh = self.m[l][j] / c1
                vh = self.v[l][j] / c2
                params[l][j] = params[l][j] - lr * mh / (np.sqrt(vh) + self.eps)
        return params


def cosine_lr(lr0: float, step: int, total: int) -> float:
    """lr0 * (1 + cos(pi * step / total)) / 2."""
    return 0.5 * lr0 * (1.0 + math.cos(math.pi * step / max(total, 1)))
