"""FP64 reference of the row-size predictor (TEST INFRASTRUCTURE ONLY).

The predictor is not part of the paper: it sizes each output row's
accumulator without a symbolic pass.  The paper motivates it: computing the
output's structure up front is about as hard as the product itself
(Section 3), and the work of a row is what flops(A,B) counts (Section 2).

Network: features x = (log1p nnz(A(i,:)), log1p flops_i, log1p max_k nnz(B(k,:)))
  h1 = relu(W1 x + b1)      W1: 32 x 3
  h2 = relu(W2 h1 + b2)     W2: 32 x 32
  y  = w3 . h2 + b3         w3: 32
y estimates log1p nnz(C(i,:)).  Parameters are one flat float vector in the
order W1 (row-major), b1, W2 (row-major), b2, w3, b3: 1217 values.

Loss over N rows with targets t = log1p nnz(C(i,:)):
  L = (1/N) sum_i a_i (y_i - t_i)^2,  a_i = alpha if y_i < t_i else 1,
so under-prediction (which overflows a sized accumulator) costs alpha times
more.  Capacity of a row: clamp(ceil((1 + margin) expm1(y)) + 8, lower =
max_k nnz(B(k,:)), upper = min(flops_i, n)); both bounds are exact bounds
of nnz(C(i,:)).

Only the tests and the benchmark's baseline may import this module.
"""

from __future__ import annotations

import numpy as np

H = 32
NPARAMS = 3 * H + H + H * H + H + H + 1  # 1217


def unpack(p: np.ndarray):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (NPARAMS,)
    o = 0
    W1 = p[o:o + 3 * H].reshape(H, 3); o += 3 * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def features(nnz_a, flops, maxb) -> np.ndarray:
    return np.stack([np.log1p(np.asarray(nnz_a, np.float64)), np.log1p(np.asarray(flops, np.float64)),
                     np.log1p(np.asarray(maxb, np.float64))], axis=1)


def forward(p, X):
    """y (N,) and the intermediate values needed by backward."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (X, z1, h1, z2, h2)


def loss(p, X, t, alpha: float) -> float:
    y, _ = forward(p, X)
    d = y - np.asarray(t, np.float64)
    a = np.where(d < 0.0, alpha, 1.0)
    return float(np.mean(a * d * d))


def backward(p, X, t, alpha: float) -> np.ndarray:
    """Analytic gradient of the loss with respect to the flat parameters
    (chain rule through the two ReLU layers)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    y, (X, z1, h1, z2, h2) = forward(p, X)
    N = X.shape[0]
    d = y - np.asarray(t, np.float64)
    a = np.where(d < 0.0, alpha, 1.0)
    gy = 2.0 * a * d / N                    # dL/dy
    g_w3 = h2.T @ gy
    g_b3 = gy.sum()
    g_h2 = np.outer(gy, w3)                 # N x H
    g_z2 = g_h2 * (z2 > 0.0)
    g_W2 = g_z2.T @ h1
    g_b2 = g_z2.sum(axis=0)
    g_h1 = g_z2 @ W2
    g_z1 = g_h1 * (z1 > 0.0)
    g_W1 = g_z1.T @ X
    g_b1 = g_z1.sum(axis=0)
    return pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def capacity(y, maxb, flops, n: int, margin: float) -> np.ndarray:
    pred = np.expm1(np.asarray(y, np.float64))
    cap = np.ceil((1.0 + margin) * pred) + 8.0
    lo = np.asarray(maxb, np.float64)
    hi = np.minimum(np.asarray(flops, np.float64), float(n))
    return np.minimum(np.maximum(cap, lo), hi).astype(np.int64)


def init_params(seed: int = 0) -> np.ndarray:
    """He-style random initialisation (input generator for tests)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0.0, np.sqrt(2.0 / 3), (H, 3))
    W2 = rng.normal(0.0, np.sqrt(2.0 / H), (H, H))
    w3 = rng.normal(0.0, np.sqrt(1.0 / H), H)
    return pack(W1, np.zeros(H) + 0.01, W2, np.zeros(H) + 0.01, w3, 0.0)
