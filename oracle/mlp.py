"""Float64 reference of the 8-64-64-3 cost-model network (test infrastructure only).

The learned cost model is not part of the paper (parity unpinned with
respect to the paper).  It maps features of (q, d, n, c_total) to the natural
log of the three stage times of Eq. (runtime_decomp) (T_pre, T_sub, T_merge).
Gradients here are pinned by central finite differences in the tests.

Network: h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 W3 + b3.
Loss: mean squared error over rows and the three outputs.
Optimiser: Adam (Kingma and Ba, 2015) with bias correction.

Flat parameter layout (4931 values): W1[8][64] row-major, b1[64],
W2[64][64], b2[64], W3[64][3], b3[3].
"""

from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

N_IN, N_H, N_OUT = 8, 64, 3
SHAPES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_H, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(flat: np.ndarray) -> Dict[str, np.ndarray]:
    flat = np.asarray(flat, dtype=np.float64)
    out, off = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = flat[off:off + size].reshape(shape)
        off += size
    return out


def flatten(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def features(q: int, d: int, n: int, c_total: int) -> np.ndarray:
    """Input encoding: centred and scaled (q, log2 d, n, c_total), then the cost terms of
    Table I for equal blocks and evenly spread cuts: log2 N_sub (N_sub = sum over segments
    of 2^{c_i}, c_i the cuts on the segment's boundaries), the largest segment q_max =
    ceil(q / n), log2 (N_sub 2^{q_max} d) (subcircuit stage) and log2 (2^{c_total} 2^q)
    (merge, K = 2^{c_total} terms).  Uncut rows use n = 1, c_total = 0, N_sub = 1, q_max = q."""
    ld = math.log2(d)
    lsub, qmax = 0.0, q
    if n >= 2:
        nb = n - 1
        cb = [c_total // nb + (1 if b < c_total % nb else 0) for b in range(nb)]
        ci = [(cb[i - 1] if i > 0 else 0) + (cb[i] if i < nb else 0) for i in range(n)]
        lsub = math.log2(sum(2.0 ** c for c in ci))
        qmax = -(-q // n)
    return np.array([(q - 24.0) / 8.0, ld - math.log2(20.0), (n - 3.0), (c_total - 4.0) / 4.0,
                     (lsub - 6.0) / 4.0, (qmax - 12.0) / 4.0, (lsub + qmax + ld - 24.0) / 6.0,
                     (c_total + q - 30.0) / 6.0])


def forward(flat: np.ndarray, x: np.ndarray) -> Tuple[np.ndarray, dict]:
    p = unflatten(flat)
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ p["W1"] + p["b1"]
    h1 = np.tanh(a1)
    a2 = h1 @ p["W2"] + p["b2"]
    h2 = np.tanh(a2)
    y = h2 @ p["W3"] + p["b3"]
    return y, {"x": x, "h1": h1, "h2": h2}


def loss(y: np.ndarray, t: np.ndarray) -> float:
    return float(np.mean((y - t) ** 2))


def backward(flat: np.ndarray, cache: dict, y: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Gradient of the mean squared error with respect to the flat parameters."""
    p = unflatten(flat)
    rows = y.shape[0]
    gy = 2.0 * (y - t) / (rows * N_OUT)
    g = {}
    g["W3"] = cache["h2"].T @ gy
    g["b3"] = gy.sum(axis=0)
    gh2 = gy @ p["W3"].T
    ga2 = gh2 * (1.0 - cache["h2"] ** 2)
    g["W2"] = cache["h1"].T @ ga2
    g["b2"] = ga2.sum(axis=0)
    gh1 = ga2 @ p["W2"].T
    ga1 = gh1 * (1.0 - cache["h1"] ** 2)
    g["W1"] = cache["x"].T @ ga1
    g["b1"] = ga1.sum(axis=0)
    return flatten(g)


def adam_step(flat, grad, m, v, step: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return flat - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(flat0, x, t, epochs: int, lr: float):
    """Full-batch Adam training; returns final parameters and the loss history."""
    flat = np.array(flat0, dtype=np.float64)
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)
    hist = []
    for e in range(1, epochs + 1):
        y, cache = forward(flat, x)
        hist.append(loss(y, t))
        g = backward(flat, cache, y, t)
        flat, m, v = adam_step(flat, g, m, v, e, lr)
    return flat, hist
