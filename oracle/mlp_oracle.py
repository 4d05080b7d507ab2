"""FP64 reference for the learned cost model (a 3-layer perceptron).

TEST INFRASTRUCTURE ONLY (tests and the benchmark's CPU-baseline leg).

The model maps a feature vector f (64 values describing a fused pass) to a
predicted log run time:
    h1 = relu(W1 f + b1)      W1: 128 x 64
    h2 = relu(W2 h1 + b2)     W2: 128 x 128
    y  = W3 h2 + b3           W3: 1 x 128
Loss over a batch of B rows: L = (1/B) sum_i (y_i - t_i)^2.
Gradients are the analytic chain rule written out layer by layer; the Adam
update is Kingma & Ba's (bias-corrected first and second moments).
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

SIZES = (64, 128, 128, 1)


def init_params(seed: int) -> Dict[str, np.ndarray]:
    """He-uniform initial weights from a seeded generator (input to both the
    GPU trainer and this reference)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for i in range(3):
        fan_in, fan_out = SIZES[i], SIZES[i + 1]
        lim = np.sqrt(6.0 / fan_in)
        p[f"W{i + 1}"] = rng.uniform(-lim, lim, size=(fan_out, fan_in))
        p[f"b{i + 1}"] = np.zeros(fan_out)
    return p


def unflatten(flat: np.ndarray) -> Dict[str, np.ndarray]:
    """Flat parameter vector (W1, b1, W2, b2, W3, b3; W_i out x in) -> dict."""
    flat = np.asarray(flat, dtype=np.float64)
    p, o = {}, 0
    for i in range(3):
        fi, fo = SIZES[i], SIZES[i + 1]
        p[f"W{i + 1}"] = flat[o:o + fo * fi].reshape(fo, fi)
        o += fo * fi
        p[f"b{i + 1}"] = flat[o:o + fo].copy()
        o += fo
    assert o == flat.size
    return p


def flatten(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([p[f"{k}{i}"].ravel() for i in (1, 2, 3) for k in ("W", "b")])


def forward(p: Dict[str, np.ndarray], X: np.ndarray) -> Tuple[np.ndarray, Dict[str, np.ndarray]]:
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ p["W3"].T + p["b3"])[:, 0]
    return y, {"X": X, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def loss(p, X, t) -> float:
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def backward(p, X, t) -> Tuple[float, Dict[str, np.ndarray]]:
    """Returns the loss and dL/dparam for every parameter."""
    y, c = forward(p, X)
    t = np.asarray(t, dtype=np.float64)
    B = X.shape[0]
    dy = 2.0 * (y - t) / B                      # dL/dy
    g = {}
    g["W3"] = dy[None, :] @ c["h2"]            # 1 x 128
    g["b3"] = np.array([dy.sum()])
    dh2 = dy[:, None] * p["W3"]                # B x 128
    dz2 = dh2 * (c["z2"] > 0)
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (c["z1"] > 0)
    g["W1"] = dz1.T @ c["X"]
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean((y - t) ** 2)), g


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8) -> None:
    """One Adam update in place (step counts from 1)."""
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] ** 2
        mh = m[k] / (1 - beta1 ** step)
        vh = v[k] / (1 - beta2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
