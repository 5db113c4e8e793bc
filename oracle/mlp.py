"""FP64 reference of the segment-proposal network — TEST INFRASTRUCTURE ONLY.

Network: 12 inputs -> 64 ReLU -> 64 ReLU -> 2 sigmoid outputs (alpha_lo, alpha_hi).
Loss: mean over rows of the pinball (quantile) loss of each output against the target segment
opacity t: rho_q(t - y) = max(q (t - y), (q - 1)(t - y)), with q_lo for output 0 and q_hi for
output 1 (both outputs summed).

Parameter packing (shared convention with the library, not code): W1 [12][64] row-major
(input-major), b1 [64], W2 [64][64], b2 [64], W3 [64][2], b3 [2], all float.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 12, 64, 2
SHAPES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NOUT)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(w: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(w[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(w: np.ndarray, X: np.ndarray):
    """Returns (Y, cache) with Y = [n, 2] outputs in (0, 1)."""
    p = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["W3"] + p["b3"]
    y = 1.0 / (1.0 + np.exp(-z3))
    return y, (X, z1, h1, z2, h2, y)


def pinball(y: np.ndarray, t: np.ndarray, q_lo: float, q_hi: float) -> float:
    t = np.asarray(t, dtype=np.float64)
    total = 0.0
    for j, q in enumerate((q_lo, q_hi)):
        r = t - y[:, j]
        total += np.maximum(q * r, (q - 1.0) * r).sum()
    return total / len(t)


def backward(w: np.ndarray, X: np.ndarray, t: np.ndarray, q_lo: float, q_hi: float):
    """Returns (loss, dW) for the mean pinball loss; the subgradient at r = 0 is taken as
    (1 - q) (the y > t branch's slope is used when t <= y)."""
    p = unpack(w)
    y, (X, z1, h1, z2, h2, _) = forward(w, X)
    n = len(t)
    t = np.asarray(t, dtype=np.float64)
    dy = np.zeros_like(y)
    for j, q in enumerate((q_lo, q_hi)):
        dy[:, j] = np.where(t > y[:, j], -q, 1.0 - q) / n
    dz3 = dy * y * (1.0 - y)
    g = {"W3": h2.T @ dz3, "b3": dz3.sum(0)}
    dh2 = dz3 @ p["W3"].T
    dz2 = dh2 * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (z1 > 0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(0)
    return pinball(y, t, q_lo, q_hi), pack(g)


def init(rng: np.random.Generator) -> np.ndarray:
    """He-style initialisation, zero biases except a negative output bias (initial bounds low)."""
    p = {"W1": rng.normal(0, np.sqrt(2.0 / NIN), (NIN, NH)), "b1": np.zeros(NH),
         "W2": rng.normal(0, np.sqrt(2.0 / NH), (NH, NH)), "b2": np.zeros(NH),
         "W3": rng.normal(0, np.sqrt(1.0 / NH), (NH, NOUT)), "b3": np.array([-4.0, -2.0])}
    return pack(p)


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba), bias-corrected; returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
