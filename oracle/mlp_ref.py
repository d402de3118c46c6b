"""Reference for the learned branching scorer: TEST INFRASTRUCTURE ONLY.

The scorer is a 3-layer perceptron F -> H -> H -> 1 with ReLU, bf16 weights
and activations and fp32 accumulation, trained by mean squared error.  This
module computes it in float64 and rounds to bf16 (round to nearest, ties to
even) at exactly the points where the GPU kernels store bf16:

* forward:  Xb = bf16(X); A1 = bf16(relu(Xb W1b + b1)); A2 = bf16(relu(A1 W2b
  + b2)); y = A2 w3b + b3 (fp32 out), where W*b = bf16(W*) are the bf16 copies
  of the fp32 master weights;
* backward: dy = 2 (y - t) / B; dZ2 = bf16(dy w3b^T * [A2 > 0]);
  dZ1 = bf16(dZ2 W2b^T * [A1 > 0]); dW1 = Xb^T dZ1; db1 = sum dZ1;
  dW2 = A1^T dZ2; db2 = sum dZ2; dw3 = A2^T dy; db3 = sum dy.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), returned as
    float64.  Goes through float32 first (the GPU rounds fp32 values)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    is_nan = np.isnan(f)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(is_nan, np.nan, out)


def bf16_bits(x) -> np.ndarray:
    """The 16-bit patterns of bf16_round(x)."""
    return (bf16_round(x).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def init_params(rng: np.random.Generator, F: int = 16, H: int = 128):
    """He-style initial fp32 master weights."""
    return {
        "W1": (rng.standard_normal((F, H)) * np.sqrt(2.0 / F)).astype(np.float32),
        "b1": np.zeros(H, np.float32),
        "W2": (rng.standard_normal((H, H)) * np.sqrt(2.0 / H)).astype(np.float32),
        "b2": np.zeros(H, np.float32),
        "w3": (rng.standard_normal(H) * np.sqrt(1.0 / H)).astype(np.float32),
        "b3": np.zeros(1, np.float32),
    }


def forward(p, X, rounding: bool = True):
    """(y, cache).  rounding=False gives the exact float64 model (used by
    the finite-difference check)."""
    r = bf16_round if rounding else (lambda a: np.asarray(a, np.float64))
    Xb = r(X)
    W1, W2, w3 = r(p["W1"]), r(p["W2"]), r(p["w3"])
    b1, b2, b3 = (np.asarray(p[k], np.float64) for k in ("b1", "b2", "b3"))
    A1 = r(np.maximum(Xb @ W1 + b1, 0.0))
    A2 = r(np.maximum(A1 @ W2 + b2, 0.0))
    y = A2 @ w3 + b3[0]
    return y, dict(Xb=Xb, A1=A1, A2=A2, W2=W2, w3=w3)


def loss(p, X, t, rounding: bool = True) -> float:
    y, _ = forward(p, X, rounding)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def backward(p, X, t, rounding: bool = True):
    r = bf16_round if rounding else (lambda a: np.asarray(a, np.float64))
    y, c = forward(p, X, rounding)
    B = len(y)
    dy = 2.0 * (y - np.asarray(t, np.float64)) / B
    dZ2 = r(np.outer(dy, c["w3"]) * (c["A2"] > 0))
    dZ1 = r((dZ2 @ c["W2"].T) * (c["A1"] > 0))
    return {
        "W1": c["Xb"].T @ dZ1, "b1": dZ1.sum(axis=0),
        "W2": c["A1"].T @ dZ2, "b2": dZ2.sum(axis=0),
        "w3": c["A2"].T @ dy, "b3": np.array([dy.sum()]),
    }, y


def adam_step(p, g, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the fp32 master weights (in place); step >= 1."""
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] * g[k]
        mh = m[k] / (1 - beta1 ** step)
        vh = v[k] / (1 - beta2 ** step)
        p[k] = (p[k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
    return p
