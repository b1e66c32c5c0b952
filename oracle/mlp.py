"""The slice-planner network in FP64 (test infrastructure).

An 80 -> 256 -> 256 -> 64 perceptron with ReLU hidden layers predicts the
normalised eigenvalue counts n_-(s_k)/n at 64 shifts from cheap band
features; its proposals are always judged by exact inertia (Section 3.1 uses
inertia, or the density of states, to partition the spectrum).  Every matrix
product takes its operands rounded to BF16 (round to nearest, ties to even),
as the GPU kernels do; sums, biases and the optimiser run in FP64 here.
Loss: mean squared error over the batch and the 64 outputs.  Optimiser: Adam
(Kingma and Ba 2015) with bias correction.

Pinned by: BF16 rounding against torch's bfloat16 conversion; finite
differences of the loss (rounding off) for the backward pass; a closed-form
single Adam step (tests).  Trained weights and predictions are parity
unpinned (stochastic training); the exactness of a plan never depends on
them.
"""
from __future__ import annotations

import numpy as np

SIZES = (80, 256, 256, 64)


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    x32 = np.asarray(x, dtype=np.float32)
    bits = x32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    r = ((bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(x32), np.nan, out)


def init_params(seed: int = 0) -> dict:
    """He-uniform weights W_l (fan_in x fan_out) and zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for l in range(3):
        fi, fo = SIZES[l], SIZES[l + 1]
        lim = np.sqrt(6.0 / fi)
        p[f"W{l + 1}"] = rng.uniform(-lim, lim, (fi, fo))
        p[f"b{l + 1}"] = np.zeros(fo)
    return p


def forward(p: dict, X: np.ndarray, rounding: bool = True):
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    Z1 = r(X) @ r(p["W1"]) + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = r(H1) @ r(p["W2"]) + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    Y = r(H2) @ r(p["W3"]) + p["b3"]
    return Y, (X, Z1, H1, Z2, H2)


def loss(p: dict, X: np.ndarray, T: np.ndarray, rounding: bool = True) -> float:
    Y, _ = forward(p, X, rounding)
    return float(np.mean((Y - T) ** 2))


def backward(p: dict, X: np.ndarray, T: np.ndarray, rounding: bool = True):
    """Loss and gradients of the mean squared error."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    Y, (X, Z1, H1, Z2, H2) = forward(p, X, rounding)
    B = X.shape[0]
    dY = 2.0 * (Y - T) / (B * Y.shape[1])
    g = {}
    g["W3"] = r(H2).T @ r(dY)
    g["b3"] = dY.sum(axis=0)
    dZ2 = (r(dY) @ r(p["W3"]).T) * (Z2 > 0)
    g["W2"] = r(H1).T @ r(dZ2)
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (r(dZ2) @ r(p["W2"]).T) * (Z1 > 0)
    g["W1"] = r(X).T @ r(dZ1)
    g["b1"] = dZ1.sum(axis=0)
    return float(np.mean((Y - T) ** 2)), g


def adam_step(p: dict, g: dict, state: dict, t: int, lr: float = 1e-3, b1: float = 0.9,
              b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (t >= 1) of every parameter, in place."""
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p
