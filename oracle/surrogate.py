"""Float64 reference of the surrogate network -- TEST INFRASTRUCTURE ONLY.

The paper's hybrid decision making (section 1, Figure 1) trains machine-learning
models on scenario simulations and lets them make decisions.  Here the
scenario simulator is the exact plan evaluator and the model is an MLP that
predicts a plan's total route distance from its slotting alone (category ->
zone, encoded one-hot as a 64 x 64 matrix, row = category, column = zone).

Network: x (4096) -> Linear 1024 -> GELU -> Linear 256 -> GELU -> Linear 1.
GELU is the tanh form of Hendrycks & Gimpel (2016):
    gelu(u) = 0.5 u (1 + tanh(sqrt(2/pi) (u + 0.044715 u^3))).
Loss: mean squared error on standardised targets, L = mean_b (y_b - t_b)^2.
Optimiser: Adam (Kingma & Ba 2015) with bias correction.

Plain numpy in float64; the weight layout is W[in, out] (y = x @ W + b).
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

N_IN = 4096
N_H1 = 1024
N_H2 = 256
SQRT_2_OVER_PI = math.sqrt(2.0 / math.pi)


def one_hot(zone_of: np.ndarray, n_cat: int) -> np.ndarray:
    """``[n, 4096]``: x[b, c*64 + zone_of[b, c]] = 1 for c < n_cat, zero elsewhere."""
    zone_of = np.asarray(zone_of)
    n = zone_of.shape[0]
    x = np.zeros((n, 64, 64), dtype=np.float64)
    b = np.repeat(np.arange(n), n_cat)
    c = np.tile(np.arange(n_cat), n)
    x[b, c, zone_of[:, :n_cat].reshape(-1).astype(np.int64)] = 1.0
    return x.reshape(n, N_IN)


def gelu(u):
    return 0.5 * u * (1.0 + np.tanh(SQRT_2_OVER_PI * (u + 0.044715 * u ** 3)))


def gelu_grad(u):
    t = np.tanh(SQRT_2_OVER_PI * (u + 0.044715 * u ** 3))
    dt = (1.0 - t * t) * SQRT_2_OVER_PI * (1.0 + 3.0 * 0.044715 * u * u)
    return 0.5 * (1.0 + t) + 0.5 * u * dt


def init_params(seed: int) -> Dict[str, np.ndarray]:
    """He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero biases (float32 values)."""
    rng = np.random.default_rng([seed, 7])
    p = {}
    for name, (fi, fo) in (("W1", (N_IN, N_H1)), ("W2", (N_H1, N_H2)), ("W3", (N_H2, 1))):
        lim = math.sqrt(6.0 / fi)
        p[name] = rng.uniform(-lim, lim, size=(fi, fo)).astype(np.float32)
    p["b1"] = np.zeros(N_H1, np.float32)
    p["b2"] = np.zeros(N_H2, np.float32)
    p["b3"] = np.zeros(1, np.float32)
    return p


def forward(params, x) -> Tuple[np.ndarray, dict]:
    """Standardised prediction y [n] and the cache the backward pass needs."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], np.float64)
                              for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    u1 = x @ W1 + b1
    h1 = gelu(u1)
    u2 = h1 @ W2 + b2
    h2 = gelu(u2)
    y = (h2 @ W3)[:, 0] + b3[0]
    return y, dict(x=x, u1=u1, h1=h1, u2=u2, h2=h2)


def loss(params, x, t) -> float:
    y, _ = forward(params, x)
    return float(np.mean((y - t) ** 2))


def backward(params, cache, y, t) -> Dict[str, np.ndarray]:
    """Gradients of L = mean (y - t)^2 with respect to every parameter."""
    W2 = np.asarray(params["W2"], np.float64)
    W3 = np.asarray(params["W3"], np.float64)
    n = y.shape[0]
    dy = 2.0 * (y - t) / n                       # dL/dy
    g = {}
    g["W3"] = cache["h2"].T @ dy[:, None]
    g["b3"] = np.array([dy.sum()])
    dh2 = dy[:, None] @ W3.T
    du2 = dh2 * gelu_grad(cache["u2"])
    g["W2"] = cache["h1"].T @ du2
    g["b2"] = du2.sum(axis=0)
    dh1 = du2 @ W2.T
    du1 = dh1 * gelu_grad(cache["u1"])
    g["W1"] = cache["x"].T @ du1
    g["b1"] = du1.sum(axis=0)
    return g


def adam_step(params, grads, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); ``step`` counts from 1.  In place."""
    for k in params:
        m[k] = beta1 * m[k] + (1 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1 - beta2) * grads[k] ** 2
        mh = m[k] / (1 - beta1 ** step)
        vh = v[k] / (1 - beta2 ** step)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params, m, v


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).reshape(a.shape)


def spearman(a, b) -> float:
    """Spearman rank correlation with average ranks for ties."""
    def ranks(x):
        x = np.asarray(x, np.float64)
        order = np.argsort(x, kind="mergesort")
        r = np.empty(len(x), np.float64)
        sx = x[order]
        i = 0
        while i < len(x):
            j = i
            while j + 1 < len(x) and sx[j + 1] == sx[i]:
                j += 1
            r[order[i:j + 1]] = 0.5 * (i + j)
            i = j + 1
        return r
    ra, rb = ranks(a), ranks(b)
    ra -= ra.mean()
    rb -= rb.mean()
    return float((ra * rb).sum() / math.sqrt((ra * ra).sum() * (rb * rb).sum()))
