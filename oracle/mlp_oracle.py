"""FP64 CPU reference of the alpha-predictor network (addition, not from the paper).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network: 33 -> 64 -> 64 -> 1, GELU (exact erf form) after the two hidden layers,
mean-squared-error loss, Adam.  Flat parameter layout (6401 values):
    W1 [64 x 33] row-major (out, in) | b1 [64] | W2 [64 x 64] | b2 [64] | W3 [64] | b3 [1]
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

D_IN, D_H = 33, 64
SIZES = [("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)),
         ("W3", (D_H,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)  # 6401


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.ravel(parts[name]) for name, _ in SIZES])


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(theta: np.ndarray, X: np.ndarray):
    """X: (B, 33) -> (out (B,), cache)."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    h1 = X @ p["W1"].T + p["b1"]
    a1 = gelu(h1)
    h2 = a1 @ p["W2"].T + p["b2"]
    a2 = gelu(h2)
    out = a2 @ p["W3"] + p["b3"][0]
    return out, (X, h1, a1, h2, a2)


def loss_and_grad(theta: np.ndarray, X: np.ndarray, y: np.ndarray):
    """MSE = mean((out - y)^2) and its gradient with respect to theta (backpropagation)."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    out, (X, h1, a1, h2, a2) = forward(theta, X)
    B = X.shape[0]
    r = out - np.asarray(y, dtype=np.float64)
    loss = float(np.mean(r * r))
    dout = 2.0 * r / B
    g = {}
    g["W3"] = dout @ a2
    g["b3"] = np.array([dout.sum()])
    dh2 = np.outer(dout, p["W3"]) * gelu_grad(h2)
    g["W2"] = dh2.T @ a1
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ p["W2"]) * gelu_grad(h1)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(0)
    return loss, pack(g)


def init_params(rng: np.random.Generator) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases."""
    parts = {}
    for name, shape in SIZES:
        fan_in = D_IN if name in ("W1", "b1") else D_H
        a = 1.0 / math.sqrt(fan_in)
        parts[name] = rng.uniform(-a, a, size=shape)
    return pack(parts)


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), returning new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
