"""FP64 reference of the PAH-emission surrogate network (TEST INFRASTRUCTURE ONLY).

Network: x (n_in) -> SiLU(W1 x + b1) (n_h) -> SiLU(W2 h1 + b2) (n_h) -> W3 h2 + b3 (n_out),
trained by mean squared error with Adam.  ``bf16=True`` rounds, to bfloat16
(round to nearest even), exactly the tensors the GPU keeps in bfloat16: the
input, the weights and the stored activations in the forward pass, and the
output/pre-activation gradients that enter the backward products.  Products
and sums are then done in FP64, so a GPU result differs from this one only
by its FP32 accumulation order.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return out.reshape(np.shape(a))


def _q(a, bf16):
    return bf16_round(a) if bf16 else np.asarray(a, dtype=np.float64)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def init_params(n_in=200, n_h=256, n_out=217, seed=4):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, (o, i) in dict(W1=(n_h, n_in), W2=(n_h, n_h), W3=(n_out, n_h)).items():
        lim = 1.0 / np.sqrt(i)
        p[name] = rng.uniform(-lim, lim, size=(o, i))
    p["b1"], p["b2"], p["b3"] = np.zeros(n_h), np.zeros(n_h), np.zeros(n_out)
    return p


def forward(p, X, bf16=False):
    X = _q(X, bf16)
    W1, W2, W3 = (_q(p[k], bf16) for k in ("W1", "W2", "W3"))
    Z1 = X @ W1.T + p["b1"]
    H1 = _q(silu(Z1), bf16)
    Z2 = H1 @ W2.T + p["b2"]
    H2 = _q(silu(Z2), bf16)
    Y = H2 @ W3.T + p["b3"]
    return Y, dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2, W1=W1, W2=W2, W3=W3)


def mse(Y, T):
    """Mean over all elements of (Y - T)^2 and its gradient."""
    d = Y - T
    return float((d * d).mean()), 2.0 * d / d.size


def backward(cache, dY, bf16=False):
    dY = _q(dY, bf16)
    g = {"W3": dY.T @ cache["H2"], "b3": dY.sum(0)}
    dZ2 = _q((dY @ cache["W3"]) * silu_grad(cache["Z2"]), bf16)
    g["W2"] = dZ2.T @ cache["H1"]
    g["b2"] = dZ2.sum(0)
    dZ1 = _q((dZ2 @ cache["W2"]) * silu_grad(cache["Z1"]), bf16)
    g["W1"] = dZ1.T @ cache["X"]
    g["b1"] = dZ1.sum(0)
    g["X"] = dZ1 @ cache["W1"]
    return g


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; t counts from 1."""
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mh = m[k] / (1.0 - beta1 ** t)
        vh = v[k] / (1.0 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v
