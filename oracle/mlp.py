"""FP64 reference of the learned warm start's network (oracle; test
infrastructure only).

Not part of the paper: the learned form predicts an IPM starting point.  The
network is a plain multilayer perceptron

    z1 = x W1^T + b1,  a1 = gelu(z1)
    z2 = a1 W2^T + b2, a2 = gelu(z2)
    out = a2 W3^T + b3

with gelu(x) = x Phi(x) = (x / 2)(1 + erf(x / sqrt 2)), trained on the mean
squared error  loss = (1 / 2B) sum_b ||out_b - t_b||^2  with Adam
(Kingma and Ba, 2015: bias-corrected first and second moments).  Written
from those definitions; the gradients are the chain rule, pinned in the
tests by central finite differences.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np
from scipy.special import erf

Params = List[Tuple[np.ndarray, np.ndarray]]   # [(W [out x in], b [out])] per layer

SQRT2 = np.sqrt(2.0)
INV_SQRT_2PI = 1.0 / np.sqrt(2.0 * np.pi)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def gelu_grad(x):
    """d gelu / dx = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * INV_SQRT_2PI * np.exp(-0.5 * x * x)


def forward(params: Params, x: np.ndarray):
    """Returns the output and the per-layer (input, pre-activation) cache."""
    cache = []
    a = np.asarray(x, dtype=np.float64)
    for i, (W, b) in enumerate(params):
        z = a @ W.T + b
        cache.append((a, z))
        a = gelu(z) if i + 1 < len(params) else z
    return a, cache


def loss_and_grad(params: Params, x: np.ndarray, t: np.ndarray):
    out, cache = forward(params, x)
    B = x.shape[0]
    diff = out - t
    loss = 0.5 * float(np.sum(diff * diff)) / B
    grads: Params = [None] * len(params)
    dz = diff / B
    for i in range(len(params) - 1, -1, -1):
        a_in, _ = cache[i]
        W, _ = params[i]
        grads[i] = (dz.T @ a_in, dz.sum(axis=0))
        if i > 0:
            dz = (dz @ W) * gelu_grad(cache[i - 1][1])
    return loss, grads


def adam_init(params: Params):
    return dict(t=0, m=[[np.zeros_like(W), np.zeros_like(b)] for W, b in params],
                v=[[np.zeros_like(W), np.zeros_like(b)] for W, b in params])


def adam_step(params: Params, grads: Params, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8) -> Params:
    """m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
    p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)."""
    state["t"] += 1
    t = state["t"]
    out = []
    for i, (layer, glayer) in enumerate(zip(params, grads)):
        new = []
        for j in range(2):
            g = glayer[j]
            m = b1 * state["m"][i][j] + (1.0 - b1) * g
            v = b2 * state["v"][i][j] + (1.0 - b2) * g * g
            state["m"][i][j], state["v"][i][j] = m, v
            new.append(layer[j] - lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps))
        out.append((new[0], new[1]))
    return out


def flatten(params: Params) -> np.ndarray:
    """[W1, b1, W2, b2, ...] row-major, the library's parameter layout."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(flat: np.ndarray, dims) -> Params:
    out, o = [], 0
    for din, dout in zip(dims[:-1], dims[1:]):
        W = flat[o:o + dout * din].reshape(dout, din)
        o += dout * din
        b = flat[o:o + dout]
        o += dout
        out.append((np.array(W, dtype=np.float64), np.array(b, dtype=np.float64)))
    return out
