"""CPU oracle for the variant-selector MLP -- TEST INFRASTRUCTURE ONLY.

FP64 numpy definitions of the network the GPU trains and runs:

    h1  = relu(X @ W1 + b1)
    h2  = relu(h1 @ W2 + b2)
    out = h2 @ W3 + b3                      (predicted log2 time per variant)

    loss = sum(M * (out - Y)^2) / max(sum(M), 1)    (masked mean squared error)

Backward is the chain rule written out by hand (no autograd). The optimiser is
Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization", ICLR 2015,
Algorithm 1) with bias correction. Weight layout: W is [fan_in, fan_out],
row-major, matching the GPU kernels' argument layout. The selector is not part
of the paper; it chooses among edgeMap variants, which per the paper's API
study change only the running time, never the result.
"""
from __future__ import annotations

import numpy as np

PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def shapes(F: int, H: int, K: int):
    return {"W1": (F, H), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (H, K), "b3": (K,)}


def forward(p, X):
    X = np.asarray(X, np.float64)
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    out = h2 @ p["W3"] + p["b3"]
    return out, (X, z1, h1, z2, h2)


def loss(out, Y, M):
    M = np.asarray(M, np.float64)
    den = max(float(M.sum()), 1.0)
    r = out - Y
    return float((M * r * r).sum() / den)


def loss_grad(out, Y, M):
    """d loss / d out."""
    M = np.asarray(M, np.float64)
    den = max(float(M.sum()), 1.0)
    return 2.0 * M * (out - Y) / den


def backward(p, cache, dout):
    X, z1, h1, z2, h2 = cache
    g = {}
    g["W3"] = h2.T @ dout
    g["b3"] = dout.sum(axis=0)
    dh2 = dout @ p["W3"].T
    dz2 = dh2 * (z2 > 0.0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (z1 > 0.0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g


def loss_and_grads(p, X, Y, M):
    out, cache = forward(p, X)
    return loss(out, Y, M), backward(p, cache, loss_grad(out, Y, M))


def adam_step(p, g, state, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); state holds 'm' and 'v' dicts."""
    for k in PARAM_NAMES:
        m = state["m"][k] = beta1 * state["m"][k] + (1.0 - beta1) * g[k]
        v = state["v"][k] = beta2 * state["v"][k] + (1.0 - beta2) * g[k] * g[k]
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        p[k] = p[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return p


def adam_init(p):
    return {"m": {k: np.zeros_like(p[k]) for k in PARAM_NAMES},
            "v": {k: np.zeros_like(p[k]) for k in PARAM_NAMES}}


def train(p, X, Y, M, steps, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Full-batch Adam for `steps` steps; returns (params, per-step losses)."""
    p = {k: np.array(v, np.float64, copy=True) for k, v in p.items()}
    st = adam_init(p)
    losses = []
    for t in range(1, steps + 1):
        L, g = loss_and_grads(p, X, Y, M)
        losses.append(L)
        adam_step(p, g, st, t, lr, beta1, beta2, eps)
    return p, losses


def predict_argmin(p, X, allowed=None):
    """Index of the smallest predicted time per row (ties -> lowest index)."""
    out, _ = forward(p, X)
    if allowed is not None:
        out = np.where(np.asarray(allowed, bool), out, np.inf)
    return np.argmin(out, axis=1)


def selector_features(k, degsum, unvisited, n, m, max_deg, cv, dense_in):
    """Raw features of one edgeMap level, in FP64, as the selector defines them:
    log2(1+k), log2(1+sum deg U), log2(1+unvisited), log2(1+n), log2(1+m),
    (k + sum deg U)/(m+1), k/(n+1), log2(1+max degree), degree CV,
    log2(1 + sum deg U/(k+1)), unvisited/(n+1), dense-only flag."""
    import math
    return [math.log2(1 + k), math.log2(1 + degsum), math.log2(1 + unvisited), math.log2(1 + n),
            math.log2(1 + m), (k + degsum) / (m + 1), k / (n + 1), math.log2(1 + max_deg), cv,
            math.log2(1 + degsum / (k + 1)), unvisited / (n + 1), float(dense_in)]
