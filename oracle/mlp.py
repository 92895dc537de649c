"""Float64 reference of the selector network: forward pass, loss, gradients by
the chain rule, and the Adam update.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network: 12 features -> 64 -> 64 (ReLU) -> 7 logits, softmax over the classes
that are valid for the sample (join: partitioned GFTR, partitioned GFUR,
sort-merge GFTR; group-by: hash, sort, partition, sort on dictionary-encoded
keys), loss = mean over the batch of -log p[label]. Adam follows Kingma and
Ba (2015) with bias correction. Parameters are kept as a flat vector in the order
W1 (64x12, row-major), b1, W2 (64x64), b2, W3 (7x64), b3.
"""
from __future__ import annotations

import numpy as np

N_CLASSES = 7
JOIN_CLASSES = (0, 1, 6)
GROUPBY_CLASSES = (2, 3, 4, 5)
SHAPES = [(64, 12), (64,), (64, 64), (64,), (N_CLASSES, 64), (N_CLASSES,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)  # 5447


def unflatten(theta: np.ndarray):
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(theta[o:o + k].reshape(s))
        o += k
    return out


def init(seed: int) -> np.ndarray:
    """Kaiming-uniform weights (He et al. 2015): U(-sqrt(6/fan_in), +sqrt(6/fan_in)); zero biases."""
    g = np.random.Generator(np.random.Philox(seed))
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            lim = np.sqrt(6.0 / s[1])
            parts.append(g.uniform(-lim, lim, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def forward(theta: np.ndarray, X: np.ndarray, mask: np.ndarray):
    """Returns (probabilities [B, N_CLASSES], cache). mask[b, c] is 1 for valid classes."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ W3.T + b3
    logits = np.where(mask > 0, z3, -np.inf)
    m = logits.max(axis=1, keepdims=True)
    e = np.where(mask > 0, np.exp(logits - m), 0.0)
    p = e / e.sum(axis=1, keepdims=True)
    return p, (X, z1, h1, z2, h2, p)


def loss(theta, X, mask, y) -> float:
    p, _ = forward(theta, X, mask)
    return float(-np.mean(np.log(p[np.arange(len(y)), y])))


def grad(theta, X, mask, y):
    """(loss, gradient) by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta)
    p, (X, z1, h1, z2, h2, p) = forward(theta, X, mask)
    B = len(y)
    L = float(-np.mean(np.log(p[np.arange(B), y])))
    d3 = p.copy()
    d3[np.arange(B), y] -= 1.0
    d3 /= B                      # dL/dz3 (zero on masked classes since p = 0 there)
    gW3 = d3.T @ h2
    gb3 = d3.sum(axis=0)
    d2 = (d3 @ W3) * (z2 > 0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (z1 > 0)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    return L, np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1). Returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def predict(theta, X, mask) -> np.ndarray:
    p, _ = forward(theta, X, mask)
    return np.argmax(p, axis=1)
