"""Double-precision reference of the stop-rule perceptron's training objective.

TEST INFRASTRUCTURE ONLY (the GPU kernels' gradients are checked against it).

Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3, with
x in R^24, h1, h2 in R^64, z in R^2; parameters flattened as W1[64][24], b1,
W2[64][64], b2, W3[2][64], b3.  Objective over n samples with labels
(y0, c, y1, m):

    L = (1/n) sum_s [ c * (log(1 + e^z0) - y0 z0) + lam * m * (z1 - y1)^2 ]

Backward pass by the chain rule, written out layer by layer.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 24, 64, 2
SIZES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (OUT, HID)), ("b3", (OUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init(seed: int = 0):
    """He-style initial parameters (float32)."""
    g = np.random.default_rng(seed)
    d = {"W1": g.normal(0, np.sqrt(2 / IN), (HID, IN)), "b1": np.zeros(HID),
         "W2": g.normal(0, np.sqrt(2 / HID), (HID, HID)), "b2": np.zeros(HID),
         "W3": g.normal(0, np.sqrt(1 / HID), (OUT, HID)), "b3": np.zeros(OUT)}
    return pack(d).astype(np.float32)


def forward(p, X):
    w = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ w["W1"].T + w["b1"]
    h1 = np.maximum(a1, 0)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(a2, 0)
    z = h2 @ w["W3"].T + w["b3"]
    return z, (X, a1, h1, a2, h2)


def loss_and_grad(p, X, Y, lam=1.0):
    """Mean objective and its gradient (flat, float64)."""
    w = unpack(p)
    Y = np.asarray(Y, dtype=np.float64)
    n = len(Y)
    z, (X, a1, h1, a2, h2) = forward(p, X)
    y0, c, y1, m = Y[:, 0], Y[:, 1], Y[:, 2], Y[:, 3]
    z0, z1 = z[:, 0], z[:, 1]
    bce = np.logaddexp(0.0, z0) - y0 * z0
    loss = float(np.sum(c * bce + lam * m * (z1 - y1) ** 2) / n)
    sig = 1.0 / (1.0 + np.exp(-z0))
    dz = np.stack([c * (sig - y0) / n, 2.0 * lam * m * (z1 - y1) / n], axis=1)
    g = {"W3": dz.T @ h2, "b3": dz.sum(0)}
    dh2 = dz @ w["W3"]
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(0)
    dh1 = da2 @ w["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(0)
    return loss, pack(g)


def adam_step(p, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
