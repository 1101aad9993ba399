"""The 8-64-64-6 tanh network that predicts weight corrections, in FP64 (oracle, test infrastructure only).

Parameter vector layout (5126 entries):
  W1[64][8], b1[64], W2[64][64], b2[64], W3[6][64], b3[6]
y = 0.1 (W3 tanh(W2 tanh(W1 x + b1) + b2) + b3).
Backward is written out by the chain rule; Adam is the bias-corrected update
of Kingma and Ba.  Plain numpy, no fusion.
"""
from __future__ import annotations

import numpy as np

NI, NH, NO = 8, 64, 6
OUT_SCALE = 0.1
SIZES = [("W1", (NH, NI)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NO, NH)), ("b3", (NO,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SIZES:
        m = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + m], dtype=np.float64).reshape(shp)
        o += m
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def forward(theta, X):
    p = unpack(theta)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    y = OUT_SCALE * (h2 @ p["W3"].T + p["b3"])
    return y, (X, h1, h2)


def backward(theta, cache, dY):
    """Gradient of sum(dY * y) with respect to theta."""
    p = unpack(theta)
    X, h1, h2 = cache
    dz3 = OUT_SCALE * dY
    g = {"W3": dz3.T @ h2, "b3": dz3.sum(axis=0)}
    dz2 = (dz3 @ p["W3"]) * (1.0 - h2 * h2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (1.0 - h1 * h1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def adam_step(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
