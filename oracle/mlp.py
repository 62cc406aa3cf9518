"""FP64 NumPy reference of the per-pair degree model (test infrastructure only).

Written from the textbook definition of a fully connected network with tanh
hidden layers and a linear output, the mean squared error, and reverse-mode
differentiation (backpropagation).  Parameter layout of a model record:
W1[64][4], b1[64], W2[64][64], b2[64], W3[11][64], b3[11], then input mean[4],
scale[4], feature range lo[4], hi[4].
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 4, 64, 11
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)
N_MODEL = N_PARAMS + 4 * N_IN


def unpack(model):
    m = np.asarray(model, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = m[o:o + k].reshape(shape)
        o += k
    out["mean"], out["scale"] = m[o:o + 4], m[o + 4:o + 8]
    return out


def forward(model, feats):
    p = unpack(model)
    x = (np.asarray(feats, np.float64) - p["mean"]) * p["scale"]
    a1 = np.tanh(x @ p["W1"].T + p["b1"])
    a2 = np.tanh(a1 @ p["W2"].T + p["b2"])
    return a2 @ p["W3"].T + p["b3"], (x, a1, a2)


def loss(model, feats, targets):
    y, _ = forward(model, feats)
    t = np.asarray(targets, np.float64)
    ok = ~np.isnan(t)
    d = np.where(ok, y - np.where(ok, t, 0.0), 0.0)
    return float(np.sum(d * d) / ok.sum())


def grad(model, feats, targets):
    """Gradient of loss() with respect to the parameters (flat, record order)."""
    p = unpack(model)
    y, (x, a1, a2) = forward(model, feats)
    t = np.asarray(targets, np.float64)
    ok = ~np.isnan(t)
    dy = np.where(ok, 2.0 * (y - np.where(ok, t, 0.0)), 0.0) / ok.sum()
    gW3, gb3 = dy.T @ a2, dy.sum(0)
    dz2 = (dy @ p["W3"]) * (1.0 - a2 ** 2)
    gW2, gb2 = dz2.T @ a1, dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (1.0 - a1 ** 2)
    gW1, gb1 = dz1.T @ x, dz1.sum(0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])
