"""FP64 reference of the extrapolation MLP -- TEST INFRASTRUCTURE ONLY.

A plain NumPy forward and backward pass of the network the GPU library
trains: F inputs -> 64 -> 64 -> O outputs, tanh hidden layers, weights
rounded to bfloat16 (round to nearest, ties to even) before use.  The O
outputs c mix the first O groups of nc inputs (the recorded updates):
yhat[j] = sum_k c_k x[k nc + j], and the loss is
L = sum_i |yhat_i - t_i|^2 / (2 n).  The gradient is the chain rule written
out layer by layer.  Weight layout: W1 [64][F], b1 [64], W2 [64][64],
b2 [64], W3 [O][64], b3 [O], row-major, concatenated.
"""
from __future__ import annotations

import numpy as np

HID = 64


def shapes(F, O):
    return [("W1", (HID, F)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (O, HID)), ("b3", (O,))]


def n_weights(F, O):
    return sum(int(np.prod(s)) for _, s in shapes(F, O))


def unpack(w, F, O):
    out, k = {}, 0
    for name, s in shapes(F, O):
        n = int(np.prod(s))
        out[name] = np.asarray(w[k:k + n], dtype=np.float64).reshape(s)
        k += n
    return out


def pack(parts, F, O):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in shapes(F, O)])


def bf16_round(w):
    """float32 values rounded to the nearest bfloat16 (ties to even)."""
    u = np.ascontiguousarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def forward(w, X, F, O):
    p = unpack(bf16_round(w), F, O)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    return h2 @ p["W3"].T + p["b3"]


def groups(X, O, nc):
    """The first O groups of nc inputs, shape (n, O, nc)."""
    return np.asarray(X, dtype=np.float64)[:, :O * nc].reshape(-1, O, nc)


def mix(c, X, nc):
    """yhat[i, j] = sum_k c[i, k] X[i, k nc + j]."""
    return np.einsum("ik,ikj->ij", np.asarray(c, dtype=np.float64), groups(X, c.shape[1], nc))


def loss_and_gradient(w, X, T, F, O, nc):
    """L and dL/dw (with respect to the rounded weights, as used)."""
    p = unpack(bf16_round(w), F, O)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    n = X.shape[0]
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    c = h2 @ p["W3"].T + p["b3"]
    r = mix(c, X, nc) - T
    L = 0.5 * np.sum(r * r) / n
    dy = np.einsum("ij,ikj->ik", r, groups(X, O, nc)) / n      # dL/dc
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    d2 = (dy @ p["W3"]) * (1.0 - h2 * h2)
    g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 * h1)
    g["W1"], g["b1"] = d1.T @ X, d1.sum(0)
    return L, pack(g, F, O)
