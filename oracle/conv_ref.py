"""FP64 reference of the warm-start network's layers (test infrastructure only).

A 3x3 convolution with dilation d and zero padding on NHWC tensors,
y[b, y, x, co] = bias[co] + sum_{tap, ci} w[co, tap, ci] x[b, y + d*dy, x + d*dx, ci]
with tap = 3*(dy + 1) + (dx + 1), an optional ReLU, and its gradients with
respect to the input, the weights and the bias; a mean-squared loss; Adam.
Plain numpy, one tap at a time, so a reader can check it by eye.  Used only
by the tests, which also pin it against scipy's 2-D correlation and finite
differences.
"""
from __future__ import annotations

import numpy as np


def _shift(x: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """s[b, y, x] = x[b, y + dy, x + dx], zero outside the image."""
    B, H, W, C = x.shape
    out = np.zeros_like(x)
    if abs(dy) >= H or abs(dx) >= W:
        return out     # the whole shifted window lies in the zero padding
    ys = slice(max(0, -dy), min(H, H - dy))
    xs = slice(max(0, -dx), min(W, W - dx))
    yt = slice(max(0, dy), min(H, H + dy))
    xt = slice(max(0, dx), min(W, W + dx))
    out[:, ys, xs, :] = x[:, yt, xt, :]
    return out


def conv3x3_fwd(x, w, b, dil, relu):
    """x [B,H,W,Cin], w [Cout, 9, Cin], b [Cout] -> (z, y) pre/post activation."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    z = np.zeros(x.shape[:3] + (w.shape[0],)) + np.asarray(b, dtype=np.float64)
    for tap in range(9):
        dy, dx = (tap // 3 - 1) * dil, (tap % 3 - 1) * dil
        z += _shift(x, dy, dx) @ w[:, tap, :].T
    y = np.maximum(z, 0.0) if relu else z
    return z, y


def conv3x3_bwd(x, z, dy_out, w, dil, relu):
    """Gradients (dx, dw, db) of sum(dy_out * y) for the layer above."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    dz = np.asarray(dy_out, dtype=np.float64) * ((z > 0) if relu else 1.0)
    db = dz.sum(axis=(0, 1, 2))
    dw = np.zeros_like(w)
    dx = np.zeros_like(x)
    for tap in range(9):
        sy, sx = (tap // 3 - 1) * dil, (tap % 3 - 1) * dil
        xs = _shift(x, sy, sx)
        dw[:, tap, :] = np.einsum("bhwo,bhwi->oi", dz, xs)
        dx += _shift(dz @ w[:, tap, :], -sy, -sx)
    return dx, dw, db


def adam(w, g, m, v, lr, b1, b2, eps, step):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
