"""The selector network in FP64 numpy (oracle).

Test infrastructure only.  8 -> 64 -> 64 -> 2, tanh hidden layers, linear
output; loss = mean over all B x 2 outputs of (y - t)^2.  Parameters in one
vector: W1 (64 x 8), b1 (64), W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2).
The gradient is the chain rule written out layer by layer.
"""
from __future__ import annotations

import numpy as np

F, H, O = 8, 64, 2
SHAPES = ((H, F), (H,), (H, H), (H,), (O, H), (O,))
NPARAM = sum(int(np.prod(s)) for s in SHAPES)


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(w[o:o + k].reshape(s))
        o += k
    return out


def forward(w, X):
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ W3.T + b3
    return h1, h2, y


def loss(w, X, T):
    _, _, y = forward(w, X)
    return float(np.mean((y - np.asarray(T, dtype=np.float64)) ** 2))


def grad(w, X, T):
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    h1, h2, y = forward(w, X)
    dy = 2.0 * (y - T) / y.size                # d loss / d y
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dz2 = (dy @ W3) * (1.0 - h2 * h2)          # through tanh
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return np.concatenate([g.reshape(-1) for g in (gW1, gb1, gW2, gb2, gW3, gb3)])
