"""Reference of the warm-start network (oracle).  TEST INFRASTRUCTURE ONLY.

A two-hidden-layer MLP n_in -> h -> h -> n_out with ReLU, loss
L = mean over all outputs of (y - t)^2, and Adam (Kingma & Ba 2015,
Algorithm 1).  Parameters are packed as W1 (h x n_in), b1 (h), W2 (h x h),
b2 (h), W3 (n_out x h), b3 (n_out), row-major, each layer y = x W^T + b.
Everything in FP64 NumPy; backward by the chain rule written out per layer.
"""

from __future__ import annotations

import numpy as np


def sizes(ni: int, h: int, no: int):
    return [(h, ni), (h,), (h, h), (h,), (no, h), (no,)]


def param_count(ni: int, h: int, no: int) -> int:
    return h * ni + h + h * h + h + no * h + no


def unpack(p: np.ndarray, ni: int, h: int, no: int):
    out = []
    k = 0
    for shp in sizes(ni, h, no):
        cnt = int(np.prod(shp))
        out.append(p[k:k + cnt].reshape(shp))
        k += cnt
    return out


def pack(arrs) -> np.ndarray:
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in arrs])


def init_params(rng: np.random.Generator, ni: int, h: int, no: int) -> np.ndarray:
    """He-normal weights, zero biases."""
    W1 = rng.standard_normal((h, ni)) * np.sqrt(2.0 / ni)
    W2 = rng.standard_normal((h, h)) * np.sqrt(2.0 / h)
    W3 = rng.standard_normal((no, h)) * np.sqrt(2.0 / h)
    return pack([W1, np.zeros(h), W2, np.zeros(h), W3, np.zeros(no)])


def forward(p, x, ni, h, no):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, dtype=np.float64), ni, h, no)
    x = np.asarray(x, dtype=np.float64)
    H1 = np.maximum(x @ W1.T + b1, 0.0)
    H2 = np.maximum(H1 @ W2.T + b2, 0.0)
    Y = H2 @ W3.T + b3
    return Y, (x, H1, H2)


def loss_and_grads(p, x, t, ni, h, no):
    """L = mean((Y - T)^2) and dL/dp (packed)."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, dtype=np.float64), ni, h, no)
    Y, (x, H1, H2) = forward(p, x, ni, h, no)
    t = np.asarray(t, dtype=np.float64)
    D = Y - t
    L = float(np.mean(D * D))
    dY = 2.0 * D / D.size
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dH2 = (dY @ W3) * (H2 > 0)
    dW2 = dH2.T @ H1
    db2 = dH2.sum(axis=0)
    dH1 = (dH2 @ W2) * (H1 > 0)
    dW1 = dH1.T @ x
    db1 = dH1.sum(axis=0)
    return L, pack([dW1, db1, dW2, db2, dW3, db3])


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
