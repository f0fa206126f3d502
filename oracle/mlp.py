"""Float64 reference of the learned plan-cost model (TEST INFRASTRUCTURE).

y = W3^T tanh(W2^T tanh(W1^T x + b1) + b2) + b3, loss = mean((y - t)^2),
parameters flattened as W1[n_in][h], b1[h], W2[h][h], b2[h], W3[h], b3.
Plain numpy, written from the definitions: the forward pass, the gradient of
the loss by the chain rule (checked in the tests against central finite
differences of the loss itself), and one Adam update (Kingma and Ba, 2015:
beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected moments).
"""
from __future__ import annotations

import numpy as np


def unpack(p, n_in, h):
    p = np.asarray(p, dtype=np.float64)
    i = 0
    out = []
    for shape in ((n_in, h), (h,), (h, h), (h,), (h,), (1,)):
        size = int(np.prod(shape))
        out.append(p[i:i + size].reshape(shape))
        i += size
    assert i == p.size
    return out


def forward(p, x, n_in, h):
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, h)
    a1 = np.tanh(x @ W1 + b1)
    a2 = np.tanh(a1 @ W2 + b2)
    return a2 @ W3 + b3[0]


def loss(p, x, t, n_in, h):
    y = forward(p, x, n_in, h)
    return float(np.mean((y - t) ** 2))


def grad(p, x, t, n_in, h):
    """Gradient of loss() with respect to the flat parameter vector."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, h)
    B = x.shape[0]
    a1 = np.tanh(x @ W1 + b1)
    a2 = np.tanh(a1 @ W2 + b2)
    y = a2 @ W3 + b3[0]
    dy = 2.0 * (y - t) / B
    gW3 = a2.T @ dy
    gb3 = np.array([dy.sum()])
    dz2 = np.outer(dy, W3) * (1 - a2 ** 2)
    gW2 = a1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * (1 - a1 ** 2)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def numeric_grad(p, x, t, n_in, h, idx, eps=1e-6):
    """Central finite differences of loss() at the given parameter indices."""
    p = np.asarray(p, dtype=np.float64)
    out = []
    for i in idx:
        e = np.zeros_like(p)
        e[i] = eps
        out.append((loss(p + e, x, t, n_in, h) - loss(p - e, x, t, n_in, h)) / (2 * eps))
    return np.array(out)


def adam(p, g, m, v, step, lr):
    """One Adam update; returns (p, m, v)."""
    b1, b2, eps = 0.9, 0.999, 1e-8
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
