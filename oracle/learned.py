"""FP64 reference of the learned index's router network.

TEST INFRASTRUCTURE ONLY (the tests and the benchmark's baseline leg use it;
the product library never does).  It shares no code with the HIP path.

The network maps x in [0,1) to a scalar y (a CDF estimate):
    h1 = clip(w1 * x + b1, 0, 1)            w1 >= 0, 32 units
    h2 = clip(W2 @ h1 + b2, 0, 1)           W2 >= 0, 32 x 32
    y  = w3 . h2 + b3                       w3 >= 0
with the mean squared error against targets t.  Parameters travel as one
flat vector in the order w1[32], b1[32], W2[32][32] (row = output unit),
b2[32], w3[32], b3[1] (1153 values).  This module gives the forward pass,
the loss and its exact gradient (backpropagation written out from the chain
rule); its own tests pin the gradient against central finite differences.
"""
from __future__ import annotations

import numpy as np

H = 32
NPARAM = H + H + H * H + H + H + 1


def unpack(p):
    p = np.asarray(p, np.float64)
    o = 0
    w1 = p[o:o + H]; o += H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return w1, b1, W2, b2, w3, b3


def pack(w1, b1, W2, b2, w3, b3):
    return np.concatenate([w1, b1, np.asarray(W2).ravel(), b2, w3, [b3]]).astype(np.float64)


def forward(p, x):
    """(y, cache) for inputs x (1-D)."""
    w1, b1, W2, b2, w3, b3 = unpack(p)
    x = np.asarray(x, np.float64)
    a1 = np.outer(x, w1) + b1
    h1 = np.clip(a1, 0.0, 1.0)
    a2 = h1 @ W2.T + b2
    h2 = np.clip(a2, 0.0, 1.0)
    y = h2 @ w3 + b3
    return y, (x, a1, h1, a2, h2)


def loss(p, x, t):
    y, _ = forward(p, x)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def grad(p, x, t):
    """Gradient of the mean squared error, flat like p.  The clip's
    derivative is 1 strictly inside (0, 1) and 0 elsewhere."""
    w1, b1, W2, b2, w3, b3 = unpack(p)
    y, (x, a1, h1, a2, h2) = forward(p, x)
    t = np.asarray(t, np.float64)
    g = 2.0 * (y - t) / len(x)                       # dL/dy
    gw3 = h2.T @ g
    gb3 = g.sum()
    d2 = np.outer(g, w3) * ((a2 > 0.0) & (a2 < 1.0))  # dL/da2
    gW2 = d2.T @ h1
    gb2 = d2.sum(0)
    d1 = (d2 @ W2) * ((a1 > 0.0) & (a1 < 1.0))       # dL/da1
    gw1 = d1.T @ x
    gb1 = d1.sum(0)
    return pack(gw1, gb1, gW2, gb2, gw3, gb3)


def quantile_init(xs):
    """Ramp units between the 33 quantiles of the sample inputs, identity
    second layer, equal output weights: the network starts as the piecewise
    linear interpolant of the sample CDF through those quantiles."""
    xs = np.sort(np.asarray(xs, np.float64))
    q = xs[np.minimum((np.arange(H + 1) * len(xs)) // H, len(xs) - 1)]
    w1 = np.zeros(H)
    b1 = np.zeros(H)
    for j in range(H):
        span = max(q[j + 1] - q[j], 2.0 ** -24)   # a step becomes a steep ramp
        w1[j] = 1.0 / span
        b1[j] = -q[j] / span
    return pack(w1, b1, np.eye(H), np.zeros(H), np.full(H, 1.0 / H), 0.0)
