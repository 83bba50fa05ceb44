"""Plain FP64 reference of the warm-start MLP (forward, mean-squared loss and
backward) in numpy.

TEST INFRASTRUCTURE ONLY: used by tests to check the HIP network's outputs and
gradients; the product never imports it.

Network: x (15) -> W1 x + b1 -> GELU -> W2 . + b2 -> GELU -> W3 . + b3 -> y;
GELU(z) = z Phi(z) with Phi the standard normal CDF; loss = mean (y - t)^2.
Parameters are one flat vector laid out W1[w x 15], b1[w], W2[w x w], b2[w],
W3[1 x w], b3[1] (row-major).
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT = 15

_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + _erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def unpack(p, width: int):
    p = np.asarray(p, dtype=np.float64)
    F, W = N_FEAT, width
    o = 0
    W1 = p[o:o + W * F].reshape(W, F); o += W * F
    b1 = p[o:o + W]; o += W
    W2 = p[o:o + W * W].reshape(W, W); o += W * W
    b2 = p[o:o + W]; o += W
    W3 = p[o:o + W].reshape(1, W); o += W
    b3 = p[o:o + 1]; o += 1
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def forward(p, width: int, x):
    W1, b1, W2, b2, W3, b3 = unpack(p, width)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    y = (h2 @ W3.T + b3)[:, 0]
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(p, width: int, x, t):
    """Mean squared error and its gradient with respect to the flat parameters,
    by the chain rule written out layer by layer."""
    W1, b1, W2, b2, W3, b3 = unpack(p, width)
    y, (x, z1, h1, z2, h2) = forward(p, width, x)
    t = np.asarray(t, dtype=np.float64)
    B = len(y)
    d = y - t
    loss = float(np.mean(d * d))
    dy = 2.0 * d / B                       # (B,)
    dW3 = dy[None, :] @ h2                 # (1, W)
    db3 = np.array([dy.sum()])
    dh2 = dy[:, None] @ W3                 # (B, W)
    dz2 = dh2 * gelu_grad(z2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * gelu_grad(z1)
    dW1 = dz1.T @ x
    db1 = dz1.sum(axis=0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])
    return loss, g
