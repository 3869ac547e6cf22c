"""FP64 CPU oracle of the MLP cost model (11 -> 64 -> 64 -> 1, ReLU, mean squared
error).  TEST INFRASTRUCTURE ONLY: the tests use it to check the GPU kernels'
forward values and gradients.  Parameter layout: W1 [64][11], b1 [64],
W2 [64][64], b2 [64], W3 [1][64], b3 [1], concatenated.

Pinned in tests/test_mlp_oracle.py against central finite differences of its
own forward pass (the gradient is the derivative of the loss it computes)."""
from __future__ import annotations

import numpy as np

NIN, NH = 11, 64
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (1, NH)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, o = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def forward(p, X):
    """y [n] and the activations."""
    q = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ q["W1"].T + q["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ q["W2"].T + q["b2"]
    H2 = np.maximum(Z2, 0.0)
    y = (H2 @ q["W3"].T + q["b3"])[:, 0]
    return y, (X, Z1, H1, Z2, H2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def loss_grad(p, X, t):
    """Mean squared error and its gradient by the chain rule, layer by layer."""
    q = unpack(p)
    y, (X, Z1, H1, Z2, H2) = forward(p, X)
    n = X.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / n           # [n]
    gW3 = dy[None, :] @ H2                                          # [1,64]
    gb3 = np.array([dy.sum()])
    dZ2 = (dy[:, None] @ q["W3"]) * (Z2 > 0)                        # [n,64]
    gW2 = dZ2.T @ H1
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ q["W2"]) * (Z1 > 0)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return float(np.mean((y - t) ** 2)), g


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba 2015, Algorithm 1) in FP64: exponential
    moving averages of the gradient and of its square, each divided by its
    bias factor 1 - beta^step, then p -= lr * mhat / (sqrt(vhat) + eps).
    Returns the new (p, m, v); step counts from 1."""
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
