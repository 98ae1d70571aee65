"""FP64 reference of the plan selector's network -- TEST INFRASTRUCTURE.

Only the tests call this; the library's HIP kernels are checked against it.

Network (two hidden ReLU layers), parameters as one vector
W1[H][D], b1[H], W2[H][H], b2[H], w3[H], b3:
    a1 = relu(W1 x + b1),  a2 = relu(W2 a1 + b2),  y = w3 . a2 + b3
Loss over a minibatch: mean_b (y_b - t_b)^2.
The backward pass below is derived by hand from these formulas (chain rule);
finite differences and an autograd run pin it.
Adam: Kingma & Ba, "Adam: A Method for Stochastic Optimization" (2015),
Algorithm 1, with bias-corrected moments.
"""
from __future__ import annotations

import numpy as np


def nparams(D: int, H: int) -> int:
    return H * D + H + H * H + H + H + 1


def unpack(p, D, H):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * D].reshape(H, D); o += H * D
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(p, X, D, H):
    """y for each row of X, plus the pre-activations and activations."""
    W1, b1, W2, b2, w3, b3 = unpack(p, D, H)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    y = a2 @ w3 + b3
    return y, (z1, a1, z2, a2)


def loss(p, X, T, D, H) -> float:
    y, _ = forward(p, X, D, H)
    return float(np.mean((y - np.asarray(T, dtype=np.float64)) ** 2))


def gradient(p, X, T, D, H):
    """(grad vector, loss) of the mean squared error."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    B = X.shape[0]
    W1, b1, W2, b2, w3, b3 = unpack(p, D, H)
    y, (z1, a1, z2, a2) = forward(p, X, D, H)
    dy = 2.0 * (y - T) / B                       # dL/dy_b
    g_w3 = a2.T @ dy                             # dL/dw3
    g_b3 = np.sum(dy)
    d2 = np.outer(dy, w3) * (z2 > 0)             # dL/dz2
    g_W2 = d2.T @ a1
    g_b2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (z1 > 0)                    # dL/dz1
    g_W1 = d1.T @ X
    g_b1 = d1.sum(axis=0)
    g = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])
    return g, float(np.mean((y - T) ** 2))


def finite_difference(p, X, T, D, H, h=1e-6, which=None):
    """Central differences of the loss for parameter indices `which`."""
    p = np.asarray(p, dtype=np.float64).copy()
    which = range(p.size) if which is None else which
    out = []
    for q in which:
        old = p[q]
        p[q] = old + h
        lp = loss(p, X, T, D, H)
        p[q] = old - h
        lm = loss(p, X, T, D, H)
        p[q] = old
        out.append((lp - lm) / (2 * h))
    return np.array(out)


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t >= 1); returns new (p, m, v)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
