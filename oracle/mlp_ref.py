"""Float64 reference of the cost-model MLP -- TEST INFRASTRUCTURE ONLY.

Network: 7 -> 64 -> 64 -> 64 -> 2, ReLU on the hidden layers, linear head.
Parameters are one flat array W1 [64][7], b1, W2 [64][64], b2, W3 [64][64],
b3, W4 [2][64], b4.  Adam follows Kingma and Ba (ICLR 2015, Algorithm 1) with
bias correction.
"""
from __future__ import annotations

import numpy as np

SIZES = [(64, 7), (64, 64), (64, 64), (2, 64)]
NPARAM = sum(o * i + o for o, i in SIZES)


def unpack(W):
    W = np.asarray(W, dtype=np.float64)
    out, p = [], 0
    for o, i in SIZES:
        w = W[p:p + o * i].reshape(o, i)
        p += o * i
        b = W[p:p + o]
        p += o
        out.append((w, b))
    return out


def forward(W, X):
    """Y [B][2] and the post-ReLU activations of the three hidden layers."""
    layers = unpack(W)
    h = np.asarray(X, dtype=np.float64)
    acts = []
    for li, (w, b) in enumerate(layers):
        z = h @ w.T + b
        if li < 3:
            h = np.maximum(z, 0.0)
            acts.append(h)
        else:
            h = z
    return h, acts


def backward(W, X, acts, dY):
    """Gradient of sum_b <dY_b, Y_b> with respect to the flat parameters (summed over the batch)."""
    layers = unpack(W)
    X = np.asarray(X, dtype=np.float64)
    ins = [X] + acts
    grads = [None] * 4
    delta = np.asarray(dY, dtype=np.float64)
    for li in range(3, -1, -1):
        w, _ = layers[li]
        grads[li] = (delta.T @ ins[li], delta.sum(axis=0))
        if li > 0:
            delta = (delta @ w) * (acts[li - 1] > 0)
    return np.concatenate([np.concatenate([g.ravel(), b]) for g, b in grads])


def adam(W, dW, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * dW
    v = b2 * v + (1 - b2) * dW * dW
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return W - lr * mh / (np.sqrt(vh) + eps), m, v


def mse(W, X, T):
    Y, _ = forward(W, X)
    return float(np.mean((Y - T) ** 2))


def init(seed):
    """He-style initialisation (float32-representable)."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in SIZES:
        parts.append((rng.standard_normal(o * i) * np.sqrt(2.0 / i)).astype(np.float32))
        parts.append(np.zeros(o, dtype=np.float32))
    return np.concatenate(parts)
