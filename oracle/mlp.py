"""FP64 multilayer perceptron: forward, backward, MSE loss and Adam.

Layers: y = x W_l^T + b_l with W_l of shape [out][in]; ReLU after every layer
but the last.  Loss: mean over batch and outputs of (y - t)^2.  Adam with bias
correction: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
p <- p - lr * (m / (1-b1^k)) / (sqrt(v / (1-b2^k)) + eps).
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def forward(x, params: List[Tuple[np.ndarray, np.ndarray]]):
    """Return (output, activations) where activations[l] is the input of layer l."""
    acts = [np.asarray(x, dtype=np.float64)]
    h = acts[0]
    for l, (W, b) in enumerate(params):
        z = h @ W.T + b
        h = np.maximum(z, 0.0) if l < len(params) - 1 else z
        acts.append(h)
    return h, acts


def mse(y, t) -> float:
    d = np.asarray(y, dtype=np.float64) - t
    return float((d * d).mean())


def backward(acts, params, t):
    """Gradients [(dW, db)] of the MSE loss; acts from :func:`forward`."""
    y = acts[-1]
    B, K = y.shape
    g = 2.0 * (y - t) / (B * K)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        h_in = acts[l]
        grads[l] = (g.T @ h_in, g.sum(axis=0))
        if l > 0:
            g = (g @ W) * (acts[l] > 0.0)
    return grads


def adam_step(p, g, m, v, k: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** k)
    vh = v / (1 - b2 ** k)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
