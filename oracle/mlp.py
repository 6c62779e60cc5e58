"""FP64 multilayer perceptron: forward, backward and Adam.  TEST INFRASTRUCTURE ONLY.

Reference for the warm-start network of the GPU library: an MLP with GELU
hidden layers and a linear output layer, trained on the mean squared error
    L = (1 / (B * n_out)) * sum_{b, j} (y_bj - t_bj)^2.
GELU is the exact form x * Phi(x) with Phi the standard normal CDF, so
GELU'(x) = Phi(x) + x * phi(x).
Parameters are packed layer by layer as [W_1 (n_in x w), b_1 (w), W_2, b_2,
..., W_L (w x n_out), b_L]; W is stored row-major with the input index first,
so a layer computes y = x W + b.
Adam: m <- b1 m + (1 - b1) g; v <- b2 v + (1 - b2) g^2;
      p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def layer_sizes(n_in, width, depth, n_out):
    return [n_in] + [width] * depth + [n_out]


def n_params(sizes):
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def unpack(params, sizes):
    out = []
    o = 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = params[o:o + a * b].reshape(a, b)
        o += a * b
        bias = params[o:o + b]
        o += b
        out.append((W, bias))
    return out


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(params, sizes, X):
    """Returns the output and the list of (input, pre-activation) per layer."""
    h = np.asarray(X, dtype=np.float64)
    cache = []
    layers = unpack(np.asarray(params, dtype=np.float64), sizes)
    for k, (W, b) in enumerate(layers):
        z = h @ W + b
        cache.append((h, z))
        h = gelu(z) if k < len(layers) - 1 else z
    return h, cache


def loss_and_grad(params, sizes, X, T):
    """Mean squared error and its gradient with respect to the packed parameters."""
    Y, cache = forward(params, sizes, X)
    B, n_out = Y.shape
    diff = Y - T
    loss = float(np.sum(diff * diff) / (B * n_out))
    g = 2.0 * diff / (B * n_out)
    layers = unpack(np.asarray(params, dtype=np.float64), sizes)
    grads = []
    for k in range(len(layers) - 1, -1, -1):
        h, z = cache[k]
        if k < len(layers) - 1:
            g = g * gelu_grad(z)
        W, _ = layers[k]
        grads.append((h.T @ g, g.sum(axis=0)))
        g = g @ W.T
    flat = []
    for dW, db in reversed(grads):
        flat.append(dW.ravel())
        flat.append(db)
    return loss, np.concatenate(flat)


def adam_step(params, m, v, grad, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(sizes, rng):
    """He-style initialisation (weights N(0, 2/fan_in), zero biases), seeded."""
    flat = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        flat.append(rng.standard_normal(a * b) * math.sqrt(2.0 / a))
        flat.append(np.zeros(b))
    return np.concatenate(flat)
