"""Oracle of the warm-start network in plain numpy FP64.  TEST INFRASTRUCTURE ONLY.

The network is a two-layer perceptron, y = tanh(x W1 + b1) W2 + b2, with its
parameters packed in one vector as W1 (n_in x n_hidden, row-major), b1, W2
(n_hidden x n_out), b2.  The training loss is the mean over rows and outputs
of the squared error.  The gradient follows the chain rule layer by layer
(backpropagation); Adam follows Kingma and Ba (2015), Algorithm 1, with the
bias-corrected moment estimates.  The paper names learned components only as
future work (Discussion); the network, its loss and its optimiser are
textbook definitions.
"""
from __future__ import annotations

import numpy as np


def n_params(ni, nh, no):
    return ni * nh + nh + nh * no + no


def unpack(p, ni, nh, no):
    p = np.asarray(p, dtype=np.float64)
    if p.size != n_params(ni, nh, no):
        raise ValueError("parameter vector has the wrong size")
    i = 0
    W1 = p[i:i + ni * nh].reshape(ni, nh); i += ni * nh
    b1 = p[i:i + nh]; i += nh
    W2 = p[i:i + nh * no].reshape(nh, no); i += nh * no
    b2 = p[i:i + no]
    return W1, b1, W2, b2


def forward(x, p, ni, nh, no):
    """Returns (hidden activations, outputs)."""
    W1, b1, W2, b2 = unpack(p, ni, nh, no)
    x = np.asarray(x, dtype=np.float64)
    h = np.tanh(x @ W1 + b1)
    return h, h @ W2 + b2


def loss(x, t, p, ni, nh, no):
    """Mean squared error over rows and outputs."""
    _, y = forward(x, p, ni, nh, no)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def gradient(x, t, p, ni, nh, no):
    """d loss / d p, packed like p."""
    W1, b1, W2, b2 = unpack(p, ni, nh, no)
    x = np.asarray(x, dtype=np.float64)
    h, y = forward(x, p, ni, nh, no)
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / y.size
    gW2 = h.T @ dy
    gb2 = dy.sum(axis=0)
    dz = (dy @ W2.T) * (1.0 - h * h)
    gW1 = x.T @ dz
    gb1 = dz.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2])


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at 1-based step number `step`; returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
