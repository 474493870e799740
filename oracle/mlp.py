"""FP64 oracle of the candidate-count regressor that steers scheduling.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper trains an offline model that maps data characteristics to a cache
split (Section 5.2, "Cost Models of qwLSH", and its workflow in Section 5.3).
The GPU path keeps that idea -- a learned model steers resources, never results
-- with a different target: a two-layer perceptron

    z = W1 f + b1,  a = relu(z),  y = W2 a + b2

over the features f_l = log(1 + s_l) (s_l = size of the query's bucket in layer
l, l < L), regressed onto t = log(1 + |C(q)|) with the mean squared error

    loss = (1/B) * sum_i (y_i - t_i)^2

over a minibatch of B queries.  This module computes the loss and its exact
gradient by hand-written backpropagation in float64, and one Adam step
(Kingma & Ba 2015, bias-corrected moments).
"""
from __future__ import annotations

import numpy as np


def features(sizes: np.ndarray) -> np.ndarray:
    """f = log(1 + s) per (query, layer)."""
    return np.log1p(np.asarray(sizes, dtype=np.float64))


def forward(W1, b1, W2, b2, f):
    """Returns (y [B], cache).  W1 [H,L], b1 [H], W2 [H], b2 scalar, f [B,L]."""
    W1 = np.asarray(W1, np.float64); b1 = np.asarray(b1, np.float64)
    W2 = np.asarray(W2, np.float64); b2 = float(np.asarray(b2, np.float64).reshape(()))
    f = np.asarray(f, np.float64)
    z = f @ W1.T + b1          # [B,H]
    a = np.maximum(z, 0.0)
    y = a @ W2 + b2            # [B]
    return y, (f, z, a)


def loss_and_grad(W1, b1, W2, b2, f, t):
    """MSE loss and its gradient (dW1 [H,L], db1 [H], dW2 [H], db2 scalar)."""
    y, (f, z, a) = forward(W1, b1, W2, b2, f)
    t = np.asarray(t, np.float64)
    B = f.shape[0]
    r = y - t
    loss = float(np.sum(r * r) / B)
    dy = 2.0 * r / B           # d loss / d y
    dW2 = a.T @ dy
    db2 = float(np.sum(dy))
    da = np.outer(dy, np.asarray(W2, np.float64))
    dz = da * (z > 0.0)
    dW1 = dz.T @ f
    db1 = dz.sum(axis=0)
    return loss, (dW1, db1, dW2, db2)


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of parameter p with gradient g; step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
