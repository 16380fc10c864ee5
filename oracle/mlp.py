"""FP64 reference of the learned-start network (test infrastructure only).

The network maps a descriptor x (n_in) to coefficients y (n_out):
    z1 = x W1 + b1, a1 = silu(z1), z2 = a1 W2 + b2, a2 = silu(z2), y = a2 W3 + b3
with silu(z) = z / (1 + exp(-z)); the loss is the mean of (y - t)^2 over all
rows and outputs; Adam uses beta1 = 0.9, beta2 = 0.999, eps = 1e-8 with bias
correction.  Parameters are packed as W1, b1, W2, b2, W3, b3 (row-major,
input index first), the order of the library's interface.
"""

from __future__ import annotations

import numpy as np


def unpack(params, n_in, n_hidden, n_out):
    p = np.asarray(params, np.float64)
    sizes = [n_in * n_hidden, n_hidden, n_hidden * n_hidden, n_hidden, n_hidden * n_out, n_out]
    if p.size != sum(sizes):
        raise ValueError("parameter count")
    out, o = [], 0
    for s in sizes:
        out.append(p[o:o + s])
        o += s
    W1, b1, W2, b2, W3, b3 = out
    return (W1.reshape(n_in, n_hidden), b1, W2.reshape(n_hidden, n_hidden), b2,
            W3.reshape(n_hidden, n_out), b3)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, shape):
    W1, b1, W2, b2, W3, b3 = unpack(params, *shape)
    x = np.asarray(x, np.float64)
    z1 = x @ W1 + b1
    a1 = silu(z1)
    z2 = a1 @ W2 + b2
    a2 = silu(z2)
    return a2 @ W3 + b3, (x, z1, a1, z2, a2)


def loss_grad(params, x, t, shape):
    """Mean squared error and its gradient (packed like the parameters)."""
    W1, b1, W2, b2, W3, b3 = unpack(params, *shape)
    y, (x, z1, a1, z2, a2) = forward(params, x, shape)
    t = np.asarray(t, np.float64)
    d = y - t
    loss = float(np.mean(d * d))
    dy = 2.0 * d / d.size
    gW3 = a2.T @ dy
    gb3 = dy.sum(0)
    dz2 = (dy @ W3.T) * silu_grad(z2)
    gW2 = a1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * silu_grad(z1)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(params, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
