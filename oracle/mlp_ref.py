"""FP64 reference of the surrogate network -- TEST INFRASTRUCTURE ONLY.

h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 W3 + b3 + x Ws (a linear
skip), loss = sum (y - t)^2 / (2 B n_out), and its gradient by reverse-mode
differentiation written out by hand (chain rule, layer by layer).
"""
from __future__ import annotations

import numpy as np


def n_params(n_in, H, n_out):
    return n_in * H + H + H * H + H + H * n_out + n_out + n_in * n_out


def split(flat, n_in, H, n_out):
    sizes = [n_in * H, H, H * H, H, H * n_out, n_out, n_in * n_out]
    shapes = [(n_in, H), (H,), (H, H), (H,), (H, n_out), (n_out,), (n_in, n_out)]
    out, o = [], 0
    for n, sh in zip(sizes, shapes):
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(sh))
        o += n
    return out


def forward(flat, x, n_in, H, n_out):
    W1, b1, W2, b2, W3, b3, Ws = split(flat, n_in, H, n_out)
    h1 = np.tanh(x @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    return h2 @ W3 + b3 + x @ Ws, (h1, h2)


def loss(flat, x, t, n_in, H, n_out):
    y, _ = forward(flat, x, n_in, H, n_out)
    return float(np.sum((y - t) ** 2) / (2.0 * y.size))


def loss_grad(flat, x, t, n_in, H, n_out):
    W1, b1, W2, b2, W3, b3, Ws = split(flat, n_in, H, n_out)
    y, (h1, h2) = forward(flat, x, n_in, H, n_out)
    dy = (y - t) / y.size
    gWs = x.T @ dy
    gW3 = h2.T @ dy
    gb3 = dy.sum(0)
    dz2 = (dy @ W3.T) * (1.0 - h2 ** 2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * (1.0 - h1 ** 2)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3, gWs.ravel()])
    return float(np.sum((y - t) ** 2) / (2.0 * y.size)), g
