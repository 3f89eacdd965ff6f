"""FP64 reference of the learned importance-sampling proposal's network
(test infrastructure only; independent of the GPU kernels).

Network: inputs x (n_in) -> 3 hidden layers of `width` units with SiLU
(silu(z) = z / (1 + exp(-z))) -> 1 linear output, optionally plus a skip
term scale * x[col] (skip = (col, scale)).  Loss: weighted mean squared
error  L = sum_i w_i (y_i - t_i)^2 / sum_i w_i.

Flat parameter layout (shared interface with the library, row-major):
  W1 [width][n_in], b1 [width], W2 [width][width], b2 [width],
  W3 [width][width], b3 [width], W4 [1][width], b4 [1].
"""
from __future__ import annotations

import numpy as np


def n_params(n_in: int, width: int) -> int:
    return width * n_in + width + 2 * (width * width + width) + width + 1


def unpack(p: np.ndarray, n_in: int, width: int):
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    shapes = [(width, n_in), (width, width), (width, width), (1, width)]
    for (r, c) in shapes:
        W = p[o:o + r * c].reshape(r, c)
        o += r * c
        b = p[o:o + r]
        o += r
        out.append((W, b))
    assert o == p.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, X, n_in, width, keep=False, skip=None):
    layers = unpack(p, n_in, width)
    H = np.asarray(X, dtype=np.float64)
    sk = 0.0 if skip is None else skip[1] * H[:, skip[0]]
    cache = [H]
    Zs = []
    for l, (W, b) in enumerate(layers):
        Z = H @ W.T + b
        if l < 3:
            Zs.append(Z)
            H = silu(Z)
            cache.append(H)
        else:
            y = Z[:, 0] + sk
    return (y, cache, Zs) if keep else y


def loss(p, X, t, w, n_in, width, skip=None):
    y = forward(p, X, n_in, width, skip=skip)
    w = np.asarray(w, dtype=np.float64)
    return float(np.sum(w * (y - t) ** 2) / np.sum(w))


def grad(p, X, t, w, n_in, width, skip=None):
    """Manual backward pass; returns (loss, flat gradient)."""
    layers = unpack(p, n_in, width)
    y, cache, Zs = forward(p, X, n_in, width, keep=True, skip=skip)
    w = np.asarray(w, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    sw = np.sum(w)
    L = float(np.sum(w * (y - t) ** 2) / sw)
    dy = 2.0 * w * (y - t) / sw                      # dL/dy
    grads = [None] * 4
    W4, _ = layers[3]
    grads[3] = (dy[None, :] @ cache[3], np.array([dy.sum()]))
    dH = dy[:, None] * W4                            # [B][width]
    for l in (2, 1, 0):
        dZ = dH * dsilu(Zs[l])
        W, _ = layers[l]
        grads[l] = (dZ.T @ cache[l], dZ.sum(axis=0))
        dH = dZ @ W
    return L, pack(grads)


def init_params(n_in: int, width: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    layers = []
    for (r, c) in [(width, n_in), (width, width), (width, width), (1, width)]:
        a = 1.0 / np.sqrt(c)
        layers.append((rng.uniform(-a, a, (r, c)), rng.uniform(-a, a, r)))
    return pack(layers)
