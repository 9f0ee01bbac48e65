"""FP64 NumPy reference of the warm-start network -- TEST INFRASTRUCTURE ONLY.

The network (not part of the paper's method) is a plain multilayer perceptron
applied to each column's sketch: dims = [in, h, ..., h, out], ReLU after every
layer but the last.  Parameters are one flat vector, layer by layer: W_l
(dims[l+1] x dims[l], row-major) then b_l (dims[l+1]).
"""
from __future__ import annotations

import numpy as np


def layer_slices(dims):
    out, off = [], 0
    for a, b in zip(dims[:-1], dims[1:]):
        out.append((slice(off, off + a * b), slice(off + a * b, off + a * b + b), b, a))
        off += a * b + b
    return out, off


def unpack(params, dims):
    sl, total = layer_slices(dims)
    assert params.size == total
    return [(params[w].reshape(o, i), params[b]) for w, b, o, i in sl]


def forward(params, dims, x):
    """x: (batch, dims[0]).  Returns (y, acts) with acts[l] the input of layer l."""
    layers = unpack(np.asarray(params, np.float64), dims)
    a = np.asarray(x, np.float64)
    acts = [a]
    for l, (W, b) in enumerate(layers):
        z = a @ W.T + b
        a = np.maximum(z, 0.0) if l + 1 < len(layers) else z
        acts.append(a)
    return a, acts


def backward(params, dims, acts, dy):
    """Gradient of sum(dy * y) with respect to the flat parameters."""
    layers = unpack(np.asarray(params, np.float64), dims)
    sl, total = layer_slices(dims)
    grad = np.zeros(total)
    dz = np.asarray(dy, np.float64)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a_in = acts[l]
        grad[sl[l][0]] = (dz.T @ a_in).reshape(-1)
        grad[sl[l][1]] = dz.sum(axis=0)
        if l > 0:
            dz = (dz @ W) * (acts[l] > 0)
    return grad


def loss_grad(y, t, w_last):
    """Loss (1/B) sum_j [sum_{k<K-1} (y_jk - t_jk)^2 + w_last (y_j,K-1 - t_j,K-1)^2]
    and its gradient with respect to y."""
    y = np.asarray(y, np.float64)
    t = np.asarray(t, np.float64)
    wts = np.ones(y.shape[1])
    wts[-1] = w_last
    r = y - t
    B = y.shape[0]
    return float((wts * r * r).sum() / B), 2.0 * wts * r / B


def adam(params, grad, m, v, lr, b1, b2, eps, step):
    """One Adam step (Kingma & Ba 2015) with bias correction; step counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(dims, seed):
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    sl, total = layer_slices(dims)
    p = np.zeros(total)
    for w, b, o, i in sl:
        lim = np.sqrt(6.0 / i)
        p[w] = rng.uniform(-lim, lim, o * i)
    return p


def features(Y, d, c):
    """Network inputs (n x 68) from a 65 x n sketch of a d x n matrix with c groups:
    y_j / (s sqrt(d) / 8), log(||X_j|| / (s sqrt(d))), log(d)/8, log(n)/8, c/50,
    with s = ||X||_F / sqrt(d n)."""
    Y = np.asarray(Y, np.float64)
    n = Y.shape[1]
    s = np.sqrt(np.sum(Y[64] ** 2) / (d * n))
    col = s * np.sqrt(d)
    F = np.empty((n, 68))
    F[:, :64] = Y[:64].T / (0.125 * col)
    F[:, 64] = np.log(Y[64] / col + 1e-12)
    F[:, 65] = np.log(d) / 8.0
    F[:, 66] = np.log(n) / 8.0
    F[:, 67] = c / 50.0
    return F
