"""CPU float64 oracle of the warm-start network.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  It shares no code with
the HIP library and must never be used as a fallback for it.

The network maps the parameters of a Hamiltonian family to the coefficients
of a FEAST start block (the project's extension built on the subspace reuse
of Sec. IV.C, Example III): a multilayer perceptron d0 -> d1 -> d2 -> d3 with
ReLU after the hidden layers, trained on the mean squared error by Adam
(Kingma and Ba, "Adam: a method for stochastic optimization", ICLR 2015).

Parameters are packed as W1 [d1][d0], b1 [d1], W2 [d2][d1], b2 [d2],
W3 [d3][d2], b3 [d3] (float32 vectors in the library; float64 here).

With ``rounding=True`` every operand of a matrix product is first rounded to
bfloat16 (round to nearest even), as on the matrix cores of the GPU path:
the input x, the weights, the hidden activations, and the output gradient
and hidden-layer gradients that enter the backward products; bias
gradients are sums of the unrounded gradients.  Everything else is exact
float64.  With ``rounding=False`` the same steps run in plain float64, which
the finite-difference pins check.
"""
from __future__ import annotations

import numpy as np


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (via float32, round to nearest even) and widen to float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params: np.ndarray, dims):
    d0, d1, d2, d3 = dims
    out, off = [], 0
    for rows, cols in ((d1, d0), (d2, d1), (d3, d2)):
        W = params[off:off + rows * cols].reshape(rows, cols)
        off += rows * cols
        b = params[off:off + rows]
        off += rows
        out.append((W, b))
    assert off == len(params)
    return out


def n_params(dims) -> int:
    d0, d1, d2, d3 = dims
    return d1 * d0 + d1 + d2 * d1 + d2 + d3 * d2 + d3


def forward(params, dims, x, rounding=True):
    """Network output y [B][d3] and the cache of the backward pass."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    (W1, b1), (W2, b2), (W3, b3) = unpack(np.asarray(params, dtype=np.float64), dims)
    x0 = r(x)
    z1 = x0 @ r(W1).T + b1
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ r(W2).T + b2
    h2 = r(np.maximum(z2, 0.0))
    y = h2 @ r(W3).T + b3
    return y, (x0, z1, h1, z2, h2)


def loss_and_gradients(params, dims, x, t, rounding=True):
    """Mean squared error mean((y - t)^2) over all B x d3 entries and its
    gradient with respect to the packed parameters (back-propagation)."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    (W1, _), (W2, _), (W3, _) = unpack(np.asarray(params, dtype=np.float64), dims)
    y, (x0, z1, h1, z2, h2) = forward(params, dims, x, rounding)
    B, d3 = y.shape
    diff = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(diff * diff))
    dy = 2.0 * diff / (B * d3)
    dyr = r(dy)
    gW3 = dyr.T @ h2
    gb3 = dy.sum(axis=0)
    dz2 = (dyr @ r(W3)) * (z2 > 0)
    dz2r = r(dz2)
    gW2 = dz2r.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2r @ r(W2)) * (z1 > 0)
    dz1r = r(dz1)
    gW1 = dz1r.T @ x0
    gb1 = dz1.sum(axis=0)
    grads = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, grads


def adam_step(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update with bias correction; returns (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grads
    v = b2 * v + (1.0 - b2) * grads * grads
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
