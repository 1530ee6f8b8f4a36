"""Three-layer MLP of the learned warm start (oracle; test infrastructure only).

y = W3^T tanh(W2^T tanh(W1^T x + b1) + b2) + b3, loss = mean((y - t)^2) over
all outputs of the batch.  Forward and backward in FP64 by the explicit chain
rule, used to check the GPU kernels' gradients.  Layout of the flat parameter
vector: W1 [in, H], b1 [H], W2 [H, H], b2 [H], W3 [H, out], b3 [out]
(row-major).

parity unpinned as a method of the paper (the warm start is not in it); the
gradient itself is pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np


def unpack(theta, n_in, H, n_out):
    shapes = [(n_in, H), (H,), (H, H), (H,), (H, n_out), (n_out,)]
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def n_params(n_in, H, n_out):
    return n_in * H + H + H * H + H + H * n_out + n_out


def forward(theta, X, n_in, H, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, np.float64), n_in, H, n_out)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    return h2 @ W3 + b3, (h1, h2)


def loss_and_grad(theta, X, T, n_in, H, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, np.float64), n_in, H, n_out)
    y, (h1, h2) = forward(theta, X, n_in, H, n_out)
    d = y - T
    loss = float(np.mean(d * d))
    dy = 2.0 * d / d.size
    gW3 = h2.T @ dy
    gb3 = dy.sum(0)
    da2 = (dy @ W3.T) * (1.0 - h2 * h2)
    gW2 = h1.T @ da2
    gb2 = da2.sum(0)
    da1 = (da2 @ W2.T) * (1.0 - h1 * h1)
    gW1 = X.T @ da1
    gb1 = da1.sum(0)
    return loss, np.concatenate([g.reshape(-1) for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def features(spec, inflow, theta, eps, dx):
    """Input row of the warm-start network for one cell: the transport part of
    the right-hand side of eq. r times dx (K values), then the density, the three
    bulk-velocity components and the temperature read from the parameters
    theta = (alpha, beta, gamma) of the cell's discrete Maxwellian
    (rho = sum_k w M_theta, U = beta / (2 gamma), T = 1 / (2 gamma)), then log10(eps)."""
    from .maxwellian import gaussian

    rho = spec.w * np.sum(gaussian(spec, theta))
    T = 0.5 / theta[-1]
    U = np.asarray(theta[1:-1]) * T
    return np.concatenate([np.asarray(inflow) * dx, [rho], U, [T], [np.log10(eps)]])
