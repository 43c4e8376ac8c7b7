"""Float64 CPU reference of the scheduler network and its training.

TEST INFRASTRUCTURE ONLY: the test-suite uses it to check the GPU network
kernels (forward, backward, Adam, model fitting); the GPU library never imports
or calls it.  The paper has no learned component; this module is the plain
definition of the network the library's scheduler uses:

    y = W2 tanh(W1 x + b1) + b2,
    parameters packed as W1[H][F], b1[H], W2[O][H], b2[O] (row-major),

the weighted squared-error loss L = sum Wt (y - T)^2 / sum Wt, its gradient by
the chain rule, and Adam (Kingma & Ba, 2015) with beta1 0.9, beta2 0.999,
eps 1e-8.  Everything is float64 numpy.
"""
from __future__ import annotations

import numpy as np

BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def param_count(F: int, H: int, O: int) -> int:
    return H * F + H + O * H + O


def unpack(p, F, H, O):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == param_count(F, H, O)
    W1 = p[:H * F].reshape(H, F)
    b1 = p[H * F:H * F + H]
    W2 = p[H * F + H:H * F + H + O * H].reshape(O, H)
    b2 = p[H * F + H + O * H:]
    return W1, b1, W2, b2


def pack(W1, b1, W2, b2):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2)]).astype(np.float64)


def forward(p, X, F, H, O):
    """Network outputs (B x O) and hidden activations (B x H)."""
    W1, b1, W2, b2 = unpack(p, F, H, O)
    X = np.asarray(X, dtype=np.float64).reshape(-1, F)
    h = np.tanh(X @ W1.T + b1)
    return h @ W2.T + b2, h


def backward(p, X, dY, F, H, O):
    """Gradient of sum(dY * Y) with respect to the packed parameters (the
    vector-Jacobian product of the network)."""
    W1, b1, W2, b2 = unpack(p, F, H, O)
    X = np.asarray(X, dtype=np.float64).reshape(-1, F)
    G = np.asarray(dY, dtype=np.float64).reshape(-1, O)
    _, h = forward(p, X, F, H, O)
    gW2 = G.T @ h
    gb2 = G.sum(axis=0)
    dz = (G @ W2) * (1.0 - h * h)
    gW1 = dz.T @ X
    gb1 = dz.sum(axis=0)
    return pack(gW1, gb1, gW2, gb2)


def loss(p, X, T, Wt, F, H, O):
    Y, _ = forward(p, X, F, H, O)
    Wt = np.asarray(Wt, dtype=np.float64).reshape(Y.shape)
    T = np.asarray(T, dtype=np.float64).reshape(Y.shape)
    return float((Wt * (Y - T) ** 2).sum() / Wt.sum())


def loss_grad(p, X, T, Wt, F, H, O):
    Y, _ = forward(p, X, F, H, O)
    Wt = np.asarray(Wt, dtype=np.float64).reshape(Y.shape)
    T = np.asarray(T, dtype=np.float64).reshape(Y.shape)
    G = 2.0 * Wt * (Y - T) / Wt.sum()
    return backward(p, X, G, F, H, O)


def adam_train(p, m, v, X, T, Wt, F, H, O, steps, step0, lr):
    """`steps` full-batch Adam steps; returns (p, m, v)."""
    p = np.array(p, dtype=np.float64)
    m = np.array(m, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    for s in range(steps):
        t = step0 + s + 1
        g = loss_grad(p, X, T, Wt, F, H, O)
        m = BETA1 * m + (1 - BETA1) * g
        v = BETA2 * v + (1 - BETA2) * g * g
        p = p - lr * (m / (1 - BETA1 ** t)) / (np.sqrt(v / (1 - BETA2 ** t)) + EPS)
    return p, m, v


def sched_prep(X, T):
    """Normalisation and training targets of a scheduler model part: feature
    mean and 1/max(std, 1e-3); log2 of every measured time (T > 0) with row
    weight max(0.05, slowest time of the row / mean slowest time), weight 0
    where T <= 0."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    isd = 1.0 / np.maximum(sd, 1e-3)
    rowmax = np.max(np.where(T > 0, T, 0.0), axis=1)
    mean_max = rowmax[rowmax > 0].mean() if (rowmax > 0).any() else 1.0
    wr = np.maximum(0.05, rowmax / mean_max)
    ok = T > 0
    Y = np.where(ok, np.log2(np.where(ok, T, 1.0)), 0.0)
    Wt = np.where(ok, wr[:, None], 0.0)
    return mu, isd, (X - mu) * isd, Y, Wt


def model_scores(part, x):
    """Scores of raw feature rows x (B x F) under a scheduler model part
    [1205, F, H, O, mu[F], isd[F], params]."""
    part = np.asarray(part, dtype=np.float64)
    assert part[0] == 1205.0
    F, H, O = int(part[1]), int(part[2]), int(part[3])
    mu = part[4:4 + F]
    isd = part[4 + F:4 + 2 * F]
    p = part[4 + 2 * F:4 + 2 * F + param_count(F, H, O)]
    Y, _ = forward(p, (np.asarray(x, dtype=np.float64).reshape(-1, F) - mu) * isd, F, H, O)
    return Y
