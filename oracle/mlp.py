"""FP64 reference of the list-length network (test infrastructure only).

MLP 8 -> 64 -> 64 -> 1 with SiLU activations (silu(z) = z * sigmoid(z), Elfwing, Uchibe & Doya
2018), loss = mean((y - t)^2); the flat parameter layout is W1[8][64], b1[64], W2[64][64],
b2[64], W3[64], b3 (4801 values).  Forward and backward are written out layer by layer (chain
rule), with no framework autodiff.  The optimiser is Adam (Kingma & Ba 2015, Algorithm 1).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 8, 64
N_PARAMS = N_IN * N_H + N_H + N_H * N_H + N_H + N_H + 1


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    o = 0
    W1 = P[o:o + N_IN * N_H].reshape(N_IN, N_H); o += N_IN * N_H
    b1 = P[o:o + N_H]; o += N_H
    W2 = P[o:o + N_H * N_H].reshape(N_H, N_H); o += N_H * N_H
    b2 = P[o:o + N_H]; o += N_H
    W3 = P[o:o + N_H]; o += N_H
    b3 = P[o]
    return W1, b1, W2, b2, W3, b3


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(P, X):
    W1, b1, W2, b2, W3, b3 = unpack(P)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1 + b1
    h1 = silu(z1)
    z2 = h1 @ W2 + b2
    h2 = silu(z2)
    return h2 @ W3 + b3


def loss_and_grad(P, X, t):
    """mean((y - t)^2) and its gradient with respect to the flat parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(P)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = X.shape[0]
    z1 = X @ W1 + b1
    h1 = silu(z1)
    z2 = h1 @ W2 + b2
    h2 = silu(z2)
    y = h2 @ W3 + b3
    e = y - t
    loss = float(np.mean(e * e))
    dy = 2.0 * e / n                       # d loss / d y
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    dz2 = np.outer(dy, W3) * silu_grad(z2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * silu_grad(z1)
    gW1 = X.T @ dz1
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return loss, g


def adam(P, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) at step number t >= 1: first and second
    moment estimates, their bias corrections, and the parameter update; returns the new
    (P, m, v) in FP64."""
    P, m, v, g = (np.asarray(a, dtype=np.float64) for a in (P, m, v, g))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * (g * g)
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return P - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
