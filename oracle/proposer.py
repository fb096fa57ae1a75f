"""FP64 reference of the constraint-proposal scorer of the learned form.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (gradient checks of the GPU
training kernels).  The product library never imports it.

The scorer is a ReLU MLP  d -> H -> H -> 1  that gives one logit per
constraint line of a cell:

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  z = w3 . h2 + b3.

Training minimises the mean binary cross-entropy between sigmoid(z) and the
label y (1 when the line carries an edge of the cell's face):

    loss = mean( max(z, 0) - z y + log(1 + exp(-|z|)) ),

whose derivative in z is (sigmoid(z) - y) / n.  The gradients below follow
from the chain rule through the two ReLU layers (a unit with pre-activation
exactly 0 passes no gradient).  Everything is FP64; callers that model FP16
storage round their inputs before the call.  This is not part of the paper
(the learned form replaces the distance order of its pivoting routine,
Sec. 4.2.1, by a trained ranking); the arithmetic is plain definitions.

Flat parameter layout (the same order the library uses):
    W1 [H][d], b1 [H], W2 [H][H], b2 [H], w3 [H], b3 [1].
"""
from __future__ import annotations

import numpy as np


def n_params(d: int, H: int) -> int:
    return H * d + H + H * H + H + H + 1


def unpack(p: np.ndarray, d: int, H: int):
    p = np.asarray(p, np.float64)
    assert p.shape == (n_params(d, H),)
    o = 0
    W1 = p[o:o + H * d].reshape(H, d); o += H * d
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def logits(p, X, d: int, H: int) -> np.ndarray:
    """z for each row of X [n][d]."""
    W1, b1, W2, b2, w3, b3 = unpack(p, d, H)
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ w3 + b3


def loss_and_grad(p, X, y, d: int, H: int, _mutate: int = 0):
    """Mean BCE-with-logits loss and its gradient (flat, same layout as p).

    ``_mutate`` plants a mistake for the tests that check the checks
    (1: ReLU mask dropped in the backward pass, 2: sign of dz flipped,
    3: W2 used untransposed in the backward pass).
    """
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    n = X.shape[0]
    W1, b1, W2, b2, w3, b3 = unpack(p, d, H)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    loss = np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z))))
    sig = 0.5 * (1.0 + np.tanh(0.5 * z))          # sigmoid without overflow
    dz = (sig - y) / n
    if _mutate == 2:
        dz = -dz
    gw3 = h2.T @ dz
    gb3 = dz.sum()
    dh2 = np.outer(dz, w3)
    da2 = dh2 if _mutate == 1 else dh2 * (a2 > 0.0)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ (W2.T if _mutate == 3 else W2)
    da1 = dh1 * (a1 > 0.0)
    gW1 = da1.T @ X
    gb1 = da1.sum(axis=0)
    return float(loss), pack(gW1, gb1, gW2, gb2, gw3, gb3)


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (bias-corrected moments), returning new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
