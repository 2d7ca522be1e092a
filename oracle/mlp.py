"""FP64 reference of the schedule-selector network -- TEST INFRASTRUCTURE ONLY.

The selector (a learned schedule chooser; the paper motivates tuning b and the
resource split in Sec. 4.2 and Sec. 6.1) is a two-layer perceptron:

    h = relu(W1 x + b1)            x: 4 features, h: 32 hidden units
    z = W2 h + b2                  z: 10 logits = 3 heads
    heads: z[0:4] -> block size b in {64,128,256,512}
           z[4:7] -> look-ahead depth in {0,1,2}
           z[7:10]-> panel CU share in {8,16,32}
    loss = mean over the batch of the sum over heads of the softmax
           cross-entropy against the integer label of that head.

Adam (Kingma & Ba, 2015) with bias correction:
    m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2
    p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)

Parameters are kept in one flat vector in the order W1 (32x4, row-major),
b1 (32), W2 (10x32, row-major), b2 (10): 490 values.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 4, 32, 10
HEADS = ((0, 4), (4, 7), (7, 10))
N_PARAM = N_HID * N_IN + N_HID + N_OUT * N_HID + N_OUT


def split(theta: np.ndarray):
    o = 0
    W1 = theta[o:o + N_HID * N_IN].reshape(N_HID, N_IN); o += N_HID * N_IN
    b1 = theta[o:o + N_HID]; o += N_HID
    W2 = theta[o:o + N_OUT * N_HID].reshape(N_OUT, N_HID); o += N_OUT * N_HID
    b2 = theta[o:o + N_OUT]; o += N_OUT
    return W1, b1, W2, b2


def forward(theta: np.ndarray, X: np.ndarray):
    W1, b1, W2, b2 = split(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    a = X @ W1.T + b1
    h = np.maximum(a, 0.0)
    z = h @ W2.T + b2
    return a, h, z


def _log_softmax(z):
    m = z.max(axis=1, keepdims=True)
    s = z - m
    return s - np.log(np.exp(s).sum(axis=1, keepdims=True))


def loss(theta: np.ndarray, X: np.ndarray, Y: np.ndarray) -> float:
    """Y: (B, 3) integer labels, one per head."""
    _, _, z = forward(theta, X)
    tot = 0.0
    for h, (lo, hi) in enumerate(HEADS):
        ls = _log_softmax(z[:, lo:hi])
        tot -= ls[np.arange(len(X)), Y[:, h]].sum()
    return tot / len(X)


def grad(theta: np.ndarray, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Gradient of ``loss`` by reverse-mode differentiation of ``forward``."""
    W1, b1, W2, b2 = split(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    B = len(X)
    a, h, z = forward(theta, X)
    dz = np.zeros_like(z)
    for hd, (lo, hi) in enumerate(HEADS):
        p = np.exp(_log_softmax(z[:, lo:hi]))
        p[np.arange(B), Y[:, hd]] -= 1.0
        dz[:, lo:hi] = p / B
    gW2 = dz.T @ h
    gb2 = dz.sum(axis=0)
    dh = dz @ W2
    da = dh * (a > 0)
    gW1 = da.T @ X
    gb1 = da.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2])


def adam(theta, g, m, v, t, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t is the 1-based step count). Returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def predict(theta: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Argmax per head: (B, 3) integer class indices."""
    _, _, z = forward(theta, X)
    return np.stack([z[:, lo:hi].argmax(axis=1) for lo, hi in HEADS], axis=1)
