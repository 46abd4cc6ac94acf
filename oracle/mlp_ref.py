"""float64 reference of the scheduler network (TEST INFRASTRUCTURE ONLY).

The network predicts, for one bucket, the log-time of each procedure that
could finish it; the scheduler takes the cheapest feasible one.  It is not in
the paper (the paper tunes fixed thresholds by hand, Sec. 3.2-3.5); this
reference restates the textbook definitions it uses:

* a two-hidden-layer perceptron with ReLU units
      a1 = W1 x + b1,  h1 = max(a1, 0)
      a2 = W2 h1 + b2, h2 = max(a2, 0)
      y  = W3 h2 + b3
* masked mean squared error over a batch (only observed procedure times
  count):  L = sum(M * (y - t)**2) / sum(M), and L = 0 when sum(M) = 0
* gradients by the chain rule (back-propagation), with the ReLU derivative
  taken as 1 where a > 0 and 0 elsewhere (including a == 0)
* Adam (Kingma and Ba, ICLR 2015, Algorithm 1) with bias-corrected moments.

Parameters live in one flat vector in the order W1 (H x F, row-major), b1,
W2 (H x H), b2, W3 (P x H), b3 -- the layout the GPU kernels use.
"""
from __future__ import annotations

import numpy as np


def n_params(F: int, H: int, P: int) -> int:
    return H * F + H + H * H + H + P * H + P


def unpack(theta: np.ndarray, F: int, H: int, P: int):
    theta = np.asarray(theta, dtype=np.float64)
    if theta.shape != (n_params(F, H, P),):
        raise ValueError("parameter vector has the wrong length")
    o = 0
    W1 = theta[o:o + H * F].reshape(H, F); o += H * F
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    W3 = theta[o:o + P * H].reshape(P, H); o += P * H
    b3 = theta[o:o + P]; o += P
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, np.ravel(W3), b3]).astype(np.float64)


def forward(theta, X, F: int, H: int, P: int, keep: bool = False):
    """Y = network(X) for a batch X of shape (B, F); returns (B, P)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, F, H, P)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ W3.T + b3
    if keep:
        return y, (X, a1, h1, a2, h2)
    return y


def loss(theta, X, T, M, F: int, H: int, P: int) -> float:
    y = forward(theta, X, F, H, P)
    M = np.asarray(M, dtype=np.float64)
    s = M.sum()
    if s == 0:
        return 0.0
    d = np.where(M > 0, y - np.asarray(T, dtype=np.float64), 0.0)
    return float((M * d * d).sum() / s)


def loss_and_grad(theta, X, T, M, F: int, H: int, P: int, relu_gate=None):
    """(L, dL/dtheta) by back-propagation.

    ``relu_gate`` optionally fixes which hidden units count as active: a pair
    of boolean arrays (a1 > 0, a2 > 0).  A kernel that evaluates the network
    in float32 decides each gate in float32; comparing it against this
    float64 reference is only meaningful with the same decisions, so a test
    passes the float32 gates (``relu_gates_f32``) here.
    """
    W1, b1, W2, b2, W3, b3 = unpack(theta, F, H, P)
    y, (X, a1, h1, a2, h2) = forward(theta, X, F, H, P, keep=True)
    if relu_gate is not None:
        g1, g2 = relu_gate
        h1 = np.where(g1, a1, 0.0)
        a2 = h1 @ W2.T + b2
        h2 = np.where(g2, a2, 0.0)
        y = h2 @ W3.T + b3
        a1 = np.where(g1, 1.0, -1.0)
        a2 = np.where(g2, 1.0, -1.0)
    M = np.asarray(M, dtype=np.float64)
    s = M.sum()
    if s == 0:
        return 0.0, np.zeros(n_params(F, H, P))
    d = np.where(M > 0, y - np.asarray(T, dtype=np.float64), 0.0)
    L = float((M * d * d).sum() / s)
    dy = 2.0 * M * d / s                      # (B, P)
    dW3 = dy.T @ h2
    db3 = dy.sum(axis=0)
    dh2 = dy @ W3
    da2 = dh2 * (a2 > 0)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (a1 > 0)
    dW1 = da1.T @ X
    db1 = da1.sum(axis=0)
    return L, pack(dW1, db1, dW2, db2, dW3, db3)


def adam_step(theta, g, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update at step t (t >= 1); returns new (theta, m, v)."""
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = np.asarray(theta, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def relu_gates_f32(theta, X, F: int, H: int, P: int):
    """The (a1 > 0, a2 > 0) decisions of the network evaluated in float32."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(a, dtype=np.float32) for a in unpack(theta, F, H, P))
    X = np.asarray(X, dtype=np.float32)
    a1 = X @ W1.T + b1
    a2 = np.maximum(a1, np.float32(0)) @ W2.T + b2
    return a1 > 0, a2 > 0


def forward_f32(theta, X, F: int, H: int, P: int):
    """The same network evaluated in float32 (for decisions taken in float32)."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(a, dtype=np.float32) for a in unpack(theta, F, H, P))
    X = np.asarray(X, dtype=np.float32)
    h1 = np.maximum(X @ W1.T + b1, np.float32(0))
    h2 = np.maximum(h1 @ W2.T + b2, np.float32(0))
    return h2 @ W3.T + b3
