"""fp64 reference of the schedule-selector network -- TEST INFRASTRUCTURE ONLY.

Network: x (32) -> ReLU(W1 x + b1) (64) -> ReLU(W2 h1 + b2) (64) ->
W3 h2 + b3 (K).  Loss over n samples: (1 / (n K)) sum (y - t)^2.  Adam
(Kingma and Ba, 2015) with bias correction.  Parameters are one flat vector
in the order W1 (64x32 row-major), b1, W2 (64x64), b2, W3 (Kx64), b3.
Written directly from those definitions (plain matrix products and the
chain rule); it shares nothing with the GPU kernels.
"""

import numpy as np

IN, H = 32, 64


def unpack(p, K):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * IN].reshape(H, IN); o += H * IN
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + K * H].reshape(K, H); o += K * H
    b3 = p[o:o + K]; o += K
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def num_params(K):
    return H * IN + H + H * H + H + K * H + K


def forward(p, X, K):
    W1, b1, W2, b2, W3, b3 = unpack(p, K)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0)
    y = h2 @ W3.T + b3
    return y, (X, z1, h1, z2, h2)


def loss_grad(p, X, T, K):
    """Mean squared error and its gradient (flat, same layout as p)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, K)
    y, (X, z1, h1, z2, h2) = forward(p, X, K)
    T = np.asarray(T, dtype=np.float64)
    n = X.shape[0]
    d = y - T
    loss = float((d * d).sum() / (n * K))
    dy = 2.0 * d / (n * K)
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dz2 = (dy @ W3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
