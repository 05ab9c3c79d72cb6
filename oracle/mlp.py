"""Reference MLP for checking the learned parameter selector (FP64 numpy).

Part of the oracle (test infrastructure; see ``oracle/__init__.py``).

Network: x (F) -> relu(W1^T x + b1) (H) -> relu(W2^T h1 + b2) (H) -> W3^T h2 + b3 (K).
Parameters are one flat vector laid out [W1 (F x H, row-major by input),
b1 (H), W2 (H x H), b2 (H), W3 (H x K), b3 (K)].
Loss: masked mean squared error sum(mask (y - t)^2) / sum(mask).
Adam: m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
      p -= lr (m / (1 - b1^s)) / (sqrt(v / (1 - b2^s)) + eps), step s >= 1.
"""
import numpy as np


def nparams(F, H, K):
    return F * H + H + H * H + H + H * K + K


def unpack(p, F, H, K):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + F * H].reshape(F, H); o += F * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H * K].reshape(H, K); o += H * K
    b3 = p[o:o + K]; o += K
    return W1, b1, W2, b2, W3, b3


def forward(p, X, F, H, K):
    """Returns (h1, h2, y) for a batch X of shape (B, F)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, F, H, K)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h1, h2, h2 @ W3 + b3


def loss(p, X, T, mask, F, H, K):
    _, _, y = forward(p, X, F, H, K)
    mask = np.asarray(mask, dtype=np.float64)
    return float(np.sum(mask * (y - T) ** 2) / np.sum(mask))


def grad(p, X, T, mask, F, H, K):
    """Gradient of `loss` w.r.t. the flat parameters, by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unpack(p, F, H, K)
    X = np.asarray(X, dtype=np.float64)
    h1, h2, y = forward(p, X, F, H, K)
    mask = np.asarray(mask, dtype=np.float64)
    dy = 2.0 * mask * (y - T) / np.sum(mask)
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dh2 = (dy @ W3.T) * (h2 > 0)
    dW2 = h1.T @ dh2
    db2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (h1 > 0)
    dW1 = X.T @ dh1
    db1 = dh1.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
