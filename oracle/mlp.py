"""float64 reference of the autotuner's cost-model MLP -- TEST INFRASTRUCTURE.

F inputs -> H (ReLU) -> H (ReLU) -> 1 (linear), mean-squared-error loss and
Adam (Kingma & Ba, 2015), written directly from the definitions with numpy.
Parameter layout (one flat vector): W1[F][H], b1[H], W2[H][H], b2[H], W3[H],
b3 -- the layout the GPU kernels use.  The backward pass here is pinned by
central finite differences in tests/test_oracle_mlp.py.
"""
import numpy as np


def param_count(F, H):
    return F * H + H + H * H + H + H + 1


def unpack(p, F, H):
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + F * H].reshape(F, H); o += F * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def forward(p, X, F, H):
    """Returns (y [B], h1 [B][H], h2 [B][H])."""
    W1, b1, W2, b2, W3, b3 = unpack(p, F, H)
    X = np.asarray(X, np.float64)
    h1 = np.maximum(X @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ W3 + b3, h1, h2


def loss(p, X, T, F, H):
    y, _, _ = forward(p, X, F, H)
    return float(np.mean((y - np.asarray(T, np.float64)) ** 2))


def grad(p, X, T, F, H):
    """Gradient of the mean squared error with respect to every parameter."""
    W1, b1, W2, b2, W3, b3 = unpack(p, F, H)
    X = np.asarray(X, np.float64)
    y, h1, h2 = forward(p, X, F, H)
    B = X.shape[0]
    dy = 2.0 * (y - np.asarray(T, np.float64)) / B
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    g2 = np.outer(dy, W3) * (h2 > 0)
    gW2 = h1.T @ g2
    gb2 = g2.sum(0)
    g1 = (g2 @ W2.T) * (h1 > 0)
    gW1 = X.T @ g1
    gb1 = g1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])


def adam_step(p, g, m, v, lr, b1, b2, eps, step):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
