"""Pins of the cost-model MLP oracle: the analytic gradient equals central
finite differences of the loss (float64), and Adam's first step moves every
parameter by lr * sign(g) (a closed form of the definition at step 1)."""
import numpy as np

from oracle import mlp


def test_gradient_matches_finite_differences():
    F, H, B = 5, 7, 11
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.5, mlp.param_count(F, H))
    X = rng.normal(0, 1, (B, F))
    T = rng.normal(0, 1, B)
    g = mlp.grad(p, X, T, F, H)
    eps = 1e-6
    for i in range(len(p)):
        e = np.zeros_like(p)
        e[i] = eps
        fd = (mlp.loss(p + e, X, T, F, H) - mlp.loss(p - e, X, T, F, H)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(1)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p2, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1e-3, 0.9, 0.999, 0.0, 1)
    assert np.allclose(p - p2, 1e-3 * np.sign(g))


def test_relu_layers_are_piecewise_linear():
    """Scaling a positive input set by c > 0 with zero biases scales y by c."""
    F, H = 3, 4
    rng = np.random.default_rng(2)
    p = rng.normal(size=mlp.param_count(F, H))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, F, H)
    p0 = np.concatenate([W1.ravel(), 0 * b1, W2.ravel(), 0 * b2, W3, [0.0]])
    X = rng.normal(size=(6, F))
    y1, _, _ = mlp.forward(p0, X, F, H)
    y3, _, _ = mlp.forward(p0, 3 * X, F, H)
    assert np.allclose(3 * y1, y3)


def test_forward_value_of_a_hand_computed_network():
    """F = 2, H = 2, worked by hand (W1[f][h] input f to unit h):
    W1 = [[1, -1], [2, 1]], b1 = [0.5, -1], W2 = [[1, -2], [-1, 1]],
    b2 = [0, 0.5], W3 = [3, -2], b3 = 0.25.
    x = (2, 1):  z1 = (4.5, -2) -> h1 = (4.5, 0); z2 = (4.5, -8.5) -> h2 = (4.5, 0);
                 y = 13.5 + 0.25 = 13.75  (without the first ReLU 19.75,
                 without the second 30.75, with W1 transposed -2.75).
    x = (-1, 1): z1 = (1.5, 1) -> h1 = (1.5, 1); z2 = (0.5, -1.5) -> h2 = (0.5, 0);
                 y = 1.5 + 0.25 = 1.75."""
    p = np.array([1, -1, 2, 1, 0.5, -1, 1, -2, -1, 1, 0, 0.5, 3, -2, 0.25], np.float64)
    assert mlp.param_count(2, 2) == p.size
    y, h1, h2 = mlp.forward(p, np.array([[2.0, 1.0], [-1.0, 1.0]]), 2, 2)
    assert np.array_equal(y, [13.75, 1.75])
    assert np.array_equal(h1, [[4.5, 0.0], [1.5, 1.0]])
    assert np.array_equal(h2, [[4.5, 0.0], [0.5, 0.0]])
