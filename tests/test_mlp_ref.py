"""Pins of the predictor network's CPU reference (oracle/mlp_ref.py): its
gradient against central finite differences of its own loss, a hand-computed
forward pass, and the first Adam step in closed form."""
import numpy as np

from oracle import mlp_ref


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    theta = rng.normal(0, 0.3, mlp_ref.NPARAM)
    x = rng.normal(0, 1, (17, 4))
    t = rng.normal(0, 1, 17)
    g = mlp_ref.grad(theta, x, t)
    idx = np.concatenate([rng.choice(mlp_ref.NPARAM, 200, replace=False), [mlp_ref.NPARAM - 1, 0, 256, 320]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (mlp_ref.loss(theta + e, x, t) - mlp_ref.loss(theta - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_by_hand():
    # W1 = [I_4; 0], b1 = 0; W2 = I; w3 = 1, b3 = 0.5: y = 0.5 + sum of the positive inputs
    W1 = np.zeros((64, 4))
    W1[:4, :4] = np.eye(4)
    theta = mlp_ref.pack(W1, np.zeros(64), np.eye(64), np.zeros(64), np.ones(64), 0.5)
    x = np.array([[1.0, -2.0, 3.0, -4.0], [0.0, 0.0, 0.0, 0.0], [-1.0, 2.5, 0.0, 0.25]])
    y, _ = mlp_ref.forward(theta, x)
    assert np.allclose(y, [4.5, 0.5, 3.25])


def test_first_adam_step_closed_form():
    # after one step from zero moments: theta - lr * g / (|g| + eps) (bias corrections cancel)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = mlp_ref.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
