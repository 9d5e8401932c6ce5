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


def test_adam_constant_gradient_closed_form():
    # a constant gradient g from zero moments: m_t = (1 - b1^t) g and
    # v_t = (1 - b2^t) g^2, so the bias-corrected moments are g and g^2 at every
    # step and each step moves by lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 3.0])
    th, m, v = np.ones(4), np.zeros(4), np.zeros(4)
    for t in range(1, 11):
        th, m, v = mlp_ref.adam(th, g, m, v, t, 0.01)
        assert np.allclose(th, 1.0 - t * 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)
        assert np.allclose(m, (1 - 0.9 ** t) * g) and np.allclose(v, (1 - 0.999 ** t) * g * g)


def test_two_adam_steps_closed_form():
    # two steps with gradients g1, g2 from zero moments: the bias-corrected
    # moments after step 2 are (b1 g1 + g2) / (1 + b1) and (b2 g1^2 + g2^2) / (1 + b2)
    rng = np.random.default_rng(5)
    g1, g2 = rng.normal(0, 1, 16), rng.normal(0, 1, 16)
    b1, b2, lr, eps = 0.9, 0.999, 0.003, 1e-8
    th0 = rng.normal(0, 1, 16)
    th1, m1, v1 = mlp_ref.adam(th0, g1, np.zeros(16), np.zeros(16), 1, lr, b1, b2, eps)
    th2, _, _ = mlp_ref.adam(th1, g2, m1, v1, 2, lr, b1, b2, eps)
    mh = (b1 * g1 + g2) / (1 + b1)
    vh = (b2 * g1 * g1 + g2 * g2) / (1 + b2)
    want = th0 - lr * g1 / (np.abs(g1) + eps) - lr * mh / (np.sqrt(vh) + eps)
    assert np.allclose(th2, want, rtol=0, atol=1e-12)
