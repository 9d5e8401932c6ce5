"""Reference for the work predictor's network (test infrastructure).

A plain float64 NumPy statement of the 4 -> 64 -> 64 -> 1 ReLU multilayer
perceptron, the gradient of the mean squared error by the chain rule, and one
Adam step (Kingma and Ba, 2015: exponential moving averages of the gradient
and its square, bias-corrected).  The tests compare the GPU kernels with it
and pin it with central finite differences.  Only the tests use this module.

Parameter vector (4545 values): W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3.
"""
import numpy as np

IN, H = 4, 64
NPARAM = H * IN + H + H * H + H + H + 1


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + H * IN].reshape(H, IN); o += H * IN
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def forward(theta, x):
    """Returns y[n] and the activations (z1, h1, z2, h2)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (z1, h1, z2, h2)


def loss(theta, x, t):
    y, _ = forward(theta, x)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(theta, x, t):
    """Gradient of mean (y - t)^2 with respect to theta (chain rule)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    y, (z1, h1, z2, h2) = forward(theta, x)
    n = x.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / n
    dw3 = h2.T @ dy
    db3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    dW1 = dz1.T @ x
    db1 = dz1.sum(axis=0)
    return pack(dW1, db1, dW2, db2, dw3, db3)


def adam(theta, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
