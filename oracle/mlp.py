"""FP64 reference of the warm-start network of the learned IBM form.

TEST INFRASTRUCTURE ONLY (tests and the benchmark's CPU leg); the product
path never imports it.

A plain multilayer perceptron 16 -> 64 -> 64 -> 3 with SiLU activations
(x * sigmoid(x)) on the two hidden layers and a linear output, its mean
squared error loss L = 1/(2N) sum_n |y_n - t_n|^2, the gradient of L by
backpropagation, and the Adam update (Kingma & Ba, 2015, Algorithm 1).

Flat parameter layout (the same order the library uses):
    W1 (64 x 16, row-major: W[out][in]), b1 (64),
    W2 (64 x 64), b2 (64),
    W3 (3 x 64), b3 (3)
"""
from __future__ import annotations

import numpy as np

LAYERS = [(16, 64), (64, 64), (64, 3)]
N_PARAMS = sum(i * o + o for i, o in LAYERS)


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, k = [], 0
    for i, o in LAYERS:
        W = theta[k:k + o * i].reshape(o, i)
        k += o * i
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    return out


def pack(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def silu(x):
    return x * sigmoid(x)


def dsilu(x):
    s = sigmoid(x)
    return s + x * s * (1.0 - s)


def forward(theta, X):
    """X (N, 16) -> Y (N, 3) and the cache of pre-activations/activations."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(theta)
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    a1 = silu(z1)
    z2 = a1 @ W2.T + b2
    a2 = silu(z2)
    Y = a2 @ W3.T + b3
    return Y, (X, z1, a1, z2, a2)


def forward_half_operands(theta, X):
    """The forward pass with the operands of every layer -- the input and the
    two hidden activations -- rounded to IEEE binary16 (to nearest, ties to
    even), everything else in FP64: the arithmetic of an inference with FP16
    weights and operands on matrix units that accumulate in a wider format,
    up to that accumulation's own rounding."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(theta)

    def h(a):
        return np.asarray(a, np.float64).astype(np.float16).astype(np.float64)

    x = h(X)
    a1 = h(silu(x @ W1.T + b1))
    a2 = h(silu(a1 @ W2.T + b2))
    return a2 @ W3.T + b3


def loss(theta, X, T):
    Y, _ = forward(theta, X)
    return 0.5 * float(np.sum((Y - T) ** 2)) / X.shape[0]


def grad(theta, X, T):
    """dL/dtheta by backpropagation, flat in the parameter layout."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(theta)
    Y, (X, z1, a1, z2, a2) = forward(theta, X)
    n = X.shape[0]
    dY = (Y - T) / n
    gW3 = dY.T @ a2
    gb3 = dY.sum(0)
    dz2 = (dY @ W3) * dsilu(z2)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * dsilu(z1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    return pack([(gW1, gb1), (gW2, gb2), (gW3, gb3)])


def adam(theta, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new theta, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for i, o in LAYERS:
        bound = np.sqrt(6.0 / i)
        params.append((rng.uniform(-bound, bound, size=(o, i)), np.zeros(o)))
    return pack(params)
