"""Pins of the FP64 reference network: SiLU and its derivative against
calculus, the backpropagated gradient against central finite differences,
and Adam against its first-step closed form and a quadratic it must
minimize."""
import numpy as np
import pytest

from oracle import mlp


def test_silu_and_derivative():
    x = np.linspace(-8, 8, 161)
    assert np.allclose(mlp.silu(x), x / (1 + np.exp(-x)))
    h = 1e-6
    fd = (mlp.silu(x + h) - mlp.silu(x - h)) / (2 * h)
    assert np.allclose(mlp.dsilu(x), fd, atol=1e-9)
    assert mlp.silu(0.0) == 0.0 and abs(mlp.dsilu(0.0) - 0.5) < 1e-15


NIN = mlp.LAYERS[0][0]


def test_layout_round_trip():
    theta = np.arange(mlp.N_PARAMS, dtype=float)
    assert mlp.N_PARAMS == NIN * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3
    assert np.array_equal(mlp.pack(mlp.unpack(theta)), theta)
    (W1, _), _, (W3, b3) = mlp.unpack(theta)
    assert W1[1, 0] == NIN and b3[-1] == mlp.N_PARAMS - 1


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    theta = mlp.init_params(seed) + 0.01 * rng.standard_normal(mlp.N_PARAMS)
    X = rng.standard_normal((7, NIN))
    T = rng.standard_normal((7, 3))
    g = mlp.grad(theta, X, T)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    # the first and last entries of every weight and bias block
    edges, k = [], 0
    for i, o in mlp.LAYERS:
        edges += [k, k + o * i - 1, k + o * i, k + o * i + o - 1]
        k += o * i + o
    idx = np.concatenate([idx, edges])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = h
        fd = (mlp.loss(theta + e, X, T) - mlp.loss(theta - e, X, T)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, k


def test_adam_first_step_and_convergence():
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = mlp.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    # bias-corrected first step is -lr * g / (|g| + eps)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8))
    # minimizes a quadratic
    A = np.diag([1.0, 10.0, 0.1])
    x, m, v = np.array([1.0, -1.0, 2.0]), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        x, m, v = mlp.adam(x, m, v, A @ x, t, lr=0.02)
    assert np.linalg.norm(x) < 1e-2


def test_half_operand_forward():
    """The inference form rounds each layer's operands to binary16: inputs
    given already rounded change nothing; the result differs from the FP64
    forward by the rounding only (a few 1e-4 of the output scale); and with
    the output layer picking three hidden units of the last layer unchanged,
    the outputs are binary16 values."""
    rng = np.random.default_rng(2)
    theta = mlp.init_params(3) + 0.05 * rng.standard_normal(mlp.N_PARAMS)
    X = rng.standard_normal((500, NIN))
    Yh = mlp.forward_half_operands(theta, X)
    Y, _ = mlp.forward(theta, X)
    X16 = X.astype(np.float16).astype(np.float64)
    assert np.array_equal(mlp.forward_half_operands(theta, X16), Yh)
    d = np.abs(Yh - Y).max() / np.abs(Y).max()
    assert 1e-5 < d < 2e-3
    (W1, b1), (W2, b2), (W3, b3) = mlp.unpack(theta)
    W3 = np.zeros_like(W3)
    W3[np.arange(3), [5, 17, 40]] = 1.0
    pick = mlp.pack([(W1, b1), (W2, b2), (W3, np.zeros(3))])
    y = mlp.forward_half_operands(pick, X)
    assert np.array_equal(y, y.astype(np.float16).astype(np.float64))
    # and they are the FP64 hidden units to within binary16 rounding
    _, (_, _, _, _, a2) = mlp.forward(pick, X)
    assert np.max(np.abs(y - a2[:, [5, 17, 40]])) < 4e-3 * np.abs(a2).max()
