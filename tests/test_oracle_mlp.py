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


def test_layout_round_trip():
    theta = np.arange(mlp.N_PARAMS, dtype=float)
    assert mlp.N_PARAMS == 12 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3
    assert np.array_equal(mlp.pack(mlp.unpack(theta)), theta)
    (W1, _), _, (W3, b3) = mlp.unpack(theta)
    assert W1[1, 0] == 12 and b3[-1] == mlp.N_PARAMS - 1


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    theta = mlp.init_params(seed) + 0.01 * rng.standard_normal(mlp.N_PARAMS)
    X = rng.standard_normal((7, 12))
    T = rng.standard_normal((7, 3))
    g = mlp.grad(theta, X, T)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [0, 767, 768, 831, 832, 4927, 4928, 5183, 5184, 5186]])
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
