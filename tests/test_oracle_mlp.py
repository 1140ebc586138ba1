"""The FP64 MLP reference: backpropagation against central finite differences."""
import numpy as np
import pytest

from oracle import mlp


def test_param_count():
    assert mlp.n_params() == 8705


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(3) + 0.01 * rng.standard_normal(mlp.n_params())
    X = rng.standard_normal((17, 4))
    t = rng.uniform(0, 1, 17)
    g = mlp.grad(theta, X, t)
    idx = rng.choice(mlp.n_params(), 200, replace=False)
    # include the biases and the last layer explicitly
    idx = np.unique(np.concatenate([idx, [mlp.n_params() - 1, mlp.n_params() - 2, 300, 301, 4159, 4160]]))
    h = 1e-6
    for j in idx:
        e = np.zeros_like(theta); e[j] = h
        fd = (mlp.loss(theta + e, X, t) - mlp.loss(theta - e, X, t)) / (2 * h)
        assert fd == pytest.approx(g[j], rel=1e-6, abs=1e-9), j


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.dsilu(z), fd, rtol=1e-7, atol=1e-9)
