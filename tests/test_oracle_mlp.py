"""Pins for the learned predictor's FP64 reference: gradients against central
finite differences of the loss, the closed-form softmax cross-entropy
gradient, probabilities summing to one, and loss decrease under descent."""
import numpy as np
import pytest

from oracle import mlp


def setup(seed=0, B=7, n_in=4, H=16, C=9):
    rng = np.random.default_rng(seed)
    params = mlp.init_params(rng, n_in, H, C)
    # small non-zero biases so every ReLU region is exercised
    for k in ("b1", "b2", "b3"):
        params[k] = rng.normal(0, 0.1, params[k].shape)
    x = rng.normal(size=(B, n_in))
    y = rng.dirichlet(np.ones(C), size=B)
    return params, x, y


def test_probabilities_are_a_distribution():
    params, x, _ = setup()
    p, _ = mlp.forward(params, x)
    np.testing.assert_allclose(p.sum(axis=1), 1.0, atol=1e-14)
    assert np.all(p > 0)


@pytest.mark.parametrize("name", ["W1", "b1", "W2", "b2", "W3", "b3"])
def test_gradients_match_finite_differences(name):
    params, x, y = setup(seed=3)
    g = mlp.backward(params, x, y)[name]
    eps = 1e-6
    num = np.zeros_like(params[name])
    it = np.nditer(params[name], flags=["multi_index"])
    for _ in it:
        idx = it.multi_index
        pp = {k: v.copy() for k, v in params.items()}
        pm = {k: v.copy() for k, v in params.items()}
        pp[name][idx] += eps
        pm[name][idx] -= eps
        num[idx] = (mlp.loss(pp, x, y) - mlp.loss(pm, x, y)) / (2 * eps)
    np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-8)


def test_output_gradient_closed_form():
    # d L / d b3 = mean over the batch of (p - y) for softmax cross-entropy
    params, x, y = setup(seed=4)
    p, _ = mlp.forward(params, x)
    np.testing.assert_allclose(mlp.backward(params, x, y)["b3"], (p - y).mean(axis=0), atol=1e-15)


def test_descent_reduces_loss():
    params, x, y = setup(seed=5)
    l0 = mlp.loss(params, x, y)
    for _ in range(50):
        params = mlp.sgd_step(params, mlp.backward(params, x, y), 0.1)
    assert mlp.loss(params, x, y) < l0
