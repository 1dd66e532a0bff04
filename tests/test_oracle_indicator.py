"""Pins of the FP64 indicator reference: gradients against central finite
differences of the loss (which uses only the forward pass), the tanh GELU
against the exact erf GELU, feature normalisation properties and labels
from the oracle's WENO5 weights."""
import math

import numpy as np
import pytest

import oracle
from oracle import indicator as ind

RNG = np.random.default_rng(77)


def test_gradients_match_finite_differences():
    params = ind.init_params(3)
    X = RNG.uniform(-1, 1, size=(37, ind.NIN))
    y = (RNG.uniform(size=37) < 0.4).astype(np.float64)
    _, g = ind.loss_and_grads(params, X, y)
    h = 1e-6
    for k, W in params.items():
        flat = W.reshape(-1)
        for idx in RNG.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = ind.loss_and_grads(params, X, y)
            flat[idx] = old - h
            lm, _ = ind.loss_and_grads(params, X, y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert an == pytest.approx(fd, rel=1e-6, abs=1e-9), (k, idx)


def test_tanh_gelu_close_to_exact_gelu():
    x = np.linspace(-6, 6, 1001)
    exact = 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))
    assert np.abs(ind.gelu(x) - exact).max() < 1e-3
    assert ind.gelu(np.array([0.0]))[0] == 0.0


def test_bce_gradient_is_sigmoid_minus_label():
    """d(BCE)/dz = sigmoid(z) - y for a single sample (closed form)."""
    params = ind.init_params(1)
    params["W3"][:] = 0.0
    params["b3"][:] = 0.7
    X = RNG.uniform(-1, 1, size=(1, ind.NIN))
    for y in (0.0, 1.0):
        _, g = ind.loss_and_grads(params, X, np.array([y]))
        assert g["b3"][0] == pytest.approx(1.0 / (1.0 + math.exp(-0.7)) - y, rel=1e-12)


def test_features_are_normalised_and_scale_invariant():
    a = RNG.uniform(0, 1, size=(50, 5))
    r = RNG.uniform(1, 1000, size=(50, 5))
    p = RNG.uniform(1e4, 1e9, size=(50, 5))
    f = ind.features(a, r, p)
    assert f.shape == (50, 15)
    assert np.all(np.abs(f) <= 1.0) and np.all(f[:, [2, 7, 12]] == 0.0)
    assert np.all(np.abs(f).reshape(50, 3, 5).max(axis=2) == pytest.approx(1.0))
    f2 = ind.features(a, 3.0 * r + 5.0, 7.0 * p)   # affine changes of rho, scale of p
    np.testing.assert_allclose(f2[:, 5:], f[:, 5:], atol=1e-12)


def test_labels_from_weno_weights():
    """Smooth data gives label 1; a jump in any one variable gives 0."""
    x = 0.01 * np.arange(-2, 3)
    smooth = np.stack([1.0 + 0.1 * np.sin(x + k) for k in range(7)])
    assert ind.label(smooth) == 1
    jump = smooth.copy()
    jump[5] = np.where(np.arange(5) < 3, 1e6, 1e4)
    assert ind.label(jump) == 0


def test_adam_reduces_loss_on_separable_data():
    params = ind.init_params(5)
    X = RNG.uniform(-1, 1, size=(512, ind.NIN))
    y = (X[:, 1] + X[:, 6] > 0).astype(np.float64)
    state = {}
    l0, _ = ind.loss_and_grads(params, X, y)
    for _ in range(200):
        _, g = ind.loss_and_grads(params, X, y)
        ind.adam_step(params, g, state, lr=1e-2)
    l1, _ = ind.loss_and_grads(params, X, y)
    assert l1 < 0.5 * l0
