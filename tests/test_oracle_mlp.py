"""Pins for the oracle of the predictor network (oracle/mlp.py).

* back-propagation against central finite differences of the loss (an
  independent route to the same gradient);
* a 2-3-1 network evaluated by hand;
* Adam's first steps under a constant gradient have the closed form
  p - lr g / (|g| + eps) (bias-corrected moments equal g and g^2);
* the weighted MSE and its gradient at simple points;
* the feature map's layout and standardisation.
"""
import math

import numpy as np
import pytest

from oracle import mlp as M


def _loss(params, X, T, w, sizes):
    Y, _ = M.forward(params, X, sizes)
    return M.mse_loss(Y, T, w)[0]


@pytest.mark.parametrize("sizes", [(3, 5, 4, 2), M.SIZES])
def test_backprop_matches_finite_differences(sizes):
    rng = np.random.default_rng(7)
    P = M.n_params(sizes)
    params = rng.normal(scale=0.3, size=P)
    X = rng.normal(size=(5, sizes[0]))
    T = rng.normal(size=(5, sizes[-1]))
    w = np.array([1.0, 0.5])[: sizes[-1]] if sizes[-1] <= 2 else np.ones(sizes[-1])
    Y, H = M.forward(params, X, sizes)
    _, dY = M.mse_loss(Y, T, w)
    g = M.backward(params, H, dY, sizes)
    idx = np.unique(np.concatenate([rng.choice(P, size=min(P, 150), replace=False), np.arange(P - 20, P)]))
    h = 1e-6
    for i in idx:
        e = np.zeros(P)
        e[i] = h
        fd = (_loss(params + e, X, T, w, sizes) - _loss(params - e, X, T, w, sizes)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_tiny_network_by_hand():
    sizes = (2, 3, 1)
    W1 = np.array([[0.5, -1.0], [2.0, 0.25], [-0.3, 0.7]])
    b1 = np.array([0.1, -0.2, 0.05])
    W2 = np.array([[1.5, -0.5, 2.0]])
    b2 = np.array([0.3])
    params = np.concatenate([W1.ravel(), b1, W2.ravel(), b2])
    x = np.array([0.4, -1.2])
    h = [math.tanh(0.5 * 0.4 - 1.0 * -1.2 + 0.1), math.tanh(2.0 * 0.4 + 0.25 * -1.2 - 0.2),
         math.tanh(-0.3 * 0.4 + 0.7 * -1.2 + 0.05)]
    y = 1.5 * h[0] - 0.5 * h[1] + 2.0 * h[2] + 0.3
    Y, _ = M.forward(params, x[None, :], sizes)
    assert Y[0, 0] == pytest.approx(y, rel=1e-15)
    assert M.n_params(M.SIZES) == 24 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 2 + 2


def test_adam_constant_gradient_closed_form():
    p0 = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 4.0])
    lr, eps = 1e-2, 1e-8
    p, m, v = M.adam_step(p0, g, np.zeros(3), np.zeros(3), 1, lr, eps=eps)
    np.testing.assert_allclose(p, p0 - lr * g / (np.abs(g) + eps), rtol=1e-14)
    p2, m, v = M.adam_step(p, g, m, v, 2, lr, eps=eps)
    np.testing.assert_allclose(p2, p - lr * g / (np.abs(g) + eps), rtol=1e-13)


def test_mse_loss_and_gradient():
    Y = np.array([[1.0, 2.0], [0.0, -1.0]])
    T = np.array([[0.0, 2.0], [1.0, 1.0]])
    w = np.array([2.0, 0.5])
    loss, dY = M.mse_loss(Y, T, w)
    assert loss == pytest.approx((2.0 * 1.0 + 0.0 + 2.0 * 1.0 + 0.5 * 4.0) / 2.0)
    np.testing.assert_allclose(dY, [[2.0, 0.0], [-2.0, -1.0]])
    assert M.mse_loss(T, T, w)[0] == 0.0


def test_features_layout():
    a = np.arange(1.0, 13.0)
    b = np.arange(2.0, 15.0)
    raw = np.concatenate([np.log(a[:10]), np.log(b[1:11]), [math.log(5.0), math.log(2.0), math.log(1800), math.log(0.08)]])
    x = M.features(a, b, 5.0, 2.0, 1800, 0.08, np.zeros(24), np.ones(24))
    np.testing.assert_allclose(x, raw, rtol=1e-15)
    z = M.features(a, b, 5.0, 2.0, 1800, 0.08, raw, 2.0 * np.ones(24))
    assert np.all(z == 0.0)
