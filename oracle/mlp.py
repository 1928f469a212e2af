"""Plain FP64 CPU oracle of the learned predictor's network.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library.  It
shares no code with the HIP kernels.

The network (the predictor of the regularisation parameter and of the
Golub-Kahan stopping index) is a multilayer perceptron
    h_0 = x,  h_l = tanh(W_l h_{l-1} + b_l) (l = 1..L-1),  y = W_L h_{L-1} + b_L,
with the parameters stored flat, layer by layer, each layer as W_l
(out x in, row-major) followed by b_l.  Training minimises the weighted mean
squared error  (1/B) sum_b sum_k w_k (y_bk - t_bk)^2  with Adam.  Everything
here follows those definitions directly: forward pass, back-propagation by
the chain rule (d tanh(z)/dz = 1 - tanh(z)^2), the loss and its gradient, and
one Adam step (bias-corrected first and second moments).
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

# The architecture the library implements: 24 inputs, three tanh layers of
# width 128, 2 outputs.
SIZES = (24, 128, 128, 128, 2)


def n_params(sizes: Sequence[int] = SIZES) -> int:
    return sum(sizes[l + 1] * sizes[l] + sizes[l + 1] for l in range(len(sizes) - 1))


def unpack(params: np.ndarray, sizes: Sequence[int] = SIZES) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Views (W_l, b_l) into the flat parameter vector."""
    out, off = [], 0
    for l in range(len(sizes) - 1):
        o, i = sizes[l + 1], sizes[l]
        W = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((W, b))
    assert off == params.shape[0]
    return out


def forward(params: np.ndarray, X: np.ndarray, sizes: Sequence[int] = SIZES):
    """Returns (Y, H) with H[l] the input of layer l (H[0] = X), in FP64."""
    layers = unpack(np.asarray(params, dtype=np.float64), sizes)
    H = [np.asarray(X, dtype=np.float64)]
    h = H[0]
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if l < len(layers) - 1:
            h = np.tanh(z)
            H.append(h)
        else:
            h = z
    return h, H


def backward(params: np.ndarray, H: List[np.ndarray], dY: np.ndarray, sizes: Sequence[int] = SIZES) -> np.ndarray:
    """Gradient of a scalar loss with respect to the flat parameters, given dL/dY (chain rule)."""
    layers = unpack(np.asarray(params, dtype=np.float64), sizes)
    grads = [None] * len(layers)
    d = np.asarray(dY, dtype=np.float64)  # dL/dz of the current layer
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (d.T @ H[l], d.sum(axis=0))
        if l > 0:
            dh = d @ W
            d = dh * (1.0 - H[l] ** 2)  # H[l] = tanh(z_{l-1})
    return np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])


def mse_loss(Y: np.ndarray, T: np.ndarray, w: Sequence[float]):
    """(loss, dL/dY) of the weighted mean squared error over the batch."""
    Y = np.asarray(Y, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    B = Y.shape[0]
    r = Y - T
    loss = float(np.sum(w * r * r) / B)
    return loss, 2.0 * w * r / B


def adam_step(params, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step number t >= 1); returns (params, m, v)."""
    params = np.asarray(params, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def features(alpha: np.ndarray, beta: np.ndarray, kappa: float, eps: float, n: int, h: float,
             mean: np.ndarray, std: np.ndarray, n_probe: int = 10) -> np.ndarray:
    """Standardised predictor input: (log alpha_1..alpha_p, log beta_2..beta_{p+1}, log kappa,
    log eps, log n, log h), p = n_probe, then (x - mean) / std."""
    x = np.concatenate([np.log(np.asarray(alpha[:n_probe], dtype=np.float64)),
                        np.log(np.asarray(beta[1:n_probe + 1], dtype=np.float64)),
                        [math.log(kappa), math.log(eps), math.log(n), math.log(h)]])
    return (x - np.asarray(mean, dtype=np.float64)) / np.asarray(std, dtype=np.float64)
