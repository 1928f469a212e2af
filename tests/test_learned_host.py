"""Host-side pieces of the learned predictor: problem sampling (including the
pump-casing-like solid), the feature layout and the parameter initialisation.
"""
import math

import numpy as np
import pytest

from oracle import mlp as M
from paper_2511_09798_amd import learned as L


def test_casing_interior_and_boundary():
    rng = np.random.default_rng(3)
    C = L.Casing
    xi = C.interior(2000, rng)
    assert np.all(C.inside(xi))
    xb = C.boundary(600, rng)
    # every boundary point has points of the solid and of its complement within 1e-3
    dirs = rng.normal(size=(64, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    for p in xb:
        q = p + 1e-3 * dirs
        ins = C.inside(q)
        assert ins.any() and (~ins).any()
    # all five surface parts are represented (outer wall, hub, caps, pipe wall, pipe end)
    r = np.hypot(xb[:, 0], xb[:, 1])
    assert np.any(np.isclose(r, 1.0)) and np.any(np.isclose(r, 0.3))
    assert np.any(np.isclose(np.abs(xb[:, 2]), 0.3)) and np.any(np.isclose(xb[:, 0], 1.2))


def test_casing_volume():
    # ring volume plus the part of the pipe outside the ring: 0.6 pi (1 - 0.09) + pipe beyond the wall
    v = L.Casing.volume(np.random.default_rng(1), 1_000_000)
    ring = 0.6 * math.pi * (1.0 - 0.09)
    pipe = math.pi * 0.25 ** 2 * 1.2
    assert ring < v < ring + pipe
    assert L.CASING_VOLUME == pytest.approx(v, rel=0.02)


@pytest.mark.parametrize("kind", ["cube", "sphere", "casing"])
def test_sample_problem_shapes(kind):
    rng = np.random.default_rng(5)
    p = L.sample_problem(rng, kind=kind, n=1200, kappa=4.0, eps=1.5)
    assert p["x_int"].shape == (960, 3) and p["x_bnd"].shape == (240, 3)
    assert p["f_int"].shape == (960,) and np.all(p["f_int"] == 0.0)
    assert p["x_eval"].shape == (L.N_EVAL, 3)
    assert p["h"] > 0
    # g is the plane wave at the boundary nodes, with wavenumber kappa (|Lap u| = kappa^2 |u|)
    assert np.max(np.abs(p["g_bnd"])) <= 1.0


def test_raw_features_match_oracle_layout():
    rng = np.random.default_rng(2)
    a = rng.random(12) + 0.1
    b = rng.random(13) + 0.1
    x = L.raw_features(a, b, 3.0, 1.2, 5000, 0.05)
    xo = M.features(a, b, 3.0, 1.2, 5000, 0.05, np.zeros(24), np.ones(24))
    np.testing.assert_allclose(x, xo, rtol=0, atol=0)


def test_init_params_layout():
    p = L.init_params(0)
    assert p.dtype == np.float32 and p.shape == (M.n_params(),)
    layers = M.unpack(p.astype(np.float64))
    for W, b in layers:
        assert np.all(b == 0.0)
        lim = math.sqrt(6.0 / (W.shape[0] + W.shape[1]))
        assert np.max(np.abs(W)) <= lim
