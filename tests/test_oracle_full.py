"""Pins of the oracle's full-problem regularisation (Algorithm 3, eqs. (14), (17), (25)).

The GCV values are checked against their definition with explicit influence
matrices built without the SVD (Tikhonov: A (A^T A + lambda^2 I)^{-1} A^T by
a linear solve; TSVD: the projector on the span of the k leading
eigenvectors of A A^T), so a dropped s_perp term, a wrong denominator or a
transposed operand fails here.
"""
import math

import numpy as np
import pytest


def _influence_tikh(A, lam):
    n = A.shape[1]
    return A @ np.linalg.solve(A.T @ A + lam * lam * np.eye(n), A.T)


def _gcv_def(A, f, H):
    m = A.shape[0]
    r = f - H @ f
    return float(r @ r) / (m - np.trace(H)) ** 2


@pytest.mark.parametrize("shape", [(14, 9), (12, 12)])
def test_gcv_full_matches_influence_matrix(orc, shape):
    rng = np.random.default_rng(shape[0] * 31 + shape[1])
    A = rng.standard_normal(shape) @ np.diag(np.logspace(0, -4, shape[1]))
    f = rng.standard_normal(shape[0])
    U, s, V = orc.full_svd(A)
    fhat = U.T @ f
    s_perp = max(0.0, float(f @ f) - float(fhat @ fhat))
    if shape[0] > shape[1]:
        assert s_perp > 1e-3 * float(f @ f)  # the part of f outside the range of A counts
    for lam in (1e-5, 1e-3, 1e-1, 3.0):
        ref = _gcv_def(A, f, _influence_tikh(A, lam))
        assert orc.gcv_full(s, fhat, s_perp, shape[0], lam) == pytest.approx(ref, rel=1e-9)


def test_gcv_tsvd_full_matches_projector(orc):
    rng = np.random.default_rng(7)
    m, n = 13, 9
    A = rng.standard_normal((m, n)) @ np.diag(np.logspace(0, -3, n))
    f = rng.standard_normal(m)
    U, s, V = orc.full_svd(A)
    fhat = U.T @ f
    s_perp = max(0.0, float(f @ f) - float(fhat @ fhat))
    w, E = np.linalg.eigh(A @ A.T)  # ascending
    E = E[:, ::-1]
    for k in range(1, n):
        H = E[:, :k] @ E[:, :k].T
        ref = _gcv_def(A, f, H)
        assert orc.gcv_tsvd_full(s, fhat, s_perp, m, k) == pytest.approx(ref, rel=1e-9)


def test_full_tsvd_gcv_brute_force(orc):
    rng = np.random.default_rng(11)
    n = 10
    A = rng.standard_normal((n, n)) @ np.diag(np.logspace(0, -6, n))
    f = A @ rng.standard_normal(n) + 1e-4 * rng.standard_normal(n)
    alpha, k = orc.full_tsvd_gcv(A, f)
    w, E = np.linalg.eigh(A @ A.T)
    E = E[:, ::-1]
    vals = [_gcv_def(A, f, E[:, :kk] @ E[:, :kk].T) for kk in range(1, n)]
    assert k == 1 + int(np.argmin(vals))
    # the rank-k TSVD solution is the minimum-norm least-squares solution of the rank-k truncation
    U, s, V = orc.full_svd(A)
    Ak = U[:, :k] @ np.diag(s[:k]) @ V[:, :k].T
    np.testing.assert_allclose(alpha, np.linalg.pinv(Ak, rcond=1e-14) @ f, rtol=1e-8, atol=1e-10)


def test_full_tikh_gcv_minimises_on_dense_scan(orc):
    rng = np.random.default_rng(3)
    n = 30
    A = rng.standard_normal((n, n)) @ np.diag(np.logspace(0, -8, n))
    f = A @ rng.standard_normal(n) + 1e-5 * rng.standard_normal(n)
    alpha, lam = orc.full_tikh_gcv(A, f)
    U, s, V = orc.full_svd(A)
    fhat = U.T @ f
    s_perp = max(0.0, float(f @ f) - float(fhat @ fhat))
    g = orc.gcv_full(s, fhat, s_perp, n, lam)
    lo = max(s[-1], 16 * np.finfo(float).eps * s[0])
    grid = np.exp(np.linspace(math.log(lo), math.log(s[0]), 4000))
    gmin = min(orc.gcv_full(s, fhat, s_perp, n, l) for l in grid)
    assert g <= gmin * (1 + 1e-6)
    # and the returned coefficients solve the normal equations at lambda
    np.testing.assert_allclose((A.T @ A + lam * lam * np.eye(n)) @ alpha, A.T @ f, rtol=1e-7,
                               atol=1e-9 * np.linalg.norm(A.T @ f))
