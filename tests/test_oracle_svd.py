"""Pins for the oracle's dense Jacobi SVD and the projected SVD of C_l (Algorithms 2 and 4, step 2).

* Jacobi SVD against LAPACK (numpy) on random and graded matrices, plus
  orthonormality and reconstruction;
* projected data f~ = U~^T(beta_1 e_1): |f~_i| against LAPACK's U, the
  norm identity sum f~_i^2 = beta_1^2, and f~_{l+1} against the projected
  least-squares residual min ||C y - beta_1 e_1|| (computed by lstsq);
* at l = N on tiny N the Ritz values are the singular values of A,
  compared with a brute-force Jacobi SVD of the assembled A and with LAPACK.
"""
import numpy as np
import pytest

from paper_2511_09798_amd import inputs as I


@pytest.mark.parametrize("shape,seed", [((7, 7), 1), ((30, 20), 2), ((61, 60), 3), ((5, 1), 4)])
def test_jacobi_svd_random(orc, shape, seed):
    rng = np.random.default_rng(seed)
    M = rng.normal(size=shape)
    s, U, V = orc.jacobi_svd(M)
    s_ref = np.linalg.svd(M, compute_uv=False)
    assert np.max(np.abs(s - s_ref) / s_ref[0]) < 1e-14
    assert np.all(np.diff(s) <= 0)
    assert np.max(np.abs(U.T @ U - np.eye(shape[1]))) < 1e-13
    assert np.max(np.abs(V.T @ V - np.eye(shape[1]))) < 1e-13
    assert np.max(np.abs(U * s @ V.T - M)) < 1e-13 * s[0]


def test_jacobi_svd_graded_high_relative_accuracy(orc):
    # Bidiagonal with entries spanning 1e-15..1: one-sided Jacobi resolves the
    # small singular values to high relative accuracy (compared with the
    # singular values of the exactly diagonal case, which are its entries).
    d = np.logspace(0, -15, 12)
    s, U, V = orc.jacobi_svd(np.diag(d))
    assert np.max(np.abs(s - d) / d) < 1e-15
    rng = np.random.default_rng(11)
    M = np.diag(d) @ (np.eye(12) + 1e-3 * rng.normal(size=(12, 12)))
    s2, _, _ = orc.jacobi_svd(M)
    # row scaling by D keeps relative perturbation of sv tiny: |s_i/d_i - 1| <~ 1e-3 * sqrt(12)
    assert np.max(np.abs(s2 / d - 1.0)) < 1e-2


def _gkb_scalars(orc, n_int, n_bnd, kappa, eps, ell, seed=21):
    p = I.cube_scaled(n_int, n_bnd, kappa, eps, ell, seed=seed)
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    g = orc.gkb(A, p.nodes, p.n_int, p.kappa, p.eps, p.rhs, ell)
    return p, A, g


@pytest.mark.parametrize("ell", [1, 2, 10, 40])
def test_proj_svd_against_lapack(orc, ell):
    p, A, g = _gkb_scalars(orc, 120, 80, 5.0, 2.0, ell)
    s, ft, V = orc.proj_svd(g.alpha, g.beta)
    C = orc.bidiag_matrix(g.alpha, g.beta)
    Uf, sf, Vtf = np.linalg.svd(C)
    assert np.max(np.abs(s - sf) / sf[0]) < 1e-14
    b1 = g.beta[0]
    # |f~_i| = beta_1 |U~_{1,i}| for all i <= l+1 (signs of singular vectors are arbitrary)
    assert np.max(np.abs(np.abs(ft) - b1 * np.abs(Uf[0, :]))) < 1e-12 * b1
    assert np.sum(ft ** 2) == pytest.approx(b1 * b1, rel=1e-13)
    # f~_{l+1} is the residual of the projected least-squares problem
    y_ls, res, rank, _ = np.linalg.lstsq(C, np.eye(ell + 1)[:, 0] * b1, rcond=None)
    r_ls = np.linalg.norm(C @ y_ls - np.eye(ell + 1)[:, 0] * b1)
    assert abs(ft[ell]) == pytest.approx(r_ls, rel=1e-10, abs=1e-14 * b1)
    # right singular vectors: C v_i = s_i u_i, so ||C v_i|| = s_i and V orthogonal
    assert np.max(np.abs(np.linalg.norm(C @ V, axis=0) - s) / s[0]) < 1e-13
    assert np.max(np.abs(V.T @ V - np.eye(ell))) < 1e-13


@pytest.mark.parametrize("n", [8, 16, 32, 64])
def test_ritz_values_at_full_dimension(orc, n):
    # l = N with eps chosen so cond(A) <= 1e8: the GKB reaches the whole space
    # and sigma(C_N) = sigma(A).  Brute force: Jacobi SVD of the assembled A.
    X = I.random_nodes_cube(n, 100 + n)
    A = orc.assemble(X, n // 2, 2.0, 6.0)
    f = I.random_vector(n, n)
    g = orc.gkb(A, X, n // 2, 2.0, 6.0, f, n)
    assert g.ell == n
    s, ft, V = orc.proj_svd(g.alpha, g.beta)
    s_bf, _, _ = orc.jacobi_svd(A)
    s_la = np.linalg.svd(A, compute_uv=False)
    big = s_bf >= 1e-4 * s_bf[0]
    assert np.max(np.abs(s[big] - s_bf[big]) / s_bf[big]) < 1e-12
    assert np.max(np.abs(s - s_bf)) < 10 * n * np.finfo(float).eps * s_bf[0]
    assert np.max(np.abs(s_bf - s_la) / s_la) < 1e-12
    assert abs(ft[n]) < 1e-10 * g.beta[0]


@pytest.mark.parametrize("ratio,ell", [(10.0, 40), (1e10, 40), (0.5, 30)])
def test_null_vector_closed_form(orc, ratio, ell):
    # Constant alpha_j / beta_{j+1} = r: the null vector of C^T is n_j = (-r)^(j-1),
    # ||n||^2 = (r^(2(l+1)) - 1) / (r^2 - 1), so |f~_{l+1}| = beta_1 / ||n||.
    # For r = 1e10 the entries pass 1e308 (rescaling path) and the value underflows to ~0.
    alpha = np.full(ell, ratio)
    beta = np.concatenate([[2.0], np.full(ell, 1.0)])
    s, ft, V = orc.proj_svd(alpha, beta)
    assert np.all(np.isfinite(ft)) and np.all(np.isfinite(s))
    log_n2 = np.log(ratio ** 2) * (ell + 1) if ratio > 1e3 else np.log((ratio ** (2 * (ell + 1)) - 1) / (ratio ** 2 - 1))
    expect = 2.0 * np.exp(-0.5 * log_n2)
    assert abs(ft[ell]) == pytest.approx(expect, rel=1e-12, abs=1e-300)
    assert np.sum(ft ** 2) == pytest.approx(4.0, rel=1e-13)
