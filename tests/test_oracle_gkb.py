"""Pins for the oracle's products and Golub-Kahan bidiagonalisation (Algorithm 1).

* products: the C loops against numpy's BLAS matmul of the same assembled
  matrix, entry-wise vs stored, sampled vs full;
* the Krylov relations A Z = W C and A^T W_l = Z_l (C_l)_{1:l,1:l}^T, the
  orthonormality of both bases and W^T f = beta_1 e_1 (eq. (26) and the
  projected-formulation remark of Section 4.2; the paper's second relation
  misses alpha_{l+1} z_{l+1} e_{l+1}^T in its last column, so it is checked
  on the first l columns);
* invariance of alpha, beta under a permutation of the nodes (both A and f
  permute consistently; the Krylov scalars are unitarily invariant);
* breakdown: a full Krylov space at l = N, and f chosen as a left singular
  vector of A so that beta_2 = 0.
"""
import numpy as np
import pytest

from paper_2511_09798_amd import inputs as I


@pytest.fixture(scope="module")
def small(orc):
    p = I.cube_scaled(150, 90, kappa=6.0, eps=2.0, ell=30)
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    return p, A


def test_products_match_blas(orc, small):
    p, A = small
    x = I.random_vector(p.n, 1)
    y = orc.apply(A, p.nodes, p.n_int, p.kappa, p.eps, x)
    yt = orc.apply(A, p.nodes, p.n_int, p.kappa, p.eps, x, trans=True)
    scale = np.abs(A) @ np.abs(x)
    scale_t = np.abs(A).T @ np.abs(x)
    assert np.all(np.abs(y - A @ x) <= 1e-14 * scale)
    assert np.all(np.abs(yt - A.T @ x) <= 1e-14 * scale_t)
    # entry-wise evaluation gives the same products (same entries, same order)
    ym = orc.apply(None, p.nodes, p.n_int, p.kappa, p.eps, x)
    ytm = orc.apply(None, p.nodes, p.n_int, p.kappa, p.eps, x, trans=True)
    assert np.array_equal(ym, y) and np.array_equal(ytm, yt)
    idx = np.array([0, 5, p.n_int - 1, p.n_int, p.n - 1])
    assert np.array_equal(orc.apply_sampled(p.nodes, p.n_int, p.kappa, p.eps, x, idx), y[idx])
    assert np.array_equal(orc.apply_sampled(p.nodes, p.n_int, p.kappa, p.eps, x, idx, trans=True), yt[idx])


def test_gkb_relations(orc, small):
    p, A = small
    g = orc.gkb(A, p.nodes, p.n_int, p.kappa, p.eps, p.rhs, p.ell)
    assert g.ell == p.ell and g.flag == 0
    C = orc.bidiag_matrix(g.alpha, g.beta)
    c2 = np.linalg.norm(C, 2)
    assert np.linalg.norm(A @ g.Z - g.W @ C) / c2 < 1e-12
    Cl = C[: g.ell, : g.ell]
    assert np.linalg.norm(A.T @ g.W[:, : g.ell] - g.Z @ Cl.T) / c2 < 1e-12
    assert np.max(np.abs(g.W.T @ g.W - np.eye(g.ell + 1))) < 1e-12
    assert np.max(np.abs(g.Z.T @ g.Z - np.eye(g.ell))) < 1e-12
    b1 = np.linalg.norm(p.rhs)
    assert g.beta[0] == pytest.approx(b1, rel=1e-15)
    e1 = np.zeros(g.ell + 1)
    e1[0] = b1
    assert np.linalg.norm(g.W.T @ p.rhs - e1) / b1 < 1e-12
    assert np.all(g.alpha > 0) and np.all(g.beta > 0)


def test_gkb_relations_cube_n1800(orc):
    p = I.cube_small()
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    g = orc.gkb(A, p.nodes, p.n_int, p.kappa, p.eps, p.rhs, p.ell)
    C = orc.bidiag_matrix(g.alpha, g.beta)
    assert np.linalg.norm(A @ g.Z - g.W @ C) / np.linalg.norm(C, 2) < 1e-12
    assert np.max(np.abs(g.W.T @ g.W - np.eye(g.ell + 1))) < 1e-12
    assert np.max(np.abs(g.Z.T @ g.Z - np.eye(g.ell))) < 1e-12


def test_gkb_matrix_free_equals_stored(orc, small):
    p, A = small
    g1 = orc.gkb(A, p.nodes, p.n_int, p.kappa, p.eps, p.rhs, 12)
    g2 = orc.gkb(None, p.nodes, p.n_int, p.kappa, p.eps, p.rhs, 12)
    assert np.array_equal(g1.alpha, g2.alpha) and np.array_equal(g1.beta, g2.beta)


def test_gkb_permutation_invariance(orc, small):
    p, A = small
    g = orc.gkb(A, p.nodes, p.n_int, p.kappa, p.eps, p.rhs, 20)
    rng = np.random.default_rng(2)
    pi = rng.permutation(p.n_int)
    pb = p.n_int + rng.permutation(p.n_bnd)
    perm = np.concatenate([pi, pb])
    Xp = p.nodes[perm]
    Ap = orc.assemble(Xp, p.n_int, p.kappa, p.eps)
    assert np.array_equal(Ap, A[np.ix_(perm, perm)])
    gp = orc.gkb(Ap, Xp, p.n_int, p.kappa, p.eps, p.rhs[perm], 20)
    assert np.max(np.abs(gp.alpha - g.alpha) / g.alpha) < 1e-12
    assert np.max(np.abs(gp.beta - g.beta) / g.beta) < 1e-12


def test_gkb_without_reorth_loses_orthogonality(orc):
    # plain Algorithm 1 on an ill-conditioned matrix: the recurrence still
    # holds (A Z = W C up to rounding) but orthogonality is lost; full
    # reorthogonalisation keeps it.
    p = I.cube_small()
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    g0 = orc.gkb(A, p.nodes, p.n_int, p.kappa, p.eps, p.rhs, 60, reorth=False)
    C0 = orc.bidiag_matrix(g0.alpha, g0.beta)
    assert np.linalg.norm(A @ g0.Z - g0.W @ C0) / np.linalg.norm(C0, 2) < 1e-12
    assert np.max(np.abs(g0.Z.T @ g0.Z - np.eye(60))) > 1e-6


def test_gkb_full_space_breakdown(orc):
    # At l = N the Krylov space is all of R^N; the next beta vanishes.
    n = 16
    X = I.random_nodes_cube(n, 116)
    A = orc.assemble(X, 8, 2.0, 6.0)
    f = I.random_vector(n, 7)
    g = orc.gkb(A, X, 8, 2.0, 6.0, f, n)
    assert g.ell == n and g.flag == 2 and g.beta[n] == 0.0
    C = orc.bidiag_matrix(g.alpha, g.beta)
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(np.linalg.svd(C, compute_uv=False) - sv) / sv) < 1e-10


def test_gkb_beta_breakdown_on_singular_vector(orc):
    n = 24
    X = I.random_nodes_cube(n, 124)
    A = orc.assemble(X, 12, 2.0, 6.0)
    U, s, Vt = np.linalg.svd(A)
    f = 3.0 * U[:, 0]
    g = orc.gkb(A, X, 12, 2.0, 6.0, f, 5)
    assert g.flag == 2 and g.ell == 1
    assert g.alpha[0] == pytest.approx(s[0], rel=1e-12)
    assert g.beta[1] == 0.0
