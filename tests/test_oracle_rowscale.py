"""Pins of the oracle's row-scaled operator (an opt-in equilibration, not in the paper).

Reading: D = diag(A)^{-1} scales the rows of the stacked system A c = f
(eq. (11)), so the method runs on (D A) c = D f.  The diagonal of A has a
closed form (r = 0: phi = 1 and Lap phi = 3 eps^2), interior A_ii =
3 eps^2 + kappa^2, boundary A_ii = 1.  Each check below is independent of the
oracle's own scaling code: the scaled matrix is formed here with numpy from
the unscaled assembly and the closed-form diagonal, and the whole solve is
compared with textbook dense solutions.
"""
import numpy as np
import pytest

from paper_2511_09798_amd import inputs as I

EPS = np.finfo(np.float64).eps


def _case(n_int=70, n_bnd=40, kappa=4.0, eps=3.0, seed=5):
    X = I.random_nodes_cube(n_int + n_bnd, seed)
    f = I.random_vector(n_int + n_bnd, seed + 1)
    return X, n_int, kappa, eps, f


def _closed_form_d(n, n_int, kappa, eps):
    d = np.ones(n)
    d[:n_int] = 1.0 / (3.0 * eps * eps + kappa * kappa)
    return d


def test_row_scale_closed_form(orc):
    X, n_int, kappa, eps, f = _case()
    d = orc.row_scale(X, n_int, kappa, eps)
    dc = _closed_form_d(X.shape[0], n_int, kappa, eps)
    np.testing.assert_allclose(d, dc, rtol=4 * EPS, atol=0)
    # kappa = 5, eps = 2 (the 1800-node cube): interior rows scaled by 1/37
    d2 = orc.row_scale(X, n_int, 5.0, 2.0)
    assert d2[0] == pytest.approx(1.0 / 37.0, rel=4 * EPS) and d2[-1] == 1.0


@pytest.mark.parametrize("trans", [False, True])
def test_scaled_products_are_rows_of_DA(orc, trans):
    X, n_int, kappa, eps, f = _case()
    A = orc.assemble(X, n_int, kappa, eps)
    DA = A / np.diag(A)[:, None]  # rows divided by the diagonal, formed here
    d = orc.row_scale(X, n_int, kappa, eps)
    x = I.random_vector(X.shape[0], 9)
    y = orc.apply(None, X, n_int, kappa, eps, x, trans=trans, d=d)
    ref = (DA.T if trans else DA) @ x
    scale = (np.abs(DA.T) if trans else np.abs(DA)) @ np.abs(x)
    assert np.all(np.abs(y - ref) <= 1e-14 * scale)
    idx = np.array([0, 5, n_int - 1, n_int, X.shape[0] - 1], dtype=np.int64)
    ys = orc.apply_sampled(X, n_int, kappa, eps, x, idx, trans=trans, d=d)
    np.testing.assert_array_equal(ys, y[idx])
    # a stored A scaled by the caller gives the same numbers bit for bit
    y2 = orc.apply(A * d[:, None], X, n_int, kappa, eps, x, trans=trans)
    np.testing.assert_array_equal(y, y2)


@pytest.mark.parametrize("stored", [True, False])
def test_scaled_gkb_relations(orc, stored):
    # Golub-Kahan on D A from D f: the relations hold with the scaled matrix formed here
    X, n_int, kappa, eps, f = _case()
    A = orc.assemble(X, n_int, kappa, eps)
    dg = np.diag(A)
    DA = A / dg[:, None]
    Df = f / dg
    ell = 30
    r = orc.solve(X, n_int, kappa, eps, f, ell, stored=stored, row_scale=1)
    g = r.gkb
    C = orc.bidiag_matrix(g.alpha, g.beta)
    c2 = np.linalg.norm(C, 2)
    assert np.linalg.norm(DA @ g.Z - g.W @ C) / c2 < 1e-12
    assert np.linalg.norm(DA.T @ g.W[:, :ell] - g.Z @ C[:ell, :ell].T) / c2 < 1e-12
    assert np.max(np.abs(g.W.T @ g.W - np.eye(ell + 1))) < 1e-12
    e1 = np.zeros(ell + 1)
    e1[0] = g.beta[0]
    assert np.linalg.norm(g.W.T @ Df - e1) <= 1e-12 * g.beta[0]
    # the unscaled run is a different Krylov space
    r0 = orc.solve(X, n_int, kappa, eps, f, ell, stored=stored, row_scale=0)
    assert abs(r0.gkb.beta[0] - g.beta[0]) > 1e-3 * g.beta[0]


def test_scaled_stored_equals_entrywise(orc):
    X, n_int, kappa, eps, f = _case()
    a = orc.solve(X, n_int, kappa, eps, f, 25, stored=True, row_scale=1)
    b = orc.solve(X, n_int, kappa, eps, f, 25, stored=False, row_scale=1)
    np.testing.assert_array_equal(a.alpha, b.alpha)
    np.testing.assert_array_equal(a.beta, b.beta)
    np.testing.assert_array_equal(a.coef, b.coef)


def _small_well_conditioned():
    # 48 nodes, a sharp basis (large eps): A is well conditioned
    X = I.random_nodes_cube(48, 77)
    return X, 32, 2.0, 6.0, I.random_vector(48, 78)


def test_full_space_tsvd_is_the_solution_of_A(orc):
    # l = n, Ine-TSVD with k = n: both the scaled and the unscaled method
    # return A^{-1} f, since (D A)^{-1} D f = A^{-1} f
    X, n_int, kappa, eps, f = _small_well_conditioned()
    n = X.shape[0]
    A = orc.assemble(X, n_int, kappa, eps)
    cond = np.linalg.cond(A)
    assert cond < 1e8
    c_ref = np.linalg.solve(A, f)
    for rs in (0, 1):
        r = orc.solve(X, n_int, kappa, eps, f, n, method=orc.METHOD_INE_TSVD, rule=orc.RULE_FIXED, k_trunc=n,
                      row_scale=rs)
        assert r.ell == n
        err = np.linalg.norm(r.coef - c_ref) / np.linalg.norm(c_ref)
        assert err <= 1e3 * cond * EPS, (rs, err, cond)


def test_full_space_hkt_is_weighted_tikhonov(orc):
    # l = n, HKT at a fixed lambda on the scaled system: the minimiser of
    # ||D (A c - f)||^2 + lambda^2 ||c||^2, (A^T D^2 A + lambda^2 I) c = A^T D^2 f
    X, n_int, kappa, eps, f = _small_well_conditioned()
    n = X.shape[0]
    A = orc.assemble(X, n_int, kappa, eps)
    D = np.diag(1.0 / np.diag(A))
    lam = 1e-3 * np.linalg.norm(D @ A, 2)
    M = (D @ A).T @ (D @ A) + lam * lam * np.eye(n)
    c_ref = np.linalg.solve(M, (D @ A).T @ (D @ f))
    r = orc.solve(X, n_int, kappa, eps, f, n, rule=orc.RULE_FIXED, lambda_fixed=lam, row_scale=1)
    assert np.linalg.norm(r.coef - c_ref) <= 1e-9 * np.linalg.norm(c_ref)
    # and it differs from the unscaled Tikhonov solution at the same lambda
    c0 = np.linalg.solve(A.T @ A + lam * lam * np.eye(n), A.T @ f)
    assert np.linalg.norm(c0 - c_ref) > 1e-6 * np.linalg.norm(c_ref)
