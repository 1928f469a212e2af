"""Pins for the oracle's LSQR early stopping (Section 3.4) and weighted GCV.

Each check ties the oracle to something outside its own code:
* the k-th LSQR iterate equals the k-th iterate of textbook CGLS (an
  independent algorithm, conjugate gradients on the normal equations);
* at l = N the last iterate is the least-squares solution of A alpha = f;
* rho_k and eta_k equal the full-problem residual ||A alpha_k - f|| and
  ||alpha_k|| computed directly with the assembled A;
* rho_k never increases and eta_k never decreases (CGLS properties);
* the influence matrix of the k-th iterate has trace k (the Krylov GCV
  denominator);
* Menger curvature of three points on a circle of radius R is +-1/R;
* a synthetic L-shaped sequence has its corner where it is built;
* the weighted projected GCV has a closed-form minimiser at l = 1;
* the last LSQR iterate equals the HKT solution at lambda = 0 (SVD route).
"""
import math

import numpy as np
import pytest

from paper_2511_09798_amd import inputs as I


def _small_problem(orc, n_int=30, n_bnd=18, eps=1.2, kappa=2.0, seed=5):
    X = I.random_nodes_cube(n_int + n_bnd, seed)
    f = I.random_vector(n_int + n_bnd, seed + 1)
    A = orc.assemble(X, n_int, kappa, eps)
    return X, f, A, n_int, kappa, eps


def _cgls(A, f, k):
    """Textbook CGLS (Hestenes-Stiefel on A^T A x = A^T f, x_0 = 0): the first k iterates."""
    x = np.zeros(A.shape[1])
    r = f.copy()
    s = A.T @ r
    p = s.copy()
    gamma = s @ s
    out = []
    for _ in range(k):
        q = A @ p
        a = gamma / (q @ q)
        x = x + a * p
        r = r - a * q
        s = A.T @ r
        g_new = s @ s
        p = s + (g_new / gamma) * p
        gamma = g_new
        out.append(x.copy())
    return out


def test_lsqr_iterates_equal_cgls(orc):
    # the equivalence holds for any A; a well-conditioned one (singular values in [1, 20]) keeps
    # CGLS, which has no reorthogonalisation, accurate to rounding
    X, f, _, n_int, kappa, eps = _small_problem(orc)
    n = X.shape[0]
    rng = np.random.default_rng(2)
    Q1, _ = np.linalg.qr(rng.normal(size=(n, n)))
    Q2, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = Q1 @ np.diag(np.linspace(20.0, 1.0, n)) @ Q2.T
    ell = 12
    g = orc.gkb(A, X, n_int, kappa, eps, f, ell)
    rho, eta, Y = orc.lsqr_path(g.alpha, g.beta)
    xs = _cgls(A, f, ell)
    for k in range(1, ell + 1):
        ak = g.Z[:, :k] @ Y[k - 1, :k]
        assert np.linalg.norm(ak - xs[k - 1]) <= 1e-9 * np.linalg.norm(xs[k - 1])


def test_lsqr_full_space_is_least_squares(orc):
    n = 12
    X = I.random_nodes_cube(n, 31)
    f = I.random_vector(n, 32)
    A = orc.assemble(X, 8, 1.5, 0.9)
    g = orc.gkb(A, X, 8, 1.5, 0.9, f, n)
    assert g.ell == n
    rho, eta, Y = orc.lsqr_path(g.alpha, g.beta)
    a_last = g.Z @ Y[n - 1]
    ref = np.linalg.lstsq(A, f, rcond=None)[0]
    assert np.linalg.norm(a_last - ref) <= 1e-8 * np.linalg.norm(ref)
    assert rho[-1] <= 1e-8 * np.linalg.norm(f)


def test_lsqr_norms_are_full_problem_norms(orc):
    X, f, A, n_int, kappa, eps = _small_problem(orc)
    ell = 20
    g = orc.gkb(A, X, n_int, kappa, eps, f, ell)
    rho, eta, Y = orc.lsqr_path(g.alpha, g.beta)
    for k in (1, 5, 13, 20):
        ak = g.Z[:, :k] @ Y[k - 1, :k]
        assert rho[k - 1] == pytest.approx(np.linalg.norm(A @ ak - f), rel=1e-9)
        assert eta[k - 1] == pytest.approx(np.linalg.norm(ak), rel=1e-12)


def test_lsqr_monotone(orc):
    X, f, A, n_int, kappa, eps = _small_problem(orc, seed=9)
    g = orc.gkb(A, X, n_int, kappa, eps, f, 30)
    rho, eta, _ = orc.lsqr_path(g.alpha, g.beta)
    assert np.all(np.diff(rho) <= 1e-12 * rho[0])
    assert np.all(np.diff(eta) >= -1e-12 * eta[-1])


def test_krylov_gcv_trace_is_k(orc):
    # influence matrix H_k = A Z_k C_k^+ W_{k+1}^T maps f to A alpha_k; trace k
    X, f, A, n_int, kappa, eps = _small_problem(orc, seed=13)
    ell = 10
    g = orc.gkb(A, X, n_int, kappa, eps, f, ell)
    C = orc.bidiag_matrix(g.alpha, g.beta)
    for k in (1, 4, 10):
        Ck = C[: k + 1, :k]
        H = A @ g.Z[:, :k] @ np.linalg.pinv(Ck) @ g.W[:, : k + 1].T
        assert np.trace(H) == pytest.approx(k, abs=1e-9)
        assert np.allclose(H @ H, H, atol=1e-9)  # an orthogonal projector
    rho = np.array([0.5, 0.25])
    G = orc.krylov_gcv(rho, 10)
    assert G[0] == pytest.approx(0.25 / 81.0) and G[1] == pytest.approx(0.0625 / 64.0)


def test_menger_curvature_of_circle(orc):
    R = 2.5
    c0 = np.array([0.3, -1.0])
    pts = [c0 + R * np.array([math.cos(t), math.sin(t)]) for t in (0.1, 0.9, 2.0)]
    assert orc.menger_curvature(*pts) == pytest.approx(1.0 / R, rel=1e-12)  # counterclockwise
    assert orc.menger_curvature(*pts[::-1]) == pytest.approx(-1.0 / R, rel=1e-12)


def test_discrete_lcurve_corner_on_synthetic_l(orc):
    # k = 1..10: the residual falls by a decade per step at nearly constant norm;
    # k = 11..20: the residual stalls while the norm grows by a decade per step.
    k = np.arange(1, 21)
    rho = np.where(k <= 10, 10.0 ** (-(k - 1)), 10.0 ** (-9) * (1.0 - 1e-3 * (k - 10)))
    eta = np.where(k <= 10, 1.0 + 1e-3 * k, 10.0 ** (k - 10))
    kc, kap, edge, _ = orc.lcurve_discrete_corner(rho, eta)
    assert kc == 10 and not edge and kap > 0


def test_weighted_gcv_closed_form_l1(orc):
    # l = 1: C = [a; b], s = sqrt(a^2 + b^2), f~ = beta_1 (a, -b)/s; with F = f~_1^2, G = f~_2^2 the
    # weighted GCV ((1-phi)^2 F + G) / (2 - omega phi)^2 is stationary at 1 - phi = omega G / ((2-omega) F),
    # and lambda^2 = s^2 (1 - phi) / phi.  A minimum located by comparing function values is fixed
    # only to about sqrt(eps_mach) relative (the function is flat there): 1e-6 in log(lambda).
    a, b, beta1 = 2.0, 0.7, 1.3
    s = math.hypot(a, b)
    F, G = (beta1 * a / s) ** 2, (beta1 * b / s) ** 2
    sv, ft, _ = orc.proj_svd(np.array([a]), np.array([beta1, b]))
    for omega in (0.5, 1.0, 1.3):
        one_m_phi = omega * G / ((2.0 - omega) * F)
        lam_ref = s * math.sqrt(one_m_phi / (1.0 - one_m_phi))
        lam, _, edge, _, _ = orc.choose_lambda_gcv(sv, ft, 200, omega=omega)
        assert not edge
        assert math.log(lam) == pytest.approx(math.log(lam_ref), abs=1e-6)


def test_weighted_gcv_reduces_to_gcv(orc):
    rng = np.random.default_rng(4)
    s = np.sort(rng.random(12))[::-1] + 0.01
    ft = rng.normal(size=13)
    for lam in (1e-3, 0.1, 0.7):
        assert orc.gcv_proj_weighted(s, ft, lam, 1.0) == orc.gcv_proj(s, ft, lam)
    assert orc.tsvd_gcv(s, ft, 3, 1.0) == orc.tsvd_gcv(s, ft, 3)


def test_last_lsqr_iterate_is_hkt_at_zero_lambda(orc):
    X, f, A, n_int, kappa, eps = _small_problem(orc, seed=21)
    ell = 15
    r_lsqr = orc.solve(X, n_int, kappa, eps, f, ell, method=orc.METHOD_LSQR, rule=orc.RULE_FIXED, k_trunc=ell)
    r_hkt = orc.solve(X, n_int, kappa, eps, f, ell, method=orc.METHOD_HKT, rule=orc.RULE_FIXED, lambda_fixed=0.0)
    assert r_lsqr.k == ell
    assert np.linalg.norm(r_lsqr.coef - r_hkt.coef) <= 1e-8 * np.linalg.norm(r_hkt.coef)


def test_lsqr_solve_rules(orc):
    X, f, A, n_int, kappa, eps = _small_problem(orc, seed=25)
    ell = 24
    n = X.shape[0]
    r = orc.solve(X, n_int, kappa, eps, f, ell, method=orc.METHOD_LSQR, rule=orc.RULE_GCV)
    rho, eta, _ = orc.lsqr_path(r.alpha, r.beta)
    G = rho ** 2 / (n - np.arange(1, ell + 1)) ** 2
    assert r.k == 1 + int(np.argmin(G))
    assert r.resid_norm == rho[r.k - 1] and r.sol_norm == eta[r.k - 1]
    r2 = orc.solve(X, n_int, kappa, eps, f, ell, method=orc.METHOD_LSQR, rule=orc.RULE_LCURVE)
    assert 1 <= r2.k <= ell
