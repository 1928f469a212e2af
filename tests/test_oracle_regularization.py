"""Pins for the projected regularisation steps (Sections 3.2-3.3, Algorithms 2-4).

* filter factors: phi_i = 1/2 at lambda = s_i; the SVD-form projected
  Tikhonov solution against the stacked least-squares problem
  [C; lambda I] y ~ [beta_1 e_1; 0] solved by LAPACK; rho_l^2 and eta_l^2
  against the residual and norm of that solution computed directly; the
  trace of the explicit hat matrix against sum phi_i (eqs. (28), (29), (30));
* limits: lambda -> 0 gives the least-squares solution C^+ beta_1 e_1 and
  GCV_l(0) = f~_{l+1}^2; lambda -> inf gives lambda^2 y -> C^T beta_1 e_1
  and GCV_l(inf) = beta_1^2/(l+1)^2;
* reduction to the textbook methods at l = N: HKT at fixed lambda equals
  full Tikhonov (eq. (17)) and Ine-TSVD at rank k equals TSVD
  (eq. (14)), the full ones computed by LAPACK's SVD;
* GCV minimiser: closed form for l = 1, brute-force dense scan otherwise;
* L-curve: analytic curvature against finite differences of
  (log rho, log eta) in log lambda; corner near the noise level of
  synthetic data that satisfy the discrete Picard condition;
* Tikhonov with duplicate nodes (singular A): finite and unique (SVD form
  and normal equations agree, Section 4.2 existence proposition).
"""
import math

import numpy as np
import pytest

from paper_2511_09798_amd import inputs as I


@pytest.fixture(scope="module")
def proj(orc):
    p = I.cube_scaled(150, 90, kappa=6.0, eps=2.0, ell=25)
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    g = orc.gkb(A, p.nodes, p.n_int, p.kappa, p.eps, p.rhs, p.ell)
    s, ft, V = orc.proj_svd(g.alpha, g.beta)
    C = orc.bidiag_matrix(g.alpha, g.beta)
    return p, A, g, s, ft, V, C


def test_filter_half_at_singular_value(orc, proj):
    *_, s, ft, V, C = proj
    for i in (0, 5, len(s) - 1):
        assert orc.tikh_filter(s, s[i])[i] == pytest.approx(0.5, rel=1e-15)
        assert orc.tikh_filter_complement(s, s[i])[i] == pytest.approx(0.5, rel=1e-15)


@pytest.mark.parametrize("which", [0, 3, 10])
def test_projected_tikhonov_against_stacked_lstsq(orc, proj, which):
    p, A, g, s, ft, V, C = proj
    lam = float(s[which])
    ell = g.ell
    y = orc.y_tikhonov(s, ft, V, lam)
    rhs = np.zeros(2 * ell + 1)
    rhs[0] = g.beta[0]
    M = np.vstack([C, lam * np.eye(ell)])
    y_ls = np.linalg.lstsq(M, rhs, rcond=None)[0]
    assert np.linalg.norm(y - y_ls) <= 1e-10 * np.linalg.norm(y_ls)
    e1 = np.zeros(ell + 1)
    e1[0] = g.beta[0]
    assert orc.rho2_proj(s, ft, lam) == pytest.approx(np.linalg.norm(C @ y - e1) ** 2, rel=1e-9)
    assert orc.eta2_proj(s, ft, lam) == pytest.approx(np.linalg.norm(y) ** 2, rel=1e-10)
    H = C @ np.linalg.solve(C.T @ C + lam * lam * np.eye(ell), C.T)
    assert np.trace(H) == pytest.approx(float(np.sum(orc.tikh_filter(s, lam))), rel=1e-10)
    gcv_direct = np.linalg.norm((np.eye(ell + 1) - H) @ e1) ** 2 / (ell + 1 - np.trace(H)) ** 2
    assert orc.gcv_proj(s, ft, lam) == pytest.approx(gcv_direct, rel=1e-8)


def test_limits(orc, proj):
    p, A, g, s, ft, V, C = proj
    ell = g.ell
    e1 = np.zeros(ell + 1)
    e1[0] = g.beta[0]
    y0 = orc.y_tikhonov(s, ft, V, 0.0)
    y_ls = np.linalg.lstsq(C, e1, rcond=None)[0]
    assert np.linalg.norm(y0 - y_ls) <= 1e-8 * np.linalg.norm(y_ls)
    assert orc.gcv_proj(s, ft, 0.0) == pytest.approx(ft[ell] ** 2, rel=1e-12)
    big = 1e100
    assert np.allclose(big * big * orc.y_tikhonov(s, ft, V, big), C.T @ e1, rtol=1e-12,
                       atol=1e-12 * np.linalg.norm(C.T @ e1))
    assert orc.gcv_proj(s, ft, big) == pytest.approx(g.beta[0] ** 2 / (ell + 1) ** 2, rel=1e-12)


def test_tsvd_solution_against_projected_lstsq(orc, proj):
    p, A, g, s, ft, V, C = proj
    ell = g.ell
    Uf, sf, Vtf = np.linalg.svd(C, full_matrices=False)
    e1 = np.zeros(ell + 1)
    e1[0] = g.beta[0]
    for k in (1, 4, ell):
        yk = orc.y_tsvd(s, ft, V, k)
        ref = Vtf[:k].T @ ((Uf[:, :k].T @ e1) / sf[:k])
        assert np.linalg.norm(yk - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("n", [16, 32])
def test_full_dimension_reduces_to_textbook_methods(orc, n):
    X = I.random_nodes_cube(n, 200 + n)
    n_int = n // 2
    kappa, eps = 2.0, 6.0
    A = orc.assemble(X, n_int, kappa, eps)
    f = I.random_vector(n, 300 + n)
    g = orc.gkb(A, X, n_int, kappa, eps, f, n)
    assert g.ell == n
    s, ft, V = orc.proj_svd(g.alpha, g.beta)
    for lam in (1e-3 * s[0], 1e-1 * s[0], s[n // 2]):
        coef = orc.lift(g.Z, orc.y_tikhonov(s, ft, V, lam))
        ref = orc.full_tikhonov(A, f, lam)
        assert np.linalg.norm(coef - ref) <= 1e-10 * np.linalg.norm(ref)
    for k in (1, 3, n // 2, n):
        coef = orc.lift(g.Z, orc.y_tsvd(s, ft, V, k))
        ref = orc.full_tsvd(A, f, k)
        assert np.linalg.norm(coef - ref) <= 1e-10 * np.linalg.norm(ref)


def test_gcv_minimiser_closed_form_ell1(orc):
    # l = 1: C = [a; b], s = sqrt(a^2+b^2), f~ = beta_1 (a, b)/s.  With
    # psi = 1 - phi = lambda^2/(s^2+lambda^2), GCV = (psi^2 f1^2 + f2^2)/(1+psi)^2,
    # whose derivative 2(psi f1^2 - f2^2)/(1+psi)^3 vanishes at psi = f2^2/f1^2,
    # i.e. lambda*^2 = s^2 b^2 / (a^2 - b^2).
    a, b = 3.0, 1.0
    s, ft, V = orc.proj_svd(np.array([a]), np.array([2.0, b]))
    lam, gmin, edge, grid, vals = orc.choose_lambda_gcv(s, ft, 200)
    expect = math.sqrt(10.0 * b * b / (a * a - b * b))
    assert not edge
    assert lam == pytest.approx(expect, rel=1e-7)


def test_gcv_minimiser_dense_scan(orc, proj):
    p, A, g, s, ft, V, C = proj
    lam, gmin, edge, grid, vals = orc.choose_lambda_gcv(s, ft, 200)
    fine = np.exp(np.linspace(math.log(grid[0]), math.log(grid[-1]), 200001))
    fv = np.array([orc.gcv_proj(s, ft, x) for x in fine])
    best = fine[int(np.argmin(fv))]
    if not edge:
        assert gmin <= fv.min() * (1 + 1e-12)
        assert lam == pytest.approx(best, rel=2e-3)
    else:
        assert lam in (grid[0], grid[-1])


def test_gcv_top_edge_when_projected_residual_large(orc):
    # GCV(inf) = beta_1^2/(l+1)^2 < GCV(0) = f~_{l+1}^2 whenever |f~_{l+1}|/beta_1 > 1/(l+1)
    p = I.cube_small()
    r = orc.solve(p.nodes, p.n_int, p.kappa, p.eps, p.rhs, p.ell)
    assert abs(r.ftil[-1]) / r.beta[0] > 1.0 / (r.ell + 1)
    assert r.flags & orc.FLAG_GCV_AT_EDGE
    assert r.lam == pytest.approx(r.s[0], rel=1e-12)


def _picard(ell=40, noise=1e-7, seed=4):
    rng = np.random.default_rng(seed)
    s = np.logspace(0, -8, ell)
    ft = np.empty(ell + 1)
    ft[:ell] = s ** 1.5 * np.sign(rng.normal(size=ell)) + noise * rng.normal(size=ell)
    ft[ell] = noise
    return s, ft


def test_lcurve_curvature_against_finite_differences(orc):
    s, ft = _picard()
    h = 1e-3

    def xy(t):
        lam = math.exp(t)
        return 0.5 * math.log(orc.rho2_proj(s, ft, lam)), 0.5 * math.log(orc.eta2_proj(s, ft, lam))

    for lam in (1e-7, 1e-5, 1e-3, 1e-1):
        t = math.log(lam)
        (xm, ym), (x0, y0), (xp, yp) = xy(t - h), xy(t), xy(t + h)
        x1, y1 = (xp - xm) / (2 * h), (yp - ym) / (2 * h)
        x2, y2 = (xp - 2 * x0 + xm) / (h * h), (yp - 2 * y0 + ym) / (h * h)
        kfd = (x1 * y2 - x2 * y1) / (x1 * x1 + y1 * y1) ** 1.5
        assert orc.lcurve_curvature(s, ft, lam) == pytest.approx(kfd, rel=1e-5, abs=1e-6)


def test_lcurve_corner_near_noise_level(orc):
    s, ft = _picard()
    lam, kap, edge, grid, kv = orc.choose_lambda_lcurve(s, ft, 200)
    assert not edge and kap > 0
    assert 1e-8 < lam < 1e-5  # noise level 1e-7: the corner sits within a decade or so


def test_tsvd_rank_obvious_case(orc):
    ell = 20
    s = np.logspace(0, -3, ell)
    ft = np.full(ell + 1, 1e-8)
    ft[:5] = 1.0
    assert orc.choose_rank(s, ft) == 5


def test_tikhonov_unique_with_duplicate_nodes(orc):
    X = I.random_nodes_cube(30, 44)
    X[7] = X[3]  # duplicate centre: two equal columns, A singular
    A = orc.assemble(X, 15, 3.0, 4.0)
    sv = np.linalg.svd(A, compute_uv=False)
    assert sv[-1] < 1e-12 * sv[0]
    f = I.random_vector(30, 45)
    lam = 1e-3 * sv[0]
    a1 = orc.full_tikhonov(A, f, lam)
    a2 = np.linalg.solve(A.T @ A + lam * lam * np.eye(30), A.T @ f)
    assert np.all(np.isfinite(a1))
    assert np.linalg.norm(a1 - a2) <= 1e-8 * np.linalg.norm(a1)
    # the two coefficients of the duplicated centre are equal (symmetric minimiser)
    assert a1[3] == pytest.approx(a1[7], rel=1e-8)
    # the projected path on the same singular matrix stays finite as well
    r = orc.solve(X, 15, 3.0, 4.0, f, 10)
    assert np.all(np.isfinite(r.coef))


def test_lift_is_matrix_product(orc, proj):
    p, A, g, s, ft, V, C = proj
    y = I.random_vector(g.ell, 9)
    assert np.allclose(orc.lift(g.Z, y), g.Z @ y, rtol=0, atol=1e-14 * np.abs(g.Z) @ np.abs(y))


def test_solve_end_to_end_small(orc):
    # Sanity only (the paper's accuracy figures cannot be reproduced without
    # its meshes and shape parameter): the three variants return finite
    # coefficients and HKT-GCV approximates the manufactured solution.
    p = I.cube_scaled(300, 150, kappa=3.0, eps=0.5, ell=150)
    r_h = orc.solve(p.nodes, p.n_int, p.kappa, p.eps, p.rhs, p.ell)
    r_t = orc.solve(p.nodes, p.n_int, p.kappa, p.eps, p.rhs, p.ell, method=orc.METHOD_INE_TSVD)
    r_l = orc.solve(p.nodes, p.n_int, p.kappa, p.eps, p.rhs, p.ell, rule=orc.RULE_LCURVE)
    errs = []
    for r in (r_h, r_t, r_l):
        assert np.all(np.isfinite(r.coef))
        u = orc.eval_u(p.nodes, p.eps, r.coef, p.x_eval)
        errs.append(orc.rel_l2(u, p.u_eval))
    assert errs[0] < 0.1 and max(errs) < 1.0
    assert 1 <= r_t.k <= p.ell // 2
    # a second run gives bit-identical output
    r2 = orc.solve(p.nodes, p.n_int, p.kappa, p.eps, p.rhs, p.ell)
    assert np.array_equal(r2.coef, r_h.coef)
