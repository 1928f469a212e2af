"""GPU parity of the full-SVD reference path (one-sided block Jacobi on the
rows of [A | f]; Algorithm 3 and the TSVD solution of eq. (14)) against the
FP64 oracle.

Tolerances.  The Jacobi process stops when every pair of rows has the
component of the smaller along the larger at most tol ||A||_F, tol =
16 sqrt(n) eps; the singular values (row norms) then carry absolute errors
of a small multiple of that level (measured: 2.7x at 523 nodes, 6.8x at
1 800), so the bars below use tau = 8 tol ||A||_F:
* singular values: all of them within tau of LAPACK's; the leading ten to
  4 n eps sigma_1 (rows of large norm are orthogonal to far more than tol);
* U^T f: sum of squares = ||f||^2 to 16 n eps relative (the f column passes
  through sweeps x rounds computed 64 x 64 orthogonal factors, each
  orthogonal to a few ulps); magnitudes of the components of singular values
  separated from their neighbours by more than 1e-6 sigma_1 to 1e-8 ||f||
  (a component moves by about eps sigma_1 / gap);
* the parameter choice as a step of its own: lambda (Tikhonov) and the rank
  (TSVD) equal the oracle's rules applied to the GPU's own sigma and U^T f, to
  1e-5 relative (the GCV minimum is flat: its relative curvature in log lambda
  is ~0.1, so rounding at 1e-13 fixes the argmin to ~1e-6) and exactly;
* the choices and solutions end to end against the oracle's LAPACK SVD, on
  data with seeded noise of 1e-2 relative, with bars from the oracle's own
  sensitivity to a backward error (the oracle on A + E, E random, at 1 800
  nodes, where tau = 5 500 eps sigma_1; 8 draws per size): ||E|| = 3 000
  eps sigma_1 moves lambda by up to 3.4e-3 and GCV at it by up to 1.1e-6,
  ||E|| = 10 000 eps sigma_1 by up to 1.7e-2 and 2.8e-5; the rank stays, u
  moves by about 1e-5 and the residual norm by 1e-4.  Bars: GCV within 1e-5
  of the minimum and lambda to 1e-2 (the sensitivity at a backward error of
  about tau: GCV grows with ||E|| to about the 2.7th power between the two
  draws, ~5e-6 at 5 500 eps sigma_1; measured 4.0e-6 and 6.3e-3, and 3.7e-7
  and 1.9e-3 with FP64 entries whose rsqrt rounded some entries the other way
  by one ulp), the TSVD rank exactly (the runner-up's GCV lies 3e-3 above the
  minimum), u at the oracle's lambda or rank to 1e-4, coefficients to
  tau / lambda (Tikhonov) or tau / sigma_k (TSVD), the first-order
  amplification of a backward error, and ||A x - f|| to 1e-3.
  With exact (manufactured) data, or little noise, GCV on these square
  systems takes its minimum near the rounding level, where the choice is not a
  property of the problem; at 1e-2 noise it is.
At the full 20 000-node cube (in the launch configuration of the benchmark)
the Tikhonov solution is checked against the normal equations
(A^T A + lambda^2 I) x = A^T f with the oracle's own FP64 products.  n above
MQH_FULL_MAX_N is rejected.
"""
import sys

import numpy as np
import pytest

from paper_2511_09798_amd import inputs as I

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mq():
    from paper_2511_09798_amd import mqhelm

    return mqhelm


CASES = [
    ("cube_523", lambda: I.cube_scaled(333, 190, kappa=6.0, eps=2.0, ell=40)),
    ("cube_n1800", I.cube_small),
]


def _noisy(p, level=1e-2, seed=17):
    f = p.rhs
    e = np.random.default_rng(seed).standard_normal(p.n)
    g = f + level * np.linalg.norm(f) / np.linalg.norm(e) * e
    return g, np.ascontiguousarray(g[:p.n_int]), np.ascontiguousarray(g[p.n_int:])


def _problem(mq, p, mode="stored_fp64"):
    say("create", p.name, "n", p.n)
    return mq.Problem(p.x_int, p.x_bnd, p.kappa, p.eps, mode)


@pytest.mark.parametrize("name,make", CASES)
def test_full_svd_against_oracle(mq, orc, name, make):
    p = make()
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    U, s, V = orc.full_svd(A)
    f = p.rhs
    fo = U.T @ f
    with _problem(mq, p, "matfree_fp32") as pr:  # the reference path assembles FP64 whatever the mode
        say("full svd", name)
        r = pr.full_svd(f)
    assert r["status"] == 0, r
    sv, fh = r["sv"], r["fhat"]
    say("sweeps", r["sweeps"], "off", r["off"], "max |dsigma| / (eps sigma_1)", np.max(np.abs(sv - s)) / (EPS * s[0]))
    assert np.all(np.diff(sv) <= 0)
    assert np.max(np.abs(sv[:10] - s[:10])) <= 4 * p.n * EPS * s[0]
    assert np.max(np.abs(sv - s)) <= _tau(A)
    assert float(fh @ fh) == pytest.approx(float(f @ f), rel=16 * p.n * EPS)
    gap = np.minimum(np.abs(np.diff(np.r_[np.inf, s])), np.abs(np.diff(np.r_[s, -np.inf]))) / s[0]
    sep = gap > 1e-6
    assert sep.sum() >= 5
    assert np.max(np.abs(np.abs(fh[sep]) - np.abs(fo[sep]))) <= 1e-8 * np.linalg.norm(f)


def _tau(A):
    # 8 x the convergence level of the rows' orthogonality, absolute
    return 8 * 16 * np.sqrt(A.shape[0]) * EPS * np.linalg.norm(A)


def _oracle_svd(orc, p, f):
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    U, s, V = orc.full_svd(A)
    fo = U.T @ f
    return A, s, V, fo, max(0.0, float(f @ f) - float(fo @ fo))


def _gpu_choice_inputs(pr, f):
    r = pr.full_svd(f)
    assert r["status"] == 0, r
    sv, fh = r["sv"], r["fhat"]
    return sv, fh, max(0.0, float(f @ f) - float(fh @ fh))


@pytest.mark.parametrize("name,make", CASES)
def test_full_tikhonov_against_oracle(mq, orc, name, make):
    p = make()
    f, fi, gb = _noisy(p)
    A, s, V, fo, spo = _oracle_svd(orc, p, f)
    lam_o = orc.choose_lambda_full(s, fo, spo, p.n)
    alpha_o = V @ (s / (s * s + lam_o * lam_o) * fo)
    with _problem(mq, p) as pr:
        say("full tikhonov gcv", name)
        out = pr.full_solve(fi, gb, method=mq.MQH_METHOD_HKT)
        say("choice inputs", name)
        sv, fh, sp = _gpu_choice_inputs(pr, f)
        say("full tikhonov fixed", name, lam_o)
        out2 = pr.full_solve(fi, gb, method=mq.MQH_METHOD_HKT, rule=mq.MQH_RULE_FIXED, lambda_fixed=lam_o)
        u = pr.eval(out2.coef, p.x_eval)
    uo = orc.eval_u(p.nodes, p.eps, alpha_o, p.x_eval)
    g_o = orc.gcv_full(s, fo, spo, p.n, lam_o)
    du = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    dc = np.linalg.norm(out2.coef - alpha_o) / np.linalg.norm(alpha_o)
    say("lambda", out.lam, "oracle", lam_o, "gcv ratio", orc.gcv_full(s, fo, spo, p.n, out.lam) / g_o,
        "u", du, "coef", dc, "sdiff/(eps s1)", np.max(np.abs(sv - s)) / (EPS * s[0]),
        "above lambda", np.max(np.abs(sv - s)[s >= lam_o]) / (EPS * s[0]), "cg iterations", out2.t_ms[7])
    # the choice step on the GPU's own SVD
    assert out.lam == pytest.approx(orc.choose_lambda_full(sv, fh, sp, p.n), rel=1e-5)
    # end to end against the oracle's SVD
    assert orc.gcv_full(s, fo, spo, p.n, out.lam) <= g_o * (1.0 + 1e-5)
    assert out.lam == pytest.approx(lam_o, rel=1e-2)
    assert du <= 1e-4
    assert dc <= _tau(A) / lam_o
    assert not (out.flags & mq.MQH_INFO_SOLVE_NOCONV) and not (out2.flags & mq.MQH_INFO_SOLVE_NOCONV)
    # residual and solution norms of the returned coefficients (||G x - Q f|| and ||x||)
    say("resid", out2.resid_norm, "oracle", np.linalg.norm(A @ alpha_o - f), "of the GPU's coef",
        np.linalg.norm(A @ out2.coef - f))
    assert out2.resid_norm == pytest.approx(np.linalg.norm(A @ out2.coef - f), rel=1e-3)
    assert out2.resid_norm == pytest.approx(np.linalg.norm(A @ alpha_o - f), rel=1e-3)
    assert out2.sol_norm == pytest.approx(np.linalg.norm(out2.coef), rel=1e-12)


@pytest.mark.parametrize("name,make", CASES)
def test_full_tsvd_against_oracle(mq, orc, name, make):
    p = make()
    f, fi, gb = _noisy(p)
    A, s, V, fo, spo = _oracle_svd(orc, p, f)
    k_o = orc.choose_rank_full(s, fo, spo, p.n)
    alpha_o = V[:, :k_o] @ (fo[:k_o] / s[:k_o])
    with _problem(mq, p) as pr:
        say("full tsvd gcv", name)
        out = pr.full_solve(fi, gb, method=mq.MQH_METHOD_INE_TSVD)
        say("choice inputs", name)
        sv, fh, sp = _gpu_choice_inputs(pr, f)
        say("full tsvd fixed", name, k_o)
        out2 = pr.full_solve(fi, gb, method=mq.MQH_METHOD_INE_TSVD, rule=mq.MQH_RULE_FIXED, k_trunc=k_o)
        u = pr.eval(out2.coef, p.x_eval)
    uo = orc.eval_u(p.nodes, p.eps, alpha_o, p.x_eval)
    du = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    dc = np.linalg.norm(out2.coef - alpha_o) / np.linalg.norm(alpha_o)
    say("k", out.k, "oracle", k_o, "u", du, "coef", dc)
    assert out.k == orc.choose_rank_full(sv, fh, sp, p.n)
    assert out.k == k_o
    assert du <= 1e-4
    assert dc <= _tau(A) / s[k_o - 1]


def test_full_exact_data_reports_the_solution_state(mq, orc):
    # exact (manufactured) data: GCV may put lambda below the accuracy of any
    # backward-stable SVD, where the dual system's iteration need not reach its
    # tolerance; the call then says so (flag, warning status, iterations at the
    # cap) and still returns finite coefficients
    p = I.cube_small()
    with _problem(mq, p) as pr:
        say("full tikhonov exact data", p.name)
        out = pr.full_solve(p.f_int, p.g_bnd, method=mq.MQH_METHOD_HKT)
    say("status", out.status, "flags", out.flags, "cg iterations", out.t_ms[7], "lambda", out.lam)
    flagged = bool(out.flags & mq.MQH_INFO_SOLVE_NOCONV)
    if flagged:
        assert out.t_ms[7] == mq.MQH_FULL_CG_MAX and out.status == mq.MQH_WNOCONV
    if out.t_ms[7] < mq.MQH_FULL_CG_MAX:
        assert not flagged
    assert np.all(np.isfinite(out.coef))


def test_full_small_and_invalid(mq, orc):
    # n below one block (padding rows), and argument errors
    X = I.random_nodes_cube(21, 4)
    f = I.random_vector(21, 5)
    A = orc.assemble(X, 14, 2.0, 1.5)
    with mq.Problem(X[:14], X[14:], 2.0, 1.5, "matfree_fp64") as pr:
        say("full svd n = 21")
        r = pr.full_svd(f)
        s = np.linalg.svd(A, compute_uv=False)
        assert np.max(np.abs(r["sv"] - s)) <= 64 * 21 * EPS * s[0]
        with pytest.raises(mq.MQHError):
            pr.full_solve(f[:14], f[14:], method=mq.MQH_METHOD_LSQR)
        with pytest.raises(mq.MQHError):
            pr.full_solve(f[:14], f[14:], rule=mq.MQH_RULE_LCURVE)
        with pytest.raises(mq.MQHError):
            pr.full_solve(f[:14], f[14:], method=mq.MQH_METHOD_INE_TSVD, rule=mq.MQH_RULE_FIXED, k_trunc=0)


def test_full_deterministic(mq):
    # fixed-order reductions and a fixed schedule: a repeated call returns the same bits
    p = I.cube_scaled(333, 190, kappa=6.0, eps=2.0, ell=40)
    f, fi, gb = _noisy(p)
    with _problem(mq, p) as pr:
        say("full determinism")
        a = pr.full_solve(fi, gb)
        b = pr.full_solve(fi, gb)
    assert np.array_equal(a.coef, b.coef) and a.lam == b.lam and np.array_equal(a.sv, b.sv)


def test_full_size_limit(mq):
    # n = MQH_FULL_MAX_N + 1 is rejected before anything of size n^2 is allocated
    n = mq.MQH_FULL_MAX_N + 1
    X = I.random_nodes_cube(n, 32)
    f = I.random_vector(n, 33)
    with mq.Problem(X[:n - 4000], X[n - 4000:], 2.0, 1.5, "matfree_fp32") as pr:
        say("full svd n", n, "rejected")
        with pytest.raises(mq.MQHError):
            pr.full_svd(f)
        with pytest.raises(mq.MQHError):
            pr.full_solve(f[:n - 4000], f[n - 4000:])


def test_full_size_cube_normal_equations(mq, orc):
    # 20 000-node cube, data with 1e-2 noise: Algorithm 3 on the GPU.  A
    # backward error E of the SVD (||E|| <= tau sigma_1, tau = 8 sqrt(T) eps
    # for T = sweeps x rounds transforms per row, doubled for safety) leaves
    # the computed x the Tikhonov solution for A + E, so with the oracle's FP64
    # products: ||A^T (A x - f) + lambda^2 x|| <= 2 tau sigma_1 (sigma_1 ||x|| + ||f||)
    # (first order), and the reported residual norm is ||A x - f|| up to
    # tau sigma_1 ||x||; sigma_1 agrees with the leading Ritz value of a
    # 60-step Golub-Kahan run.
    p = I.cube_medium()
    f, fi, gb = _noisy(p)
    with _problem(mq, p) as pr:
        say("full tikhonov n = 20000")
        out = pr.full_solve(fi, gb, method=mq.MQH_METHOD_HKT)
        say("sweeps", out.ell_done, "off", out.t_ms[6], "lambda", out.lam, "t_ms", out.t_ms)
        assert out.status == 0
        g = pr.gkb(f, 60)
    x, lam = out.coef, out.lam
    s1 = out.sv[0]
    rounds = 2 * ((p.n + 63) // 64) - 1
    tau = 2 * 8 * np.sqrt(out.ell_done * rounds) * EPS
    say("oracle products")
    Ax = orc.apply(None, p.nodes, p.n_int, p.kappa, p.eps, x)
    lhs = orc.apply(None, p.nodes, p.n_int, p.kappa, p.eps, Ax - f, trans=True) + lam * lam * x
    nx, nf = np.linalg.norm(x), np.linalg.norm(f)
    bound = 2 * tau * s1 * (s1 * nx + nf)
    say("normal-equation residual", np.linalg.norm(lhs), "bound", bound, "lambda/s1", lam / s1,
        "resid", np.linalg.norm(Ax - f), "reported", out.resid_norm)
    assert np.linalg.norm(lhs) <= bound
    assert abs(np.linalg.norm(Ax - f) - out.resid_norm) <= tau * s1 * nx + 1e-10 * nf
    C = orc.bidiag_matrix(g["alpha"], g["beta"])
    assert s1 == pytest.approx(np.linalg.svd(C, compute_uv=False)[0], rel=1e-10)
