"""GPU parity of the row-scaled operator D A, D = diag(A)^-1 (opt-in; not in the paper).

The row scaling divides the interior rows of the stacked system (eq. (11)) by
3 eps^2 + kappa^2 (the value of L phi at r = 0) and leaves the boundary rows
(phi(0) = 1) as they are; the method then runs on (D A) c = D f.  The library
folds D into the interior rows' entry constants, so no pass over A is added;
the oracle scales each entry (or the rows of its stored matrix) by d_i.

Tolerances as for the unscaled operator: FP64 entries 4e-15, products 1e-13
of (|D A||x|)_i; FP32-evaluated entries and products 4e-6; leading Ritz
values 1e-12; lambda* 1e-6; u at the oracle's lambda 1e-8.
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


def _problem(mq, p, mode):
    say("create", p.name, "mode", mode, "n", p.n)
    return mq.Problem(p.x_int, p.x_bnd, p.kappa, p.eps, mode)


RAGGED = lambda: I.cube_scaled(333, 190, kappa=6.0, eps=2.0, ell=40)  # noqa: E731


@pytest.mark.parametrize("mode", ["stored_fp64", "matfree_fp64", "matfree_fp32"])
def test_rs_entries(mq, orc, mode):
    p = RAGGED()
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    DA = A * orc.row_scale(p.nodes, p.n_int, p.kappa, p.eps)[:, None]
    with _problem(mq, p, mode) as pr:
        say("matrix rows, row scale", mode)
        R = pr.matrix_rows(0, p.n, row_scale=1)
        R0 = pr.matrix_rows(0, p.n)  # and back to the unscaled operator
    tol = 4e-6 if mode == "matfree_fp32" else 4e-15
    assert np.all(np.abs(R - DA) <= tol * np.abs(DA)), float(np.max(np.abs(R - DA) / np.abs(DA)))
    assert np.all(np.abs(R0 - A) <= tol * np.abs(A))


@pytest.mark.parametrize("mode", ["stored_fp64", "matfree_fp64", "matfree_fp32"])
def test_rs_products(mq, orc, mode):
    p = RAGGED()
    d = orc.row_scale(p.nodes, p.n_int, p.kappa, p.eps)
    DA = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps) * d[:, None]
    x = I.random_vector(p.n, 31)
    z = I.random_vector(p.n, 32)
    tol = 4e-6 if mode == "matfree_fp32" else 1e-13
    with _problem(mq, p, mode) as pr:
        for trans in (False, True):
            say("apply, row scale", mode, "trans", trans)
            y = pr.apply(x, trans=trans, shift=0.25, z=z, row_scale=1)
            ref = orc.apply(None, p.nodes, p.n_int, p.kappa, p.eps, x, trans=trans, d=d) - 0.25 * z
            scale = (np.abs(DA.T) if trans else np.abs(DA)) @ np.abs(x) + 0.25 * np.abs(z)
            err = np.abs(y - ref) / scale
            assert np.all(err <= tol), float(err.max())


def _solve_both(mq, orc, p, mode, **kw):
    r = orc.solve(p.nodes, p.n_int, p.kappa, p.eps, p.rhs, p.ell, stored=False, row_scale=1, **kw)
    with _problem(mq, p, mode) as pr:
        say("solve, row scale", p.name, mode, kw)
        out = pr.solve(p.f_int, p.g_bnd, p.ell, row_scale=1, **kw)
        u = pr.eval(out.coef, p.x_eval)
    uo = orc.eval_u(p.nodes, p.eps, r.coef, p.x_eval)
    return r, out, u, uo


SOLVE_CASES = [
    ("cube_n1800", I.cube_small),
    ("cube_interior_lambda", lambda: I.cube_scaled(400, 240, kappa=3.0, eps=0.7, ell=80)),
]


@pytest.mark.parametrize("name,make", SOLVE_CASES)
@pytest.mark.parametrize("mode", ["stored_fp64", "matfree_fp64"])
def test_rs_solve_hkt(mq, orc, name, make, mode):
    p = make()
    r, out, u, uo = _solve_both(mq, orc, p, mode)
    assert out.ell_done == r.ell
    assert np.max(np.abs(out.sv[:10] - r.s[:10]) / r.s[:10]) < 1e-12
    assert out.lam == pytest.approx(r.lam, rel=1e-6)
    assert bool(out.flags & mq.MQH_INFO_GCV_AT_EDGE) == bool(r.flags & orc.FLAG_GCV_AT_EDGE)
    r2, out2, u2, uo2 = _solve_both(mq, orc, p, mode, rule=mq.MQH_RULE_FIXED, lambda_fixed=r.lam)
    assert np.linalg.norm(u2 - uo2) <= 1e-8 * np.linalg.norm(uo2)
    assert np.linalg.norm(out2.coef - r2.coef) <= 1e-6 * np.linalg.norm(r2.coef)
    assert out2.resid_norm == pytest.approx(r2.resid_norm, rel=1e-9)


def test_rs_solve_ine_tsvd(mq, orc):
    p = I.cube_scaled(400, 240, kappa=3.0, eps=0.7, ell=80)
    r, out, u, uo = _solve_both(mq, orc, p, "matfree_fp64", method=mq.MQH_METHOD_INE_TSVD)
    assert out.k == r.k
    assert np.linalg.norm(u - uo) <= 1e-8 * np.linalg.norm(uo)


def test_rs_solve_fp32_entries(mq, orc):
    # as for the unscaled operator: FP32 entries move a Tikhonov solution at
    # lambda = 1e-3 s_1 by about 1e-3 relative
    p = I.cube_scaled(400, 240, kappa=3.0, eps=0.7, ell=80)
    s1 = orc.solve(p.nodes, p.n_int, p.kappa, p.eps, p.rhs, p.ell, stored=False, row_scale=1).s[0]
    r, out, u, uo = _solve_both(mq, orc, p, "matfree_fp32", rule=mq.MQH_RULE_FIXED, lambda_fixed=1e-3 * s1)
    assert np.linalg.norm(u - uo) <= 1e-3 * np.linalg.norm(uo)


def test_rs_stored_switch_reassembles(mq):
    # a stored problem alternating the scaling gives what fresh problems give, bit for bit
    p = I.cube_scaled(300, 200, kappa=5.0, eps=2.0, ell=30)
    with _problem(mq, p, "stored_fp64") as pr:
        say("stored switch 1, 0, 1")
        a1 = pr.solve(p.f_int, p.g_bnd, p.ell, row_scale=1)
        a0 = pr.solve(p.f_int, p.g_bnd, p.ell, row_scale=0)
        b1 = pr.solve(p.f_int, p.g_bnd, p.ell, row_scale=1)
        y0 = pr.apply(p.rhs)
    with _problem(mq, p, "stored_fp64") as pr:
        f0 = pr.solve(p.f_int, p.g_bnd, p.ell)
    with _problem(mq, p, "stored_fp64") as pr:
        f1 = pr.solve(p.f_int, p.g_bnd, p.ell, row_scale=1)
    assert np.array_equal(a1.coef, f1.coef) and np.array_equal(b1.coef, f1.coef)
    assert np.array_equal(a0.coef, f0.coef)
    assert not np.array_equal(a0.coef, a1.coef)
    with _problem(mq, p, "matfree_fp64") as pr:
        ym = pr.apply(p.rhs)
    assert np.max(np.abs(y0 - ym) / np.abs(ym)) < 1e-12


@pytest.mark.parametrize("mode", ["stored_fp64", "matfree_fp64", "matfree_fp32"])
def test_rs_multi_matches_single(mq, orc, mode):
    # lockstep runs with the row scaling: FP64 runs equal the single solve bit
    # for bit; FP32 block products agree with the oracle at a fixed lambda
    mp = I.multi_cube(300, 180, kappa=5.0, eps=1.5, nrhs=5, ell=30, seed=3)
    F = mp.F
    with mq.Problem(mp.x_int, mp.x_bnd, mp.kappa, mp.eps, mode, fixed_shapes=True) as pr:
        say("multi solve, row scale", mode)
        if mode == "matfree_fp32":
            s1 = orc.solve(mp.nodes, mp.n_int, mp.kappa, mp.eps, F[0], mp.ell, stored=False, row_scale=1).s[0]
            lam = 1e-3 * s1
            out = pr.solve_multi(F, mp.ell, rule=mq.MQH_RULE_FIXED, lambda_fixed=lam, row_scale=1)
            xe = I.random_nodes_cube(500, 99)
            for k in (0, 4):
                r = orc.solve(mp.nodes, mp.n_int, mp.kappa, mp.eps, F[k], mp.ell, stored=False,
                              rule=orc.RULE_FIXED, lambda_fixed=lam, row_scale=1)
                u = orc.eval_u(mp.nodes, mp.eps, out.coef[k], xe)
                uo = orc.eval_u(mp.nodes, mp.eps, r.coef, xe)
                assert np.linalg.norm(u - uo) <= 1e-3 * np.linalg.norm(uo)
        else:
            out = pr.solve_multi(F, mp.ell, row_scale=1)
            for k in (0, 3):
                one = pr.solve(F[k][:mp.n_int].copy(), F[k][mp.n_int:].copy(), mp.ell, row_scale=1)
                assert np.array_equal(one.coef, out.coef[k]) and one.lam == out.lam[k]


def test_rs_rejected_where_unsupported(mq):
    p = I.cube_scaled(200, 100, kappa=4.0, eps=2.0, ell=10)
    F = np.stack([p.rhs, p.rhs[::-1].copy()])
    with _problem(mq, p, "matfree_fp64") as pr:
        say("row scale rejections")
        opts = mq.mqh_solve_opts(ell=5, reorth=1, method=mq.MQH_METHOD_HKT, rule=mq.MQH_RULE_GCV, row_scale=1)
        coef = np.zeros((2, p.n))
        assert mq.lib.mqh_solve_block(pr.h, F.ctypes.data, p.n, 2, opts, coef.ctypes.data, p.n, None, None) == \
            mq.MQH_EINVAL
        assert "row_scale" in mq.mqh_last_error()
        assert mq.lib.mqh_full_solve(pr.h, p.f_int.ctypes.data, p.g_bnd.ctypes.data, opts, coef.ctypes.data, None,
                                     None) == mq.MQH_EINVAL
        opts.row_scale = 2
        assert mq.lib.mqh_solve(pr.h, p.f_int.ctypes.data, p.g_bnd.ctypes.data, opts, coef.ctypes.data, None, None,
                                None, None) == mq.MQH_EINVAL
        # the problem still solves unscaled afterwards
        out = pr.solve(p.f_int, p.g_bnd, p.ell)
        assert np.all(np.isfinite(out.coef))
