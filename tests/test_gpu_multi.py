"""GPU parity of the multi-right-hand-side path (lockstep Golub-Kahan runs
sharing each pass over A) against the FP64 oracle, run by run.

The method for several right-hand sides is one independent run of
Algorithm 1 (and of Algorithm 4 for the solve) per right-hand side, so the
oracle is the single-run oracle applied to each column.

Tolerances:
* FP64 forms and groups of one: the multi path performs, per run, exactly
  the operations of the single-run path (same kernels, same reduction
  orders), so its outputs are compared bit for bit with mqh_gkb / mqh_solve.
* Block products (FP32-evaluated entries; the contraction on the matrix
  cores with entries and vectors each split into two fp16 parts, 2^-22
  relative, products exact in FP32; FP32 sums over one 256-node chunk,
  FP64 across chunks and slices): |dy_i| <= 4e-6 (|A||x|)_i against the
  oracle, the bar of the single FP32 product (entries to ~1e-6 relative; a
  256-term FP32 sum adds at most ~256 u32 / 2 of its absolute sum in the
  worst case, ~1e-6 typically).
* Golub-Kahan scalars with FP32 entries: leading Ritz values to 1e-5
  relative, bases orthonormal to 1e-12 (reorthogonalisation stays FP64).
* Runs in a group do not interact: a run's outputs are bit-identical
  whichever runs share its group (each output column of a block product is
  its own dot products over the same entries).
"""
import sys

import numpy as np
import pytest

from paper_2511_09798_amd import inputs as I

pytestmark = pytest.mark.gpu


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


# ragged sizes: several 128-node blocks and 256-node chunks plus tails in both classes
RAGGED = [
    ("cube_523", lambda s: I.multi_cube(333, 190, 6.0, 2.0, s, 30, seed=5)),
    ("cube_1800", lambda s: I.multi_cube(1200, 600, 5.0, 2.0, s, 30, seed=9)),
]


def _scale_rows(orc, p, X, trans):
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    Aop = A.T if trans else A
    return Aop @ X.T, np.abs(Aop) @ np.abs(X.T)


# ---------------------------------------------------------------------------
# block products
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,make", RAGGED)
@pytest.mark.parametrize("nrhs", [2, 5, 16, 19])
@pytest.mark.parametrize("mode", ["matfree_fp32", "matfree_fp64"])
def test_apply_multi_against_oracle(mq, orc, name, make, nrhs, mode):
    p = make(nrhs)
    rng = np.random.default_rng(nrhs)
    X = rng.standard_normal((nrhs, p.n))
    Zs = rng.standard_normal((nrhs, p.n))
    shifts = rng.standard_normal(nrhs)
    tol = 4e-6 if mode == "matfree_fp32" else 1e-13
    with _problem(mq, p, mode) as pr:
        for trans in (False, True):
            say("apply_multi", name, nrhs, mode, "trans", trans)
            Y = pr.apply_multi(X, trans=trans)
            ref, scale = _scale_rows(orc, p, X, trans)
            err = np.abs(Y.T - ref) / scale
            assert np.all(err <= tol), float(err.max())
            say("apply_multi shifted", name, nrhs, mode, "trans", trans)
            Y2 = pr.apply_multi(X, trans=trans, shifts=shifts, Z=Zs)
            ref2 = ref - shifts[None, :] * Zs.T
            scale2 = scale + np.abs(shifts[None, :] * Zs.T)
            err2 = np.abs(Y2.T - ref2) / scale2
            assert np.all(err2 <= tol), float(err2.max())


def test_apply_multi_full_size_sampled(mq, orc):
    # the sweep's largest shapes in the benchmark's mode: the 20 596-node and 29 619-node members,
    # 16 vectors, FP32-evaluated block products; 64 sampled outputs of A X and A^T X per vector
    # against the oracle's FP64 entries one by one, to the bar of the small cases relative to
    # |A| |x| (every entry of A is positive, so |A| |x| = A |x|, computed the same way)
    for k in (0, int(np.argmax(I.sweep_sizes()))):
        m = I.sweep_member(k)
        X = np.vstack([m.x_int, m.x_bnd])
        n, n_int = X.shape[0], m.x_int.shape[0]
        V = np.random.default_rng(20 + k).standard_normal((16, n))
        rows = np.random.default_rng(30 + k).choice(n, 64, replace=False)
        with mq.Problem(m.x_int, m.x_bnd, m.kappa, m.eps, "matfree_fp32") as pr:
            for trans in (False, True):
                say("apply_multi full size n", n, "trans", trans)
                Y = pr.apply_multi(V, trans=trans)
                for q in range(16):
                    ref = orc.apply_sampled(X, n_int, m.kappa, m.eps, V[q], rows, trans=trans)
                    scale = orc.apply_sampled(X, n_int, m.kappa, m.eps, np.abs(V[q]), rows, trans=trans)
                    err = np.abs(Y[q][rows] - ref) / scale
                    assert np.all(err <= 4e-6), (k, trans, q, float(err.max()))


def test_apply_multi_columns_independent(mq):
    # a column's block product does not depend on the other columns of its group
    p = I.multi_cube(700, 300, 4.0, 1.5, 16, 10, seed=3)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((16, p.n))
    X2 = X.copy()
    X2[5:] = rng.standard_normal((11, p.n)) * 1e3
    X2[9] = 0.0
    with _problem(mq, p, "matfree_fp32") as pr:
        for trans in (False, True):
            say("independence", trans)
            Y = pr.apply_multi(X, trans=trans)
            Y2 = pr.apply_multi(X2, trans=trans)
            assert np.array_equal(Y[:5], Y2[:5])
            assert np.all(Y2[9] == 0.0)


def test_apply_multi_single_group_of_one_is_single_product(mq):
    p = I.multi_cube(333, 190, 6.0, 2.0, 1, 10, seed=5)
    x = I.random_vector(p.n, 4)
    with _problem(mq, p, "matfree_fp32") as pr:
        say("group of one")
        for trans in (False, True):
            assert np.array_equal(pr.apply_multi(x[None, :], trans=trans)[0], pr.apply(x, trans=trans))


# ---------------------------------------------------------------------------
# lockstep Golub-Kahan runs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["stored_fp64", "matfree_fp64"])
def test_gkb_multi_bitwise_single_fp64(mq, mode):
    p = I.multi_cube(333, 190, 6.0, 2.0, 5, 30, seed=5)
    with _problem(mq, p, mode) as pr:
        say("gkb_multi fp64 vs single", mode)
        r = pr.gkb_multi(p.F, p.ell)
        for k in range(p.nrhs):
            s = pr.gkb(p.F[k], p.ell)
            assert r["ell_done"][k] == s["ell_done"]
            for key in ("alpha", "beta", "W", "Z"):
                assert np.array_equal(r[key][k], s[key]), (k, key)


def test_gkb_long_runs_across_the_fused_cgs_limit(mq, orc):
    # 240 steps: the basis grows past the 224 columns that the fused
    # update-and-projection kernel keeps in LDS, so both forms of the
    # reorthogonalisation run, in the single and in the lockstep path
    p = I.multi_cube(1000, 300, 4.0, 1.5, 3, 240, seed=17)
    ell = p.ell
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    with _problem(mq, p, "stored_fp64") as pr:
        say("gkb_multi long runs, ell", ell)
        r = pr.gkb_multi(p.F, ell)
        singles = [pr.gkb(p.F[k], ell) for k in range(p.nrhs)]
    for k in range(p.nrhs):
        s = singles[k]
        assert r["ell_done"][k] == s["ell_done"] == ell
        for key in ("alpha", "beta", "W", "Z"):
            assert np.array_equal(r[key][k], s[key]), (k, key)
        g = orc.gkb(A, p.nodes, p.n_int, p.kappa, p.eps, p.F[k], ell)
        C = orc.bidiag_matrix(s["alpha"], s["beta"])
        W, Z = s["W"].T, s["Z"].T
        assert np.max(np.abs(W.T @ W - np.eye(ell + 1))) < 1e-12
        assert np.max(np.abs(Z.T @ Z - np.eye(ell))) < 1e-12
        assert np.linalg.norm(A @ Z - W @ C) / np.linalg.norm(C, 2) < 1e-12
        s_gpu = np.linalg.svd(C, compute_uv=False)
        s_orc = np.linalg.svd(orc.bidiag_matrix(g.alpha, g.beta), compute_uv=False)
        assert np.max(np.abs(s_gpu[:10] - s_orc[:10]) / s_orc[:10]) < 1e-12, k


def test_gkb_multi_group_of_one_fp32_bitwise_single(mq):
    p = I.multi_cube(333, 190, 6.0, 2.0, 1, 30, seed=5)
    with _problem(mq, p, "matfree_fp32") as pr:
        say("gkb_multi fp32 group of one")
        r = pr.gkb_multi(p.F, p.ell)
        s = pr.gkb(p.F[0], p.ell)
    for key in ("alpha", "beta", "W", "Z"):
        assert np.array_equal(r[key][0], s[key]), key


@pytest.mark.parametrize("name,make", RAGGED)
@pytest.mark.parametrize("nrhs", [16, 19])
def test_gkb_multi_block_against_oracle(mq, orc, name, make, nrhs):
    p = make(nrhs)
    ell = 20
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    with _problem(mq, p, "matfree_fp32") as pr:
        say("gkb_multi block", name, nrhs)
        r = pr.gkb_multi(p.F, ell)
    assert np.all(r["ell_done"] == ell) and r["status"] == 0
    for k in range(nrhs):
        g = orc.gkb(A, p.nodes, p.n_int, p.kappa, p.eps, p.F[k], ell)
        C = orc.bidiag_matrix(r["alpha"][k], r["beta"][k])
        s_gpu = np.linalg.svd(C, compute_uv=False)
        s_orc = np.linalg.svd(orc.bidiag_matrix(g.alpha, g.beta), compute_uv=False)
        assert np.max(np.abs(s_gpu[:5] - s_orc[:5]) / s_orc[:5]) < 1e-5, k
        assert r["beta"][k][0] == pytest.approx(g.beta[0], rel=1e-14)
        W, Z = r["W"][k].T, r["Z"][k].T
        assert np.max(np.abs(W.T @ W - np.eye(ell + 1))) < 1e-12
        assert np.max(np.abs(Z.T @ Z - np.eye(ell))) < 1e-12
        # A Z = W C with the oracle's A, to the FP32 entry error
        R = A @ Z - W @ C
        S = np.abs(A) @ np.abs(Z) + np.abs(W) @ np.abs(C)
        assert np.max(np.abs(R) / S) < 1e-5, k


def test_gkb_multi_runs_independent_and_breakdown(mq):
    # a zero right-hand side stops at once (beta_1 = 0); the other runs of its
    # group are bit-identical to a group without it; identical columns give
    # identical runs
    p = I.multi_cube(700, 300, 4.0, 1.5, 6, 15, seed=3)
    F = p.F
    G = np.concatenate([F[:3], np.zeros((1, p.n)), F[3:], F[1:2]], axis=0)  # 8 runs
    with _problem(mq, p, "matfree_fp32") as pr:
        say("gkb_multi independence")
        r = pr.gkb_multi(F, p.ell)
        q = pr.gkb_multi(G, p.ell)
    assert q["status"] == 1  # MQH_WBREAKDOWN
    assert q["ell_done"][3] == 0 and q["beta"][3][0] == 0.0
    assert np.all(q["W"][3] == 0.0) and np.all(q["Z"][3] == 0.0)
    for k, kg in ((0, 0), (1, 1), (2, 2), (3, 4), (4, 5), (5, 6)):
        for key in ("alpha", "beta", "W", "Z"):
            assert np.array_equal(r[key][k], q[key][kg]), (k, key)
    for key in ("alpha", "beta", "W", "Z"):
        assert np.array_equal(q[key][7], q[key][1]), key


# ---------------------------------------------------------------------------
# whole solves
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("method", ["hkt", "ine_tsvd", "lsqr"])
def test_solve_multi_bitwise_single_fp64(mq, method):
    p = I.multi_cube(333, 190, 6.0, 2.0, 4, 30, seed=5)
    m = {"hkt": mq.MQH_METHOD_HKT, "ine_tsvd": mq.MQH_METHOD_INE_TSVD, "lsqr": mq.MQH_METHOD_LSQR}[method]
    with _problem(mq, p, "matfree_fp64") as pr:
        say("solve_multi vs single", method)
        r = pr.solve_multi(p.F, p.ell, method=m)
        for k in range(p.nrhs):
            s = pr.solve(p.F[k, :p.n_int], p.F[k, p.n_int:], p.ell, method=m)
            assert np.array_equal(r.coef[k], s.coef), k
            assert r.lam[k] == s.lam and r.k[k] == s.k and r.ell_done[k] == s.ell_done
            assert r.crit[k] == s.crit and r.flags[k] == s.flags


def test_solve_multi_against_oracle(mq, orc):
    # FP64 form: each run's GCV lambda to 1e-6 of the oracle's, and at a
    # fixed lambda u to 1e-8; block form: at lambda = 1e-3 max_k s_1 u
    # within 1e-3 of the oracle (the single FP32 solve's bar)
    p = I.multi_cube(400, 240, 3.0, 0.7, 17, 60, seed=11)
    x_eval = I.cube_interior_uniform(500, 12)
    refs = [orc.solve(p.nodes, p.n_int, p.kappa, p.eps, p.F[k], p.ell, stored=False) for k in range(p.nrhs)]
    lam = np.array([ro.lam for ro in refs])
    s1 = max(float(ro.s[0]) for ro in refs)
    for mode, lam_c, tol in (("matfree_fp64", float(np.median(lam)), 1e-8), ("matfree_fp32", 1e-3 * s1, 1e-3)):
        with _problem(mq, p, mode) as pr:
            if mode == "matfree_fp64":
                say("solve_multi gcv", mode)
                r = pr.solve_multi(p.F, p.ell)
                for k in range(p.nrhs):
                    assert r.lam[k] == pytest.approx(lam[k], rel=1e-6), k
            say("solve_multi fixed lambda", mode, lam_c)
            rr = pr.solve_multi(p.F, p.ell, rule=mq.MQH_RULE_FIXED, lambda_fixed=lam_c)
            for k in range(p.nrhs):
                ro = orc.solve(p.nodes, p.n_int, p.kappa, p.eps, p.F[k], p.ell, stored=False,
                               rule=orc.RULE_FIXED, lambda_fixed=lam_c)
                u = pr.eval(rr.coef[k], x_eval)
                uo = orc.eval_u(p.nodes, p.eps, ro.coef, x_eval)
                assert np.linalg.norm(u - uo) <= tol * np.linalg.norm(uo), (mode, k)


def test_multi_invalid_arguments(mq):
    p = I.multi_cube(50, 30, 3.0, 1.0, 2, 5, seed=1)
    with _problem(mq, p, "matfree_fp32") as pr:
        say("multi invalid args")
        L = mq.lib
        n = p.n
        F = np.ascontiguousarray(p.F)
        fp = F.ctypes.data_as(mq.ctypes.c_void_p)
        assert L.mqh_gkb_multi(pr.h, fp, n, 0, 5, 1, None, None, None, None, None, 0) == mq.MQH_EINVAL
        assert L.mqh_gkb_multi(pr.h, fp, n - 1, 2, 5, 1, None, None, None, None, None, 0) == mq.MQH_EINVAL
        assert L.mqh_gkb_multi(pr.h, fp, n, 2, n + 1, 1, None, None, None, None, None, 0) == mq.MQH_EINVAL
        assert L.mqh_gkb_multi(pr.h, None, n, 2, 5, 1, None, None, None, None, None, 0) == mq.MQH_EINVAL
        bad = F.copy()
        bad[1, 3] = np.nan
        assert L.mqh_gkb_multi(pr.h, bad.ctypes.data_as(mq.ctypes.c_void_p), n, 2, 5, 1, None, None, None, None,
                               None, 0) == mq.MQH_EINVAL
        Y = np.empty_like(F)
        yp = Y.ctypes.data_as(mq.ctypes.c_void_p)
        assert L.mqh_apply_multi(pr.h, 2, fp, n, 2, None, None, n, yp, n, 0) == mq.MQH_EINVAL
        assert L.mqh_apply_multi(pr.h, 0, fp, n, 2, None, None, n, yp, n - 1, 0) == mq.MQH_EINVAL
        with pytest.raises(mq.MQHError):
            pr.solve_multi(F, 5, method=7)
        # the problem is still usable after rejected calls
        r = pr.gkb_multi(F, 5)
        assert np.all(r["ell_done"] == 5)


# ---------------------------------------------------------------------------
# sweeps of independent problems run side by side
# ---------------------------------------------------------------------------

def test_solve_sweep_matches_one_by_one(mq):
    # each problem on its own stream and host thread: results bit-identical to
    # solving the problems one at a time
    probs = [I.multi_cube(300 + 97 * k, 120 + 31 * k, 2.0 + 3.0 * k, 1.0 + 0.6 * k, 3 + (k % 3) * 7, 25, seed=50 + k)
             for k in range(5)]
    handles = []
    try:
        for p in probs:
            say("sweep create", p.name)
            handles.append(mq.Problem(p.x_int, p.x_bnd, p.kappa, p.eps, "matfree_fp32"))
        say("sweep one by one")
        ref = [h.solve_multi(p.F, p.ell) for h, p in zip(handles, probs)]
        for workers in (1, 3):
            say("sweep workers", workers)
            outs = mq.mqh_solve_sweep(handles, [p.F for p in probs], 25, workers=workers)
            for k, (o, r) in enumerate(zip(outs, ref)):
                assert o.status == r.status
                assert np.array_equal(o.coef, r.coef), (workers, k)
                assert np.array_equal(o.lam, r.lam) and np.array_equal(o.ell_done, r.ell_done)
        with pytest.raises(mq.MQHError):
            mq.mqh_solve_sweep([handles[0], handles[0]], [probs[0].F, probs[0].F], 25)
    finally:
        for h in handles:
            h.close()


def test_graph_replays_match_eager(mq):
    # the captured Golub-Kahan loop, replayed several times with other work on
    # the stream in between, gives the eager results bit for bit; a new group
    # size or ell recaptures
    p = I.multi_cube(600, 260, 5.0, 1.8, 12, 30, seed=21)
    with _problem(mq, p, "matfree_fp32") as pr:
        say("graph eager reference")
        ref = pr.solve_multi(p.F, p.ell)
        ref5 = pr.solve_multi(p.F[:5], 20)
        for rep in range(3):
            say("graph replay", rep)
            out = pr.solve_multi(p.F, p.ell, graph=True)
            assert np.array_equal(out.coef, ref.coef), rep
            assert np.array_equal(out.lam, ref.lam)
            pr.apply_multi(p.F[:3], trans=True)  # eager work between the replays
            out5 = pr.solve_multi(p.F[:5], 20, graph=True)  # other shape: recapture
            assert np.array_equal(out5.coef, ref5.coef), rep


def test_fixed_shapes_against_oracle(mq, orc):
    p = I.multi_cube(333, 190, 6.0, 2.0, 7, 30, seed=5)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((7, p.n))
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    say("fixed shapes")
    with mq.Problem(p.x_int, p.x_bnd, p.kappa, p.eps, "matfree_fp32", fixed_shapes=True) as pr:
        for trans in (False, True):
            Y = pr.apply_multi(X, trans=trans)
            Aop = A.T if trans else A
            err = np.abs(Y.T - Aop @ X.T) / (np.abs(Aop) @ np.abs(X.T))
            assert np.all(err <= 4e-6), float(err.max())


# the block products' FP16 split: each column carries its own power-of-two scale, the entries one
# per problem (from a bound on the largest entry), so the bar holds whatever the columns' sizes and
# wherever the class boundary and the end of the node range fall within the 4-node quads
@pytest.mark.parametrize("n_int,n_bnd", [(5, 3), (13, 10), (61, 66), (258, 131)])
def test_apply_multi_tiny_and_unaligned(mq, orc, n_int, n_bnd):
    p = I.multi_cube(n_int, n_bnd, 9.0, 3.0, 3, 5, seed=n_int)
    rng = np.random.default_rng(n_bnd)
    X = rng.standard_normal((3, p.n))
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    with _problem(mq, p, "matfree_fp32") as pr:
        for trans in (False, True):
            say("tiny / unaligned", n_int, n_bnd, "trans", trans)
            Y = pr.apply_multi(X, trans=trans)
            Aop = A.T if trans else A
            err = np.abs(Y.T - Aop @ X.T) / (np.abs(Aop) @ np.abs(X.T))
            assert np.all(err <= 4e-6), float(err.max())


def test_apply_multi_column_scales(mq, orc):
    # columns from 1e-30 to 1e30 in one call, one of them zero, another with a single nonzero entry
    p = I.multi_cube(700, 300, 12.0, 4.0, 6, 10, seed=4)
    rng = np.random.default_rng(6)
    X = rng.standard_normal((6, p.n)) * np.array([1e-30, 1e-8, 1.0, 1e12, 1e30, 0.0])[:, None]
    X[5, 17] = 3.0
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    with _problem(mq, p, "matfree_fp32") as pr:
        for trans in (False, True):
            say("column scales, trans", trans)
            Y = pr.apply_multi(X, trans=trans)
            Aop = A.T if trans else A
            err = np.abs(Y.T - Aop @ X.T) / (np.abs(Aop) @ np.abs(X.T))
            assert np.all(err <= 4e-6), float(err.max())


def test_apply_multi_row_scaled_against_oracle(mq, orc):
    # D A (D = diag(A)^-1) through the block products: the interior constants shrink, the entry
    # scale follows them
    p = I.multi_cube(333, 190, 20.0, 5.0, 4, 10, seed=8)
    rng = np.random.default_rng(9)
    X = rng.standard_normal((4, p.n))
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    d = orc.row_scale(p.nodes, p.n_int, p.kappa, p.eps)
    DA = d[:, None] * A
    with _problem(mq, p, "matfree_fp32") as pr:
        for trans in (False, True):
            say("row scaled block product, trans", trans)
            Y = pr.apply_multi(X, trans=trans, row_scale=1)
            Aop = DA.T if trans else DA
            err = np.abs(Y.T - Aop @ X.T) / (np.abs(Aop) @ np.abs(X.T))
            assert np.all(err <= 4e-6), float(err.max())


@pytest.mark.parametrize("kappa,eps", [(80.0, 25.0), (0.5, 0.1)])
def test_apply_multi_entry_scale_extremes(mq, orc, kappa, eps):
    # entries far above the FP16 range before their power-of-two scale (kappa^2 sqrt(t) ~ 3e5)
    # and far below it (2 eps^2 + eps^2 ~ 0.03): the bar holds at both ends
    p = I.multi_cube(400, 200, kappa, eps, 4, 10, seed=12)
    rng = np.random.default_rng(13)
    X = rng.standard_normal((4, p.n))
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    with _problem(mq, p, "matfree_fp32") as pr:
        for trans in (False, True):
            say("entry scale extremes", kappa, eps, "trans", trans)
            Y = pr.apply_multi(X, trans=trans)
            Aop = A.T if trans else A
            err = np.abs(Y.T - Aop @ X.T) / (np.abs(Aop) @ np.abs(X.T))
            assert np.all(err <= 4e-6), float(err.max())
