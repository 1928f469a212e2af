"""GPU parity of the block Golub-Kahan path (mqh_gkb_block, mqh_solve_block:
several sources sharing one Krylov space) against the block oracle
(oracle/block.py).

* The recurrence, FP64 operators: the block Krylov relations A Z = W C and
  A^T W_l = Z_l (C_l)_{1:ls}^T with the oracle's FP64 A, orthonormal bases,
  W_1 E_1 = F, all to 1e-12; the structure of C (triangular blocks,
  non-negative diagonals); the singular values of C against the oracle's
  C: the leading ten to 1e-10 relative, all to 64 (l + 1) s eps sigma_1
  (two backward-stable recurrences; the QR differs: shifted Cholesky QR on
  the GPU, Householder in the oracle); the first two blocks of C element
  by element to 1e-10 of ||C|| (positive diagonals fix the signs).
* The solve, FP64 operators: at the oracle's per-source lambda (FIXED rule)
  u within 1e-8 and coefficients within 1e-6 relative; with GCV each
  source's lambda within 1e-6 relative (the projected problem is small and
  well separated: its GCV minimum moves by less under the two SVDs); one
  source (nrhs = 1) equals the single-source HKT solve (mqh_solve) to the
  same bars.
* FP32-evaluated block products (nrhs >= 2 on the matrix cores): relations
  with the oracle's A to the single FP32 product's bound scaled by ||C||
  (1e-5), u at the oracle's lambda within 1e-3.
* A block inside an invariant subspace breaks down after one step, as in
  the oracle; invalid arguments are rejected.
* Permuting the sources permutes the choices and the solutions; zero and
  linearly dependent sources are rejected, nearly dependent ones are not.
* The workspace kept on the problem: a call after calls of other sizes
  returns the bits of a fresh problem's call.
* At the benchmark's size (the 20 596-node sweep cube, 16 sources, 7 block
  steps, FP32 block products): A Z = W C on sampled rows with the oracle's
  FP64 entries (measured 1e-9 of ||C||), orthonormal bases, W_1 E_1 = F.
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


@pytest.fixture(scope="module")
def blk():
    from oracle import block

    return block


@pytest.fixture(scope="module")
def case(orc):
    p = I.cube_scaled(333, 190, kappa=6.0, eps=2.0, ell=40)
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    F = np.stack([I.random_vector(p.n, 700 + k) for k in range(5)])  # nrhs x n
    return p, A, F


def _problem(mq, p, mode):
    say("create", p.name, "n", p.n, mode)
    return mq.Problem(p.x_int, p.x_bnd, p.kappa, p.eps, mode)


@pytest.mark.parametrize("mode", ["stored_fp64", "matfree_fp64"])
def test_block_gkb_against_oracle(mq, blk, case, mode):
    p, A, F = case
    s, ell = F.shape[0], 8
    with _problem(mq, p, mode) as pr:
        say("block gkb", mode, "s", s, "ell", ell)
        g = pr.gkb_block(F, ell, want_bases=True)
    assert g["status"] == 0 and g["ell_done"] == ell
    C, W, Z = g["C"], g["W"].T, g["Z"].T
    nc = np.linalg.norm(C, 2)
    assert np.linalg.norm(A @ Z - W @ C) <= 1e-12 * nc
    assert np.linalg.norm(A.T @ W[:, : ell * s] - Z @ C[: ell * s, :].T) <= 1e-12 * nc
    assert np.linalg.norm(W[:, :s] @ g["E1"] - F.T) <= 1e-13 * np.linalg.norm(F)
    assert np.max(np.abs(W.T @ W - np.eye(W.shape[1]))) <= 1e-12
    assert np.max(np.abs(Z.T @ Z - np.eye(Z.shape[1]))) <= 1e-12
    for j in range(ell):
        D = C[j * s:(j + 1) * s, j * s:(j + 1) * s]
        E = C[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s]
        assert np.all(np.triu(D, 1) == 0.0) and np.all(np.diag(D) >= 0.0)
        assert np.all(np.tril(E, -1) == 0.0) and np.all(np.diag(E) >= 0.0)
    o = blk.block_gkb(A, F.T, ell)
    sg = np.linalg.svd(C, compute_uv=False)
    so = np.linalg.svd(o.C, compute_uv=False)
    say("sv diff", np.max(np.abs(sg - so)) / so[0], "C[:2 blocks] diff", np.max(np.abs(C[:, : 2 * s] - o.C[:, : 2 * s])) / nc)
    assert np.max(np.abs(sg[:10] - so[:10]) / so[:10]) <= 1e-10
    assert np.max(np.abs(sg - so)) <= 64 * (ell + 1) * s * EPS * so[0]
    assert np.max(np.abs(C[:, : 2 * s] - o.C[:, : 2 * s])) <= 1e-10 * nc
    assert np.max(np.abs(g["E1"] - o.E1)) <= 1e-13 * np.abs(o.E1).max()


@pytest.fixture(scope="module")
def blobs(case):
    # five Gaussian-blob sources (the sweep's kind) with 1e-3 seeded noise: at 16 block steps
    # every source's GCV minimum is interior (lambda / sigma_1 = 3e-3 .. 0.11)
    p, A, F = case
    cent = np.random.default_rng(5).random((5, 3))
    Fb = np.zeros((5, p.n))
    Fb[:, : p.n_int] = I.blob_sources(p.x_int, cent)
    noise = np.stack([np.linalg.norm(Fb[k]) * I.random_vector(p.n, 70 + k) / np.sqrt(p.n) for k in range(5)])
    return Fb + 1e-3 * noise


@pytest.mark.parametrize("mode", ["stored_fp64", "matfree_fp64"])
def test_block_solve_against_oracle(mq, orc, blk, case, blobs, mode):
    p, A, _ = case
    F = blobs
    s, ell = F.shape[0], 16
    ref = blk.block_solve(A, F.T, ell)
    assert np.all(ref.lam < ref.sv[0])
    fixed = blk.block_solve(A, F.T, ell, lambda_fixed=ref.lam)
    with _problem(mq, p, mode) as pr:
        say("block solve gcv", mode)
        out = pr.solve_block(F, ell)
        say("lambda", out.lam, "oracle", ref.lam, "sweeps", out.t_ms[0, 6], "cg", out.t_ms[:, 7])
        outs = []
        for k in range(s):
            o = pr.solve_block(F, ell, rule=mq.MQH_RULE_FIXED, lambda_fixed=float(ref.lam[k]))
            outs.append(o.coef[k])
        coef = np.stack(outs)
        u = np.stack([pr.eval(coef[k], p.x_eval) for k in range(s)])
    assert out.status == 0 and not np.any(out.flags & mq.MQH_INFO_GCV_AT_EDGE)
    np.testing.assert_allclose(out.lam, ref.lam, rtol=1e-6)
    for k in range(s):
        uo = orc.eval_u(p.nodes, p.eps, fixed.coef[:, k], p.x_eval)
        assert np.linalg.norm(u[k] - uo) <= 1e-8 * np.linalg.norm(uo)
        assert np.linalg.norm(coef[k] - fixed.coef[:, k]) <= 1e-6 * np.linalg.norm(fixed.coef[:, k])
    # reported norms: ||A coef - f|| and ||coef|| of the GCV solutions
    for k in range(s):
        assert out.resid_norm[k] == pytest.approx(np.linalg.norm(A @ out.coef[k] - F[k]), rel=1e-8)
        assert out.sol_norm[k] == pytest.approx(np.linalg.norm(out.coef[k]), rel=1e-8)


@pytest.mark.parametrize("nsrc,ell", [(5, 16), (2, 60), (16, 7)])
def test_block_band_path_matches_jacobi(mq, case, blobs, nsrc, ell):
    # the projected problem by the band reduction of C^T (the default) and by the Jacobi full SVD
    # (MQH_FLAG_BLOCK_JACOBI): the same singular values, GCV choices and fixed-lambda solutions to
    # rounding; the info flags say which path ran
    p, A, _ = case
    F = blobs if nsrc == 5 else np.stack([I.random_vector(p.n, 900 + k) for k in range(nsrc)])
    with _problem(mq, p, "stored_fp64") as pr:
        say("block solve, band and Jacobi paths, s", nsrc, "ell", ell)
        a = pr.solve_block(F, ell, want_sv=True)
        b = pr.solve_block(F, ell, want_sv=True, jacobi=True)
        lam = float(np.median(b.lam))
        af = pr.solve_block(F, ell, rule=mq.MQH_RULE_FIXED, lambda_fixed=lam)
        bf = pr.solve_block(F, ell, rule=mq.MQH_RULE_FIXED, lambda_fixed=lam, jacobi=True)
    assert not np.any(a.flags & mq.MQH_INFO_BLOCK_JACOBI) and np.all(b.flags & mq.MQH_INFO_BLOCK_JACOBI)
    assert np.all(a.ell_done == b.ell_done)
    n_sv = int(a.ell_done[0]) * nsrc
    dsv = np.max(np.abs(a.sv[:n_sv] - b.sv[:n_sv])) / b.sv[0]
    say("sv diff", dsv, "lambda", a.lam, b.lam)
    assert dsv <= 64 * n_sv * EPS
    np.testing.assert_allclose(a.lam, b.lam, rtol=1e-6)
    for k in range(nsrc):
        assert np.linalg.norm(af.coef[k] - bf.coef[k]) <= 1e-9 * np.linalg.norm(bf.coef[k])
        assert np.linalg.norm(a.coef[k] - b.coef[k]) <= 1e-5 * np.linalg.norm(b.coef[k])


@pytest.mark.parametrize("mode", ["matfree_fp32", "stored_fp64"])
def test_block_jacobi_path_twice_in_a_row(mq, case, mode):
    # two Jacobi-route solves of the same sizes back to back (the second reuses the cached run),
    # device pointers as the benchmark passes them: the same bits both times
    import torch

    p, A, _ = case
    F = torch.from_numpy(np.stack([I.random_vector(p.n, 990 + k) for k in range(16)])).to("cuda:0")
    with _problem(mq, p, mode) as pr:
        say("block solve, Jacobi route twice,", mode)
        a = pr.solve_block(F, 4, jacobi=True)
        b = pr.solve_block(F, 4, jacobi=True)
        c = pr.solve_block(F, 4)
    assert a.status in (0, mq.MQH_WEDGE) and b.status == a.status
    assert np.all(a.flags & mq.MQH_INFO_BLOCK_JACOBI) and not np.any(c.flags & mq.MQH_INFO_BLOCK_JACOBI)
    ac, bc, cc = a.coef.cpu().numpy(), b.coef.cpu().numpy(), c.coef.cpu().numpy()
    assert np.array_equal(ac, bc)
    for k in range(16):
        assert np.linalg.norm(cc[k] - ac[k]) <= 1e-5 * np.linalg.norm(ac[k])


def test_block_band_path_size_limit(mq):
    # 16 sources: 25 block steps (N = 400 columns of C) are the most the band chase holds in LDS;
    # 26 take the Jacobi path.  At 25 the two paths agree as above.
    p = I.cube_scaled(2400, 600, kappa=4.0, eps=1.5, ell=25)
    F = np.stack([I.random_vector(p.n, 950 + k) for k in range(16)])
    with _problem(mq, p, "stored_fp64") as pr:
        say("block solve at the band path's size limit")
        a = pr.solve_block(F, 25, want_sv=True)
        lam = float(np.median(a.lam))
        af = pr.solve_block(F, 25, rule=mq.MQH_RULE_FIXED, lambda_fixed=lam)
        bf = pr.solve_block(F, 25, rule=mq.MQH_RULE_FIXED, lambda_fixed=lam, jacobi=True)
        say("one step more")
        c = pr.solve_block(F, 26)
    say("ell_done", a.ell_done[0], c.ell_done[0], "flags", a.flags[0], c.flags[0])
    assert a.ell_done[0] == 25 and c.ell_done[0] == 26
    assert not np.any(a.flags & mq.MQH_INFO_BLOCK_JACOBI) and np.all(c.flags & mq.MQH_INFO_BLOCK_JACOBI)
    for k in range(16):
        assert np.linalg.norm(af.coef[k] - bf.coef[k]) <= 1e-9 * np.linalg.norm(bf.coef[k])


def test_block_one_source_is_single_hkt(mq):
    # the cube with an interior GCV minimum of the single-source parity tests
    p = I.cube_scaled(400, 240, kappa=3.0, eps=0.7, ell=80)
    f = p.rhs
    with _problem(mq, p, "stored_fp64") as pr:
        say("block solve, one source")
        out = pr.solve_block(f[None, :].copy(), p.ell)
        ref = pr.solve(p.f_int, p.g_bnd, p.ell)
        u = pr.eval(out.coef[0], p.x_eval)
        ur = pr.eval(ref.coef, p.x_eval)
    assert not (ref.flags & mq.MQH_INFO_GCV_AT_EDGE)
    say("lambda", out.lam[0], "single", ref.lam)
    assert out.lam[0] == pytest.approx(ref.lam, rel=1e-6)
    assert np.linalg.norm(u - ur) <= 1e-8 * np.linalg.norm(ur)


def test_block_fp32_products(mq, orc, blk, case):
    p, A, F = case
    F16 = np.stack([I.random_vector(p.n, 800 + k) for k in range(16)])
    s, ell = 16, 4
    with _problem(mq, p, "matfree_fp32") as pr:
        say("block gkb fp32, s", s)
        g = pr.gkb_block(F16, ell, want_bases=True)
        ref = blk.block_solve(A, F16.T, ell)
        say("block solve fp32 fixed")
        out = pr.solve_block(F16, ell, rule=mq.MQH_RULE_FIXED, lambda_fixed=float(np.median(ref.lam)))
        u = np.stack([pr.eval(out.coef[k], p.x_eval) for k in range(s)])
    C, W, Z = g["C"], g["W"].T, g["Z"].T
    nc = np.linalg.norm(C, 2)
    rel = np.linalg.norm(A @ Z - W @ C) / nc
    say("fp32 relation", rel)
    assert rel <= 1e-5
    assert np.max(np.abs(Z.T @ Z - np.eye(Z.shape[1]))) <= 1e-12
    fixed = blk.block_solve(A, F16.T, ell, lambda_fixed=float(np.median(ref.lam)))
    for k in range(s):
        uo = orc.eval_u(p.nodes, p.eps, fixed.coef[:, k], p.x_eval)
        assert np.linalg.norm(u[k] - uo) <= 1e-3 * np.linalg.norm(uo)


def test_block_breakdown_in_invariant_subspace(mq, blk, case):
    p, A, F = case
    U, sv, Vt = np.linalg.svd(A)
    Fi = (U[:, :3] @ np.array([[2.0, 0.3, 0.1], [0.0, 1.0, 0.2], [0.0, 0.0, 0.5]])).T.copy()
    with _problem(mq, p, "stored_fp64") as pr:
        say("block gkb, invariant subspace")
        g = pr.gkb_block(Fi, 5)
    o = blk.block_gkb(A, Fi.T, 5)
    assert o.flag == 2 and o.ell == 1
    assert g["status"] == mq.MQH_WBREAKDOWN and g["flag"] == 2 and g["ell_done"] == 1
    np.testing.assert_allclose(np.sort(np.linalg.svd(g["C"][:3, :3], compute_uv=False)), np.sort(sv[:3]), rtol=1e-10)


def test_block_source_order(mq, case, blobs):
    # the block Krylov space depends on the span of F only: permuting the sources permutes the
    # GCV choices and the solutions (the oracle's pin of the same property); on the GPU the
    # Cholesky QR of the permuted block rounds differently, so to the bars of the oracle parity
    p, A, _ = case
    F = blobs
    perm = np.array([3, 0, 4, 2, 1])
    with _problem(mq, p, "stored_fp64") as pr:
        say("block solve, sources in two orders")
        a = pr.solve_block(F, 16)
        b = pr.solve_block(np.ascontiguousarray(F[perm]), 16)
    assert a.status == 0 and b.status == 0
    np.testing.assert_allclose(b.lam, a.lam[perm], rtol=1e-6)
    for k in range(F.shape[0]):
        ref = a.coef[perm[k]]
        assert np.linalg.norm(b.coef[k] - ref) <= 1e-6 * np.linalg.norm(ref)


def test_block_dependent_or_zero_sources_are_rejected(mq, case, blobs):
    # as the oracle: the sources must be linearly independent to working precision
    p, A, _ = case
    F = blobs
    bad = [np.stack([F[0], F[1], F[0]]), np.stack([F[0], np.zeros(p.n), F[2]]),
           np.stack([F[0], F[1], 2.0 * F[0] - 3.0 * F[1]])]
    with _problem(mq, p, "stored_fp64") as pr:
        for k, G in enumerate(bad):
            say("block, dependent or zero sources, case", k)
            with pytest.raises(mq.MQHError):
                pr.solve_block(np.ascontiguousarray(G), 4)
            with pytest.raises(mq.MQHError):
                pr.gkb_block(np.ascontiguousarray(G), 4)
        say("block, nearly dependent sources")
        g = pr.gkb_block(np.ascontiguousarray(np.stack([F[0], F[0] + 1e-6 * F[1]])), 4)
    assert g["status"] == 0 and g["ell_done"] == 4


def test_block_relations_full_size_sampled(mq, orc):
    # the benchmark's launch configuration: the 20 596-node sweep cube, its 16 sources, 7 block
    # steps on the FP32-evaluated block products.  The relation A Z = W C on 3 columns of Z at
    # 64 sampled rows, with the oracle's FP64 entries one by one, to the FP32 products' bar of the
    # small-case test (1e-5 of ||C||); the bases orthonormal (FP64 reorthogonalisation) and
    # W_1 E_1 = F on the same rows.
    m = I.sweep_member(0)
    X = np.vstack([m.x_int, m.x_bnd])
    n_int = m.x_int.shape[0]
    with mq.Problem(m.x_int, m.x_bnd, m.kappa, m.eps, "matfree_fp32") as pr:
        say("block gkb full size n", X.shape[0], "s 16 ell 7")
        g = pr.gkb_block(m.F, 7, want_bases=True)
    assert g["status"] == 0 and g["ell_done"] == 7
    C, W, Z = g["C"], g["W"].T, g["Z"].T
    nc = np.linalg.norm(C, 2)
    rows = np.random.default_rng(11).choice(X.shape[0], 64, replace=False)
    for j in (0, 57, 111):
        az = orc.apply_sampled(X, n_int, m.kappa, m.eps, Z[:, j], rows)
        err = np.max(np.abs(az - W[rows] @ C[:, j]))
        say("column", j, "max |A z - W c| / ||C||", err / nc)
        assert err <= 1e-5 * nc
    assert np.max(np.abs(Z.T @ Z - np.eye(Z.shape[1]))) <= 1e-12
    assert np.max(np.abs(W.T @ W - np.eye(W.shape[1]))) <= 1e-12
    assert np.max(np.abs(W[rows, :16] @ g["E1"] - m.F[:, rows].T)) <= 1e-13 * np.abs(m.F).max() * 16


def test_block_deterministic(mq, case, blobs):
    # fixed-order reductions throughout: a repeated call returns the same bits
    p, A, _ = case
    with _problem(mq, p, "matfree_fp32") as pr:
        say("block determinism")
        a = pr.solve_block(blobs, 16)
        b = pr.solve_block(blobs, 16)
    assert np.array_equal(a.coef, b.coef) and np.array_equal(a.lam, b.lam)


def test_block_workspace_reuse(mq, case, blobs):
    # the block calls keep their workspace on the problem: calls of other sizes in between (another
    # step count, another source count, a bare recurrence) must not change a later call's bits
    p, A, _ = case
    F = np.ascontiguousarray(blobs)
    with _problem(mq, p, "stored_fp64") as fresh:
        say("block workspace: fresh problem")
        ref = fresh.solve_block(F, 8)
    with _problem(mq, p, "stored_fp64") as pr:
        say("block workspace: calls of other sizes in between")
        pr.solve_block(F, 16)
        pr.solve_block(np.ascontiguousarray(F[:3]), 8)
        pr.gkb_block(F, 5)
        a = pr.solve_block(F, 8)
        b = pr.solve_block(F, 8)
    assert np.array_equal(a.coef, ref.coef) and np.array_equal(b.coef, ref.coef)
    assert np.array_equal(a.lam, ref.lam)


def test_block_size_limits(mq):
    # (ell + 1) nrhs at the limit MQH_BLOCK_MAX_DIM passes the argument check, one more step does not;
    # n = 8 200 nodes so that ell nrhs <= n holds on both sides (matrix-free: nothing of size n^2)
    X = I.random_nodes_cube(8200, 31)
    f = np.stack([I.random_vector(8200, 40 + k) for k in range(2)])
    with mq.Problem(X[:7000], X[7000:], 2.0, 1.5, "matfree_fp32") as pr:
        ell_max = mq.MQH_BLOCK_MAX_DIM // 2 - 1
        say("block size limit: ell", ell_max + 1, "nrhs 2 rejected")
        with pytest.raises(mq.MQHError):
            pr.gkb_block(f, ell_max + 1)
        with pytest.raises(mq.MQHError):
            pr.solve_block(f, ell_max + 1)


def test_block_invalid_arguments(mq, case):
    p, A, F = case
    with _problem(mq, p, "stored_fp64") as pr:
        with pytest.raises(mq.MQHError):
            pr.solve_block(np.zeros((17, p.n)), 2)
        with pytest.raises(mq.MQHError):
            pr.solve_block(F, p.n)  # ell nrhs > n
        opts = mq.mqh_solve_opts(ell=2, reorth=1, method=mq.MQH_METHOD_LSQR, rule=mq.MQH_RULE_GCV)
        Fc = np.ascontiguousarray(F[:2])
        coef = np.zeros_like(Fc)
        assert mq.lib.mqh_solve_block(pr.h, Fc.ctypes.data, p.n, 2, opts, coef.ctypes.data, p.n, None,
                                      None) == mq.MQH_EINVAL
