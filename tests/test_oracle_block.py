"""Pins for the block oracle (oracle/block.py: block Golub-Kahan and block
Tikhonov for several right-hand sides sharing one Krylov space).

* one source (s = 1): the block recurrence is Algorithm 1 -- C_l equals the
  bidiagonal of the oracle's single-vector run (alpha_j = D_j,
  beta_{j+1} = E_{j+1}), and the block solve with GCV is the projected HKT
  solve of Algorithm 4 with eq. (30);
* the block Krylov relations A Z_l = W_{l+1} C_l, A^T W_l = Z_l (C_l)_{1:ls}^T,
  W_1 E_1 = F and orthonormal bases, to rounding;
* the shape of C_l: lower block bidiagonal, D_j lower triangular, E_{j+1}
  upper triangular with non-negative diagonals;
* a saturated block space (l s = n): at any fixed lambda each source's
  solution is the textbook Tikhonov solution of eq. (17) for that source;
* the sources' order does not matter: permuting the columns of F permutes
  the solutions at fixed lambda (the block Krylov space is the same);
* breakdown: a block F inside an invariant subspace of A A^T stops the
  process after one step; zero or linearly dependent sources are rejected;
* the block GCV: equal to the GCV formed from the projected influence matrix
  by dense solves (no SVD), and, for one source with a short run (large
  f~_{l+1}), to the projected HKT choice of eq. (30).
"""
import numpy as np
import pytest

from paper_2511_09798_amd import inputs as I


@pytest.fixture(scope="module")
def blk():
    from oracle import block

    return block


@pytest.fixture(scope="module")
def small(orc):
    p = I.cube_scaled(150, 90, kappa=6.0, eps=2.0, ell=30)
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    F = np.stack([I.random_vector(p.n, 900 + k) for k in range(5)], axis=1)
    return p, A, F


def test_one_source_is_algorithm_1(orc, blk, small):
    p, A, F = small
    f = F[:, :1]
    g = blk.block_gkb(A, f, 12)
    ref = orc.gkb(A, p.nodes, p.n_int, p.kappa, p.eps, f[:, 0], 12)
    assert g.ell == ref.ell == 12
    Cref = orc.bidiag_matrix(ref.alpha, ref.beta)
    assert np.max(np.abs(g.C - Cref)) <= 1e-12 * np.max(np.abs(Cref))
    assert g.E1[0, 0] == pytest.approx(ref.beta[0], rel=1e-14)
    assert np.max(np.abs(np.abs(g.Z) - np.abs(ref.Z))) <= 1e-10


def test_one_source_solve_is_hkt_gcv(orc, blk, small):
    p, A, F = small
    f = F[:, 0]
    r = blk.block_solve(A, F[:, :1], 12)
    ref = orc.solve(p.nodes, p.n_int, p.kappa, p.eps, f, 12)
    assert r.lam[0] == pytest.approx(ref.lam, rel=1e-9)
    assert np.linalg.norm(r.coef[:, 0] - ref.coef) <= 1e-9 * np.linalg.norm(ref.coef)


def test_block_relations(blk, small):
    p, A, F = small
    s, ell = F.shape[1], 8
    g = blk.block_gkb(A, F, ell)
    assert g.ell == ell and g.flag == 0
    nc = np.linalg.norm(g.C, 2)
    assert np.linalg.norm(A @ g.Z - g.W @ g.C) <= 1e-12 * nc
    Cl = g.C[: ell * s, :]
    assert np.linalg.norm(A.T @ g.W[:, : ell * s] - g.Z @ Cl.T) <= 1e-12 * nc
    assert np.linalg.norm(g.W[:, :s] @ g.E1 - F) <= 1e-13 * np.linalg.norm(F)
    assert np.max(np.abs(g.W.T @ g.W - np.eye(g.W.shape[1]))) <= 1e-12
    assert np.max(np.abs(g.Z.T @ g.Z - np.eye(g.Z.shape[1]))) <= 1e-12


def test_block_bidiagonal_shape(blk, small):
    p, A, F = small
    s, ell = F.shape[1], 6
    g = blk.block_gkb(A, F, ell)
    C = g.C
    for j in range(ell):
        D = C[j * s:(j + 1) * s, j * s:(j + 1) * s]
        E = C[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s]
        assert np.all(np.triu(D, 1) == 0.0) and np.all(np.diag(D) >= 0.0)
        assert np.all(np.tril(E, -1) == 0.0) and np.all(np.diag(E) >= 0.0)
        mask = np.ones(C.shape[0], bool)
        mask[j * s:(j + 2) * s] = False
        assert np.all(C[mask, j * s:(j + 1) * s] == 0.0)
    assert np.all(np.tril(g.E1, -1) == 0.0) and np.all(np.diag(g.E1) >= 0.0)


@pytest.mark.parametrize("n,s", [(24, 3), (32, 4)])
def test_saturated_block_space_is_textbook_tikhonov(orc, blk, n, s):
    X = I.random_nodes_cube(n, 500 + n)
    A = orc.assemble(X, n // 2, 2.0, 6.0)
    F = np.stack([I.random_vector(n, 600 + n + k) for k in range(s)], axis=1)
    sv = np.linalg.svd(A, compute_uv=False)
    for lam in (1e-3 * sv[0], 1e-1 * sv[0], sv[n // 2]):
        r = blk.block_solve(A, F, n // s, lambda_fixed=lam)
        assert r.gkb.ell == n // s
        for k in range(s):
            ref = orc.full_tikhonov(A, F[:, k], lam)
            assert np.linalg.norm(r.coef[:, k] - ref) <= 1e-9 * np.linalg.norm(ref)


def test_source_order_does_not_matter(blk, small):
    p, A, F = small
    perm = np.array([3, 0, 4, 2, 1])
    lam = np.linspace(1e-3, 1e-1, F.shape[1])
    r = blk.block_solve(A, F, 6, lambda_fixed=lam)
    rp = blk.block_solve(A, F[:, perm], 6, lambda_fixed=lam[perm])
    assert np.linalg.norm(rp.coef - r.coef[:, perm]) <= 1e-9 * np.linalg.norm(r.coef)


def test_breakdown_in_an_invariant_subspace(blk, small):
    p, A, F = small
    U, sv, Vt = np.linalg.svd(A)
    s = 3
    # F spans three left singular vectors: A^T F = V_3 S_3, A V_3 = U_3 S_3, so
    # the second W block has nothing left after reorthogonalisation
    Fi = U[:, :s] @ np.array([[2.0, 0.3, 0.1], [0.0, 1.0, 0.2], [0.0, 0.0, 0.5]])
    g = blk.block_gkb(A, Fi, 5)
    assert g.flag == 2 and g.ell == 1
    assert np.all(g.C[s:, :] == 0.0)
    np.testing.assert_allclose(np.sort(np.linalg.svd(g.C[:s, :], compute_uv=False)), np.sort(sv[:s]), rtol=1e-12)


def test_dependent_or_zero_sources_are_rejected(blk, small):
    p, A, F = small
    for G in (F[:, [0, 1, 0]], np.column_stack([F[:, 0], np.zeros(p.n), F[:, 2]]),
              np.column_stack([F[:, 0], F[:, 1], 2.0 * F[:, 0] - 3.0 * F[:, 1]])):
        with pytest.raises(ValueError):
            blk.block_gkb(A, G, 3)
    # nearly dependent but distinct sources are valid
    G = np.column_stack([F[:, 0], F[:, 0] + 1e-6 * F[:, 1]])
    assert blk.block_gkb(A, G, 3).ell == 3


def test_block_gcv_equals_explicit_influence_matrix(orc, blk, small):
    # GCV of source k from the projected influence matrix H = C (C^T C + lambda^2 I)^{-1} C^T,
    # formed by dense solves (no SVD): ||(I - H) b_k||^2 / (m - tr H)^2 equals the SVD form the
    # block solve minimises, at its chosen lambda and at two other values
    p, A, F = small
    r = blk.block_solve(A, F, 4)
    C = r.gkb.C
    m, ls = C.shape
    s = F.shape[1]
    for k in range(s):
        b = np.zeros(m)
        b[:s] = r.gkb.E1[:, k]
        for lam in (r.lam[k], 10.0 * r.lam[k], 0.1 * r.lam[k]):
            K = C.T @ C + lam * lam * np.eye(ls)
            H = C @ np.linalg.solve(K, C.T)
            g_explicit = float(np.sum(((np.eye(m) - H) @ b) ** 2)) / (m - np.trace(H)) ** 2
            g_svd = orc.gcv_full(r.sv, r.ftil[:, k], float(r.s_perp[k]), m, lam)
            assert g_svd == pytest.approx(g_explicit, rel=1e-8)


def test_one_source_short_run_is_hkt_gcv(orc, blk, small):
    # l = 3: a large projected residual f~_{l+1}, which the block GCV carries as s_perp
    p, A, F = small
    f = F[:, 1]
    r = blk.block_solve(A, F[:, 1:2], 3)
    ref = orc.solve(p.nodes, p.n_int, p.kappa, p.eps, f, 3)
    assert abs(ref.ftil[-1]) > 1e-3 * ref.beta[0]
    assert r.lam[0] == pytest.approx(ref.lam, rel=1e-9)
    assert np.linalg.norm(r.coef[:, 0] - ref.coef) <= 1e-9 * np.linalg.norm(ref.coef)
