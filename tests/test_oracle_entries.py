"""Pins for the oracle's matrix entries, manufactured data and the MQ matrix structure.

Each check ties the oracle to something fixed by the paper or by
mathematics, not to the oracle itself:
* hand-worked closed-form values (tests/golden/mq_entries.txt);
* the Laplacian as a finite-difference limit of the kernel (eq. (7): the
  interior rows apply Lap + kappa^2 to phi);
* rigid-motion invariance of A (entries depend only on distances, eq. (3));
* the interpolation matrix B having exactly one positive eigenvalue
  (the CPD(1) property of Section 4.1, with the sign the classical
  statement has: -B is conditionally positive definite);
* the manufactured solutions satisfying Lap u = -k^2 u.
"""
import math
import os

import numpy as np
import pytest

from paper_2511_09798_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mq_entries.txt")


def _golden_rows():
    env = {"sqrt": math.sqrt}
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            c = line.split()
            rows.append(tuple(float(eval(x, {"__builtins__": {}}, env)) for x in c))
    return rows


@pytest.mark.parametrize("row", _golden_rows())
def test_golden_closed_form_entries(orc, row):
    eps, r, kappa, phi, lap, lphi = row
    assert orc.phi(r, eps) == pytest.approx(phi, rel=1e-15, abs=1e-15)
    assert orc.lap_phi(r, eps) == pytest.approx(lap, rel=4e-15)
    assert orc.lphi(r, kappa, eps) == pytest.approx(lphi, rel=4e-15)


def _fd_laplacian(fun, x, h):
    """4th-order central differences along each axis."""
    acc = 0.0
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        acc += (-fun(x + 2 * e) + 16 * fun(x + e) - 30 * fun(x) + 16 * fun(x - e) - fun(x - 2 * e)) / (12 * h * h)
    return acc


@pytest.mark.parametrize("eps", [0.5, 2.0, 6.0])
def test_lap_phi_is_laplacian_of_phi(orc, eps):
    rng = np.random.default_rng(5)
    c = rng.random(3)
    for _ in range(20):
        x = c + rng.normal(size=3) * (0.3 / eps)
        r = float(np.linalg.norm(x - c))
        fd = _fd_laplacian(lambda p: orc.phi(float(np.linalg.norm(p - c)), eps), x, 1e-3 / eps)
        assert orc.lap_phi(r, eps) == pytest.approx(fd, rel=1e-7)


def test_diagonal_entries(orc):
    # A_ii = Lap phi(0) + kappa^2 phi(0) = 3 eps^2 + kappa^2 on interior rows, phi(0) = 1 on boundary rows
    p = I.cube_scaled(40, 24, kappa=7.0, eps=3.0, ell=5)
    A = orc.assemble(p.nodes, p.n_int, p.kappa, p.eps)
    d = np.diag(A)
    assert np.all(d[: p.n_int] == 3 * 9.0 + 49.0)
    assert np.all(d[p.n_int:] == 1.0)


def test_rigid_motion_invariance(orc):
    p = I.cube_scaled(50, 30, kappa=4.0, eps=2.5, ell=5)
    X = p.nodes
    A = orc.assemble(X, p.n_int, p.kappa, p.eps)
    th = 0.7
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    ph = -1.1
    Rx = np.array([[1, 0, 0], [0, math.cos(ph), -math.sin(ph)], [0, math.sin(ph), math.cos(ph)]])
    Y = X @ (Rz @ Rx).T + np.array([0.3, -2.0, 1.5])
    B = orc.assemble(Y, p.n_int, p.kappa, p.eps)
    assert np.max(np.abs(A - B) / np.abs(A)) < 1e-13


def test_interior_rows_apply_helmholtz_operator(orc):
    # Row i of H applied to coefficients c equals (Lap + kappa^2) of the expansion
    # u(x) = sum_j c_j phi(|x - X_j|) at X_i (eqs. (4), (8)).
    p = I.cube_scaled(12, 10, kappa=3.0, eps=1.5, ell=5)
    X = p.nodes
    c = I.random_vector(p.n, 3)
    A = orc.assemble(X, p.n_int, p.kappa, p.eps)

    def u(x):
        return float(sum(c[j] * orc.phi(float(np.linalg.norm(x - X[j])), p.eps) for j in range(p.n)))

    for i in range(p.n_int):
        fd = _fd_laplacian(u, X[i], 2e-3) + p.kappa ** 2 * u(X[i])
        assert (A[i] @ c) == pytest.approx(fd, rel=1e-6, abs=1e-6 * np.abs(A[i]) @ np.abs(c))
    for i in range(p.n_int, p.n):
        assert (A[i] @ c) == pytest.approx(u(X[i]), rel=1e-13)


@pytest.mark.parametrize("eps", [0.8, 3.0])
def test_mq_matrix_has_one_positive_eigenvalue(orc, eps):
    # For pairwise distinct nodes the MQ matrix B is conditionally negative
    # definite of order 1 (c^T B c < 0 when sum c = 0) and has positive entries,
    # hence exactly one positive eigenvalue (the paper's Theorem on CPD(1)
    # states the sign the other way round).
    X = I.random_nodes_cube(200, 17)
    B = orc.interp_matrix(X, X, eps)
    assert np.allclose(B, B.T)
    ev = np.linalg.eigvalsh(B)
    assert int(np.sum(ev > 0)) == 1
    rng = np.random.default_rng(3)
    for _ in range(5):
        c = rng.normal(size=200)
        c -= c.mean()
        assert c @ B @ c < 0


def test_interp_matrix_reproduces_data(orc):
    # Interpolation (eq. (5)): coefficients solving B a = g reproduce g at the nodes via eval_u.
    X = I.random_nodes_cube(60, 9)
    eps = 3.0
    B = orc.interp_matrix(X, X, eps)
    g = np.sin(X[:, 0]) + X[:, 1] * X[:, 2]
    a = np.linalg.solve(B, g)
    u = orc.eval_u(X, eps, a, X)
    assert np.max(np.abs(u - g)) < 1e-8


def test_eval_unit_coefficient_is_kernel(orc):
    X = I.random_nodes_cube(30, 4)
    P = I.random_nodes_cube(7, 5)
    eps = 2.0
    for j in (0, 11, 29):
        e = np.zeros(30)
        e[j] = 1.0
        u = orc.eval_u(X, eps, e, P)
        ref = np.sqrt(1.0 + eps * eps * np.sum((P - X[j]) ** 2, axis=1))
        assert np.max(np.abs(u - ref) / ref) < 1e-15


@pytest.mark.parametrize("which", ["cube", "plane"])
def test_manufactured_solution_laplacian(which):
    kappa = 30.0
    man = I.Manufactured("cube", I.u_cube_sines, 25.0) if which == "cube" else \
        I.Manufactured("plane", I.u_plane_wave(kappa), kappa * kappa)
    rng = np.random.default_rng(8)
    h = 1e-3 if which == "cube" else 1e-4
    for _ in range(10):
        x = rng.random(3)
        fun = lambda p: float(man.u(p[None, :])[0])
        fd = _fd_laplacian(fun, x, h)
        assert fd == pytest.approx(-man.k2 * fun(x), rel=1e-6, abs=1e-6 * man.k2)


def test_workload_shapes():
    p = I.cube_small()
    assert (p.n_int, p.n_bnd, p.kappa, p.eps, p.ell) == (1200, 600, 5.0, 2.0, 60)
    assert np.all(p.f_int == 0.0)  # kappa^2 = 25 = |k|^2 of the manufactured u
    faces = p.x_bnd
    on_face = np.any((faces == 0.0) | (faces == 1.0), axis=1)
    assert np.all(on_face)
    assert np.all((p.x_int > 0) & (p.x_int < 1))
    b = I.sphere_fibonacci(1000)
    assert np.allclose(np.linalg.norm(b, axis=1), 1.0)
    x = I.ball_interior_uniform(500, 1)
    assert np.all(np.linalg.norm(x, axis=1) < 1.0)
