"""Host build of the band reduction of the block projected matrix
(csrc/band.hpp) checked on the CPU against LAPACK (numpy).

C, (l + 1) s x l s, has the structure of the block Golub-Kahan process:
lower triangular s x s blocks on the diagonal, upper triangular blocks below
them.  The bulge chase of C^T to a bidiagonal runs in the device kernels'
pipelined step order; it must give the same result, bit for bit, as the
sweeps run one after another, keep the singular values, and, with the data
through the right reflectors and the solutions through the left ones, give
the Tikhonov solutions of min ||C y - b_k||^2 + lambda^2 ||y||^2 and the
projected data f~ = U^T b_k of the block solve (up to the signs of the
singular vectors).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "_build", "band_host.so")
pd = ctypes.POINTER(ctypes.c_double)
pi = ctypes.POINTER(ctypes.c_int)


@pytest.fixture(scope="module")
def lib():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    subprocess.check_call(["g++", "-O2", "-shared", "-fPIC", "-o", OUT, os.path.join(HERE, "host", "band_host.cpp")])
    L = ctypes.CDLL(OUT)
    L.band_reduce.argtypes = [pd, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, pd, pd, pd,
                              pd, pi]
    L.band_reduce.restype = ctypes.c_int
    L.band_data.argtypes = [pd, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, pd, pi, ctypes.c_int, pd, pd,
                            pd, pd]
    L.band_solution.argtypes = [pd, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, pd, pi, ctypes.c_int]
    return L


def _p(a):
    return a.ctypes.data_as(pd)


def block_c(ell, s, seed, decay=0.05):
    """A C with the block Golub-Kahan structure and a decaying spectrum."""
    rng = np.random.default_rng(seed)
    N, m = ell * s, (ell + 1) * s
    C = np.zeros((m, N))
    for j in range(ell):
        sc = np.exp(-decay * j * s)
        D = np.tril(rng.standard_normal((s, s))) * sc
        D[np.diag_indices(s)] = np.abs(D[np.diag_indices(s)]) + sc
        E = np.triu(rng.standard_normal((s, s))) * sc
        C[j * s:(j + 1) * s, j * s:(j + 1) * s] = D
        C[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s] = E
    E1 = np.triu(rng.standard_normal((s, s)))
    E1[np.diag_indices(s)] = np.abs(E1[np.diag_indices(s)]) + 1.0
    return C, E1


def reduce(lib, C, s, pipelined):
    m, N = C.shape
    C = np.ascontiguousarray(C)
    nt = lib.band_ntasks_total(N, m, s)
    T = lib.band_nsteps(N, m, s)
    d, e = np.zeros(N), np.zeros(N)
    RR, LL = np.zeros((max(nt, 1), s + 1)), np.zeros((max(nt, 1), s + 1))
    toff = np.zeros(T + 1, dtype=np.int32)
    T2 = lib.band_reduce(_p(C), N, N, m, s, pipelined, _p(d), _p(e), _p(RR), _p(LL), toff.ctypes.data_as(pi))
    assert T2 == T
    return d, e, RR, LL, toff, T


CASES = [(1, 2, 0), (3, 2, 1), (7, 16, 2), (25, 16, 3), (9, 5, 4), (40, 3, 5), (12, 7, 6), (2, 16, 7)]


@pytest.mark.parametrize("ell,s,seed", CASES)
def test_pipelined_equals_sequential_and_keeps_singular_values(lib, ell, s, seed):
    C, _ = block_c(ell, s, seed)
    a = reduce(lib, C, s, 1)
    b = reduce(lib, C, s, 0)
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    d, e = a[0], a[1]
    N = ell * s
    Bt = np.zeros((N, N + 1))
    Bt[np.arange(N), np.arange(N)] = d
    Bt[np.arange(N), np.arange(N) + 1] = e
    s1 = np.linalg.svd(C, compute_uv=False)
    s2 = np.linalg.svd(Bt, compute_uv=False)
    assert np.max(np.abs(s1 - s2)) <= 64 * N * np.finfo(float).eps * s1[0]


def test_schedule_tasks_of_a_step_are_disjoint(lib):
    # each task's footprint: right reflector rows r0..r1 x cols c0..c1, left
    # reflector rows c0..r1 x cols c0..ce; tasks of one step must not share an entry
    for N, s in [(100, 4), (64, 16), (45, 3), (30, 2)]:
        m = N + s
        T = lib.band_nsteps(N, m, s)
        lag = 3

        def ntasks(i):
            if Mc_3(i) < 0:
                return 0
            t1 = (m - 3 - i) // s
            t2 = (N - 2 - i) // s + 1 if N - 2 - i >= 0 else 0
            return min(t1, t2) + 1

        def Mc_3(i):
            return m - 3 - i

        for step in range(T):
            cells = set()
            for i in range(min(N, m - 1)):
                t = step - lag * i
                if t < 0 or t >= ntasks(i):
                    continue
                c0 = i + 1 + t * s
                c1 = min(c0 + s - 1, m - 1)
                r0 = i if t == 0 else c0 - s
                r1 = min(c1, N - 1)
                ce = min(c1 + s, m - 1)
                mine = {(r, c) for r in range(r0, r1 + 1) for c in range(c0, c1 + 1)}
                mine |= {(r, c) for r in range(c0, r1 + 1) for c in range(c0, ce + 1)}
                assert not (cells & mine), (N, s, step, i, t)
                cells |= mine


@pytest.mark.parametrize("ell,s,seed", [(7, 16, 11), (25, 16, 12), (9, 5, 13), (30, 2, 14)])
def test_projected_solutions_through_the_reflectors(lib, ell, s, seed):
    C, E1 = block_c(ell, s, seed)
    m, N = C.shape
    d, e, RR, LL, toff, T = reduce(lib, C, s, 1)
    X = np.zeros((m, s))
    X[:s] = E1
    du, eu = np.zeros(N), np.zeros(N)
    lib.band_data(_p(X), s, N, m, s, _p(RR), toff.ctypes.data_as(pi), T, _p(d), _p(e), _p(du), _p(eu))
    assert np.all(du >= 0.0)
    B = np.diag(du) + np.diag(eu[:-1], 1)
    Ub, sb, Vbt = np.linalg.svd(B)
    Ft = Ub.T @ X[:N]
    U, sv, Vt = np.linalg.svd(C, full_matrices=False)
    b = np.zeros((m, s))
    b[:s] = E1
    Ft_ref = U.T @ b
    assert np.max(np.abs(sb - sv)) <= 64 * N * np.finfo(float).eps * sv[0]
    big = sv > 1e-6 * sv[0]
    assert np.max(np.abs(np.abs(Ft[big]) - np.abs(Ft_ref[big]))) <= 1e-11 * np.abs(E1).max()
    # s_perp = ||b||^2 - ||f~||^2 alike
    sp = np.sum(b * b, axis=0) - np.sum(Ft * Ft, axis=0)
    sp_ref = np.sum(b * b, axis=0) - np.sum(Ft_ref * Ft_ref, axis=0)
    assert np.max(np.abs(sp - sp_ref)) <= 1e-12 * np.sum(b * b, axis=0).max()
    for lam in (sv[0] * 1e-2, sv[N // 3], sv[-1] * 3):
        Yh = np.ascontiguousarray(Vbt.T @ ((sb / (sb ** 2 + lam ** 2))[:, None] * Ft))
        lib.band_solution(_p(Yh), s, N, m, s, _p(LL), toff.ctypes.data_as(pi), T)
        Y_ref = Vt.T @ ((sv / (sv ** 2 + lam ** 2))[:, None] * Ft_ref)
        assert np.linalg.norm(Yh - Y_ref) <= 1e-10 * np.linalg.norm(Y_ref)


def test_one_source_is_already_bidiagonal(lib):
    # s = 1: C is the lower bidiagonal of the scalar process; no tasks, d = alpha, e_j = beta_{j+1}
    rng = np.random.default_rng(3)
    ell = 12
    a, bb = rng.random(ell) + 0.1, rng.random(ell) + 0.1
    C = np.zeros((ell + 1, ell))
    C[np.arange(ell), np.arange(ell)] = a
    C[np.arange(ell) + 1, np.arange(ell)] = bb
    d, e, RR, LL, toff, T = reduce(lib, C, 1, 1)
    assert T == 0
    assert np.array_equal(d, a) and np.array_equal(e, bb)
