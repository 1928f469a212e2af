"""Host build of the device projected-SVD core (csrc/bidiag_svd.hpp) checked on the CPU.

The same scalar code runs on the GPU in k_bidiag_svd; here it is compiled
with g++ and driven the way the kernel drives it.  References: LAPACK
(numpy) for singular values, f~ and the projected Tikhonov solution, and a
40-digit mpmath computation for a tiny singular value that dense SVDs
(LAPACK and the oracle's one-sided Jacobi) resolve only to ~1e-8 relative.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "host", "bsvd_host.cpp")
OUT = os.path.join(ROOT, "_build", "bsvd_host.so")


@pytest.fixture(scope="module")
def bsvd():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    subprocess.check_call(["g++", "-O2", "-shared", "-fPIC", "-o", OUT, SRC])
    L = ctypes.CDLL(OUT)
    pd = ctypes.POINTER(ctypes.c_double)
    L.bsvd_host.argtypes = [pd, pd, ctypes.c_int, pd, pd, pd, ctypes.POINTER(ctypes.c_long)]
    L.bsvd_host.restype = ctypes.c_int

    def run(alpha, beta):
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        beta = np.ascontiguousarray(beta, dtype=np.float64)
        l = len(alpha)
        sv, ft, V = np.zeros(l), np.zeros(l + 1), np.zeros((l, l))
        it = ctypes.c_long()
        st = L.bsvd_host(alpha.ctypes.data_as(pd), beta.ctypes.data_as(pd), l, sv.ctypes.data_as(pd),
                         ft.ctypes.data_as(pd), V.ctypes.data_as(pd), ctypes.byref(it))
        return st, sv, ft, V.T.copy(), it.value

    return run


def _C(a, b):
    l = len(a)
    C = np.zeros((l + 1, l))
    for j in range(l):
        C[j, j] = a[j]
        C[j + 1, j] = b[j + 1]
    return C


@pytest.mark.parametrize("l,seed", [(1, 0), (2, 1), (3, 2), (17, 3), (60, 4), (200, 5)])
def test_random_bidiagonal_against_lapack(bsvd, l, seed):
    rng = np.random.default_rng(seed)
    a = rng.random(l) + 0.1
    b = np.concatenate([[2.0], rng.random(l) + 0.1])
    st, sv, ft, V, it = bsvd(a, b)
    assert st == 0
    C = _C(a, b)
    U, s, Vt = np.linalg.svd(C)
    # LAPACK's dense SVD is accurate to ~eps * s_1 in absolute terms only
    big = s >= 1e-2 * s[0]
    assert np.max(np.abs(sv[big] - s[big]) / s[big]) < 1e-13
    assert np.max(np.abs(sv - s)) < 4 * l * np.finfo(float).eps * s[0]
    assert np.all(np.diff(sv) <= 0)
    assert np.max(np.abs(np.abs(ft) - 2.0 * np.abs(U[0, :]))[np.r_[big, True]]) < 1e-12
    assert np.max(np.abs(V.T @ V - np.eye(l))) < 1e-13
    lam = s[min(3, l - 1)]
    y = V @ (sv / (sv ** 2 + lam ** 2) * ft[:l])
    rhs = np.zeros(2 * l + 1)
    rhs[0] = 2.0
    yls = np.linalg.lstsq(np.vstack([C, lam * np.eye(l)]), rhs, rcond=None)[0]
    assert np.linalg.norm(y - yls) <= 1e-12 * np.linalg.norm(yls)


def test_graded_and_zero_beta(bsvd):
    l = 50
    a = np.logspace(0, -14, l)
    b = np.concatenate([[3.0], np.logspace(-1, -15, l)])
    st, sv, ft, V, it = bsvd(a, b)
    assert st == 0
    s = np.linalg.svd(_C(a, b), compute_uv=False)
    assert np.max(np.abs(sv - s) / s) < 1e-12
    b2 = b.copy()
    b2[-1] = 0.0  # beta_{l+1} = 0: f~_{l+1} = 0 exactly
    st, sv, ft, V, it = bsvd(a, b2)
    assert st == 0 and ft[l] == 0.0


def test_tiny_singular_value_high_relative_accuracy(bsvd):
    mp = pytest.importorskip("mpmath")
    rng = np.random.default_rng(0)
    for l in (1, 2, 3, 10, 60, 200, 300):  # same draws as the exploratory case
        a = rng.random(l) + 0.1
        b = np.concatenate([[2.0], rng.random(l) + 0.1])
    st, sv, ft, V, it = bsvd(a, b)
    assert st == 0
    mp.mp.dps = 40
    l = len(a)
    A = [mp.mpf(v) for v in a]
    B = [mp.mpf(v) for v in b]
    # C^T C is tridiagonal: diagonal a_j^2 + b_{j+1}^2, off-diagonal b_{j+1} a_{j+1}
    dg = [A[j] ** 2 + B[j + 1] ** 2 for j in range(l)]
    od = [B[j + 1] * A[j + 1] for j in range(l - 1)]

    def tri_solve(rhs):  # LDL^T (Thomas) on the SPD tridiagonal
        dd, yy = [dg[0]], [rhs[0]]
        for j in range(1, l):
            m = od[j - 1] / dd[j - 1]
            dd.append(dg[j] - m * od[j - 1])
            yy.append(rhs[j] - m * yy[j - 1])
        x = [mp.mpf(0)] * l
        x[l - 1] = yy[l - 1] / dd[l - 1]
        for j in range(l - 2, -1, -1):
            x[j] = (yy[j] - od[j] * x[j + 1]) / dd[j]
        return x

    x = [mp.mpf(1)] * l
    for _ in range(8):  # inverse iteration for the smallest eigenvalue of C^T C
        x = tri_solve(x)
        nx = mp.sqrt(sum(v * v for v in x))
        x = [v / nx for v in x]
    Cx = [A[0] * x[0]] + [B[j] * x[j - 1] + (A[j] * x[j] if j < l else 0) for j in range(1, l + 1)]
    smin = mp.sqrt(sum(v * v for v in Cx))
    u1 = Cx[0] / smin
    assert float(abs(mp.mpf(sv[-1]) - smin) / smin) < 1e-13
    assert abs(abs(ft[-2]) - abs(float(2 * u1))) < 1e-13
