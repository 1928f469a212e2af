"""Host build of the fast projected SVD (csrc/msvd.hpp) checked on the CPU.

The device path (svd_kernels.hip) computes each singular value of C_l by
multisection on the inertia of B^T B - x I, each pair of singular vectors
by twisted factorisations, and orthogonalises them symmetrically; an
acceptance test sends problems it does not resolve to the QR iteration.
Here the same scalar recurrences are compiled with g++ and run in the
kernels' order.  References: LAPACK (numpy) for the values, f~ and the
projected Tikhonov solution; the host build of the QR iteration
(bidiag_svd.hpp) for the same quantities to rounding; and a 40-digit mpmath
computation of a tiny singular value that dense SVDs resolve only to about
1e-8 relative.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "_build", "msvd_host.so")
OUT_QR = os.path.join(ROOT, "_build", "bsvd_host_for_msvd.so")
EPS = np.finfo(float).eps
pd = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def msvd():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    subprocess.check_call(["g++", "-O2", "-shared", "-fPIC", "-o", OUT, os.path.join(HERE, "host", "msvd_host.cpp")])
    L = ctypes.CDLL(OUT)
    L.msvd_host.argtypes = [pd, pd, ctypes.c_int, pd, pd, pd, ctypes.POINTER(ctypes.c_int), pd]
    L.msvd_host.restype = ctypes.c_int

    def run(alpha, beta):
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        beta = np.ascontiguousarray(beta, dtype=np.float64)
        l = len(alpha)
        sv, ft, V = np.zeros(l), np.zeros(l + 1), np.zeros((l, l))
        rounds = ctypes.c_int()
        orth = np.zeros(3)
        st = L.msvd_host(alpha.ctypes.data_as(pd), beta.ctypes.data_as(pd), l, sv.ctypes.data_as(pd),
                         ft.ctypes.data_as(pd), V.ctypes.data_as(pd), ctypes.byref(rounds), orth.ctypes.data_as(pd))
        return st, sv, ft, V.T.copy(), rounds.value, orth

    return run


@pytest.fixture(scope="module")
def qr():
    subprocess.check_call(["g++", "-O2", "-shared", "-fPIC", "-o", OUT_QR, os.path.join(HERE, "host", "bsvd_host.cpp")])
    L = ctypes.CDLL(OUT_QR)
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
        assert st == 0
        return sv, ft, V.T.copy()

    return run


def _C(a, b):
    l = len(a)
    C = np.zeros((l + 1, l))
    for j in range(l):
        C[j, j] = a[j]
        C[j + 1, j] = b[j + 1]
    return C


def _y(V, sv, ft, lam):
    return V @ (sv / (sv ** 2 + lam ** 2) * ft[: len(sv)])


@pytest.mark.parametrize("l,seed", [(1, 0), (2, 1), (3, 2), (17, 3), (60, 4), (200, 5)])
def test_random_bidiagonal_against_lapack(msvd, l, seed):
    rng = np.random.default_rng(seed)
    a = rng.random(l) + 0.1
    b = np.concatenate([[2.0], rng.random(l) + 0.1])
    st, sv, ft, V, rounds, orth = msvd(a, b)
    assert st == 0, orth
    assert rounds <= 12
    C = _C(a, b)
    U, s, Vt = np.linalg.svd(C)
    big = s >= 1e-2 * s[0]
    assert np.max(np.abs(sv[big] - s[big]) / s[big]) < 1e-13
    assert np.max(np.abs(sv - s)) < 4 * l * EPS * s[0]
    assert np.all(np.diff(sv) <= 0)
    assert np.max(np.abs(np.abs(ft) - 2.0 * np.abs(U[0, :]))[np.r_[big, True]]) < 1e-12
    # the symmetric correction: orthonormal to rounding
    assert np.max(np.abs(V.T @ V - np.eye(l))) < 1e-14
    assert np.sum(ft ** 2) == pytest.approx(4.0, rel=1e-14)
    lam = s[min(3, l - 1)]
    rhs = np.zeros(2 * l + 1)
    rhs[0] = 2.0
    yls = np.linalg.lstsq(np.vstack([C, lam * np.eye(l)]), rhs, rcond=None)[0]
    assert np.linalg.norm(_y(V, sv, ft, lam) - yls) <= 1e-12 * np.linalg.norm(yls)


@pytest.mark.parametrize("l,seed", [(40, 11), (150, 12)])
def test_matches_qr_iteration(msvd, qr, l, seed):
    # a decaying spectrum like that of a Golub-Kahan run on an ill-posed operator
    rng = np.random.default_rng(seed)
    a = np.logspace(0, -6, l) * (1.0 + 0.3 * rng.random(l))
    b = np.concatenate([[1.0], np.logspace(-0.3, -6.3, l) * (1.0 + 0.3 * rng.random(l))])
    st, sv, ft, V, rounds, orth = msvd(a, b)
    assert st == 0, orth
    s2, f2, V2 = qr(a, b)
    assert np.max(np.abs(sv - s2) / s2) < 64 * EPS
    assert np.max(np.abs(np.abs(ft) - np.abs(f2))) < 1e-13 * b[0]
    for lam in (s2[0] * 1e-2, s2[l // 3], s2[-1] * 10):
        y, y2 = _y(V, sv, ft, lam), _y(V2, s2, f2, lam)
        assert np.linalg.norm(y - y2) <= 1e-10 * np.linalg.norm(y2)


def test_graded_and_zero_beta(msvd):
    l = 50
    a = np.logspace(0, -14, l)
    b = np.concatenate([[3.0], np.logspace(-1, -15, l)])
    st, sv, ft, V, rounds, orth = msvd(a, b)
    assert st == 0
    s = np.linalg.svd(_C(a, b), compute_uv=False)
    assert np.max(np.abs(sv - s) / s) < 1e-12
    b2 = b.copy()
    b2[-1] = 0.0  # beta_{l+1} = 0: f~_{l+1} = 0 exactly
    st, sv, ft, V, rounds, orth = msvd(a, b2)
    assert st == 0 and ft[l] == 0.0


def test_tiny_singular_value_high_relative_accuracy(msvd):
    mp = pytest.importorskip("mpmath")
    rng = np.random.default_rng(0)
    for l in (1, 2, 3, 10, 60, 200, 300):  # same draws as the QR iteration's test
        a = rng.random(l) + 0.1
        b = np.concatenate([[2.0], rng.random(l) + 0.1])
    st, sv, ft, V, rounds, orth = msvd(a, b)
    assert st == 0
    mp.mp.dps = 40
    l = len(a)
    A = [mp.mpf(v) for v in a]
    B = [mp.mpf(v) for v in b]
    dg = [A[j] ** 2 + B[j + 1] ** 2 for j in range(l)]
    od = [B[j + 1] * A[j + 1] for j in range(l - 1)]

    def tri_solve(rhs):
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
    for _ in range(8):
        x = tri_solve(x)
        nx = mp.sqrt(sum(v * v for v in x))
        x = [v / nx for v in x]
    Cx = [A[0] * x[0]] + [B[j] * x[j - 1] + (A[j] * x[j] if j < l else 0) for j in range(1, l + 1)]
    smin = mp.sqrt(sum(v * v for v in Cx))
    u1 = Cx[0] / smin
    assert float(abs(mp.mpf(sv[-1]) - smin) / smin) < 1e-13
    assert abs(abs(ft[-2]) - abs(float(2 * u1))) < 1e-13


def test_close_pairs_are_accepted_and_orthogonal(msvd, qr):
    # two weakly coupled copies of a block, the second scaled by 1 + 1e-5:
    # three pairs of singular values at relative gap 1e-5, whose vectors the
    # data fix to about eps / 1e-5; accepted, orthonormal after the
    # correction, and the projected solutions agree with the QR iteration's
    blk_a = np.array([1.0, 0.7, 0.4])
    blk_b = np.array([0.6, 0.3])
    q = 1.0 + 1e-5
    a = np.concatenate([blk_a, q * blk_a])
    b = np.concatenate([[1.0], blk_b, [1e-8], q * blk_b, [0.2]])
    st, sv, ft, V, rounds, orth = msvd(a, b)
    assert st == 0, orth
    assert np.max(np.abs(V.T @ V - np.eye(6))) < 1e-14
    s2, f2, V2 = qr(a, b)
    assert np.max(np.abs(sv - s2) / s2) < 64 * EPS
    for lam in (0.05, 0.5):
        y, y2 = _y(V, sv, ft, lam), _y(V2, s2, f2, lam)
        assert np.linalg.norm(y - y2) <= 1e-9 * np.linalg.norm(y2)


def test_exact_cluster_is_rejected(msvd):
    # C_l made of two identical decoupled blocks (beta = 0 between them):
    # every singular value is double, the twisted vectors are not defined,
    # and the acceptance test sends the problem to the QR iteration
    blk_a = np.array([1.0, 0.7, 0.4])
    blk_b = np.array([0.6, 0.3, 0.0])  # each block ends in a zero subdiagonal
    a = np.concatenate([blk_a, blk_a])
    b = np.concatenate([[1.0], blk_b, blk_b])
    st, sv, ft, V, rounds, orth = msvd(a, b)
    assert st == 2
