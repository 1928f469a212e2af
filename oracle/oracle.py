"""Plain FP64 CPU oracle for the GKB / Ine-TSVD / HKT path.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg, never by the library.  It shares no code
with the HIP implementation.

The O(N^2) work (matrix entries, products, Golub-Kahan bidiagonalisation,
the small dense Jacobi SVD, lift and evaluation) is plain C in
``mqh_oracle.c``; the small projected-problem steps (filter factors,
projected residual/solution norms, GCV, L-curve curvature, parameter choice,
filtered solutions) are written here in numpy, each next to the equation of
the paper it follows (Efficient Krylov-Regularization Solvers for
Multiquadric RBF Discretizations of the 3D Helmholtz Equation, Sections
2-3).

Readings of points the paper leaves open (each is listed with its reason in
the design notes):
* grid for lambda: J log-spaced points on [max(s_l, 16 eps_mach s_1), s_1]
  (s = projected singular values), then golden-section refinement of
  log(lambda) inside the bracketing cell; ties go to the larger lambda and
  an argmin at a grid end is returned as is with an edge flag;
* L-curve corner: maximum of the signed curvature of (log rho, log eta)
  over the grid without its two end points, derivatives analytic;
* Ine-TSVD rank: minimiser of the projected TSVD-GCV function
  G(k) = (sum_{i>k} f~_i^2 + f~_{l+1}^2) / ((l+1) - k)^2, k = 1..floor(l/2),
  ties to the smaller k;
* the final Tikhonov solve of Algorithm 4 is done in the SVD-filter form,
  equal in exact arithmetic to the normal equations it prints;
* weighted GCV (opt-in): the projected GCV with the trace term scaled by a
  weight omega, rho_l^2 / ((l+1) - omega sum_i phi_i)^2 (omega = 1 is
  eq. (30)); for the rank, ((l+1) - omega k)^2;
* LSQR early stopping (Section 3.4): the k-th iterate is Z_k y_k with
  y_k = argmin ||C_k y - beta_1 e_1||; the stopping index minimises the
  GCV function of the Krylov filter, rho_k^2 / (n - k)^2 (its influence
  matrix is a rank-k orthogonal projector), or sits at the corner of the
  discrete L-curve (log rho_k, log eta_k): the maximum signed Menger
  curvature over consecutive triples, traversed from large to small k.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mqh_oracle.c")
_LIB = os.path.join(_HERE, "libmqh_oracle.so")

EPS_MACH = np.finfo(np.float64).eps

# flag bits reported by solve()
FLAG_BREAKDOWN = 1
FLAG_GCV_AT_EDGE = 2
FLAG_LCURVE_AT_EDGE = 4

METHOD_INE_TSVD = 0
METHOD_HKT = 1
METHOD_LSQR = 2
RULE_GCV = 0
RULE_LCURVE = 1
RULE_FIXED = 2
RULE_WGCV = 3


def build(force: bool = True) -> str:
    """Compile mqh_oracle.c with gcc (-O2, OpenMP, no fast-math) into libmqh_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_d = ctypes.c_double
_i64 = ctypes.c_int64
_pd = ctypes.POINTER(ctypes.c_double)
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pint = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_phi.restype = _d
        L.orc_phi.argtypes = [_d, _d]
        L.orc_lap_phi.restype = _d
        L.orc_lap_phi.argtypes = [_d, _d]
        L.orc_lphi.restype = _d
        L.orc_lphi.argtypes = [_d, _d, _d]
        L.orc_entry.restype = _d
        L.orc_entry.argtypes = [_pd, _i64, _i64, _i64, _d, _d]
        L.orc_assemble.restype = None
        L.orc_assemble.argtypes = [_pd, _i64, _i64, _d, _d, _pd]
        L.orc_interp_matrix.restype = None
        L.orc_interp_matrix.argtypes = [_pd, _i64, _pd, _i64, _d, _pd]
        L.orc_apply.restype = None
        L.orc_apply.argtypes = [_pd, _pd, _i64, _i64, _d, _d, ctypes.c_int, _pd, _pd]
        L.orc_apply_sampled.restype = None
        L.orc_apply_sampled.argtypes = [_pd, _i64, _i64, _d, _d, ctypes.c_int, _pd, _pi64, _i64, _pd]
        L.orc_gkb.restype = _i64
        L.orc_gkb.argtypes = [_pd, _pd, _i64, _i64, _d, _d, _pd, _i64, ctypes.c_int, _pd, _pd, _pd, _pd, _pint]
        L.orc_row_scale.restype = None
        L.orc_row_scale.argtypes = [_pd, _i64, _i64, _d, _d, _pd]
        L.orc_apply_rs.restype = None
        L.orc_apply_rs.argtypes = [_pd, _pd, _i64, _i64, _d, _d, _pd, ctypes.c_int, _pd, _pd]
        L.orc_apply_sampled_rs.restype = None
        L.orc_apply_sampled_rs.argtypes = [_pd, _i64, _i64, _d, _d, _pd, ctypes.c_int, _pd, _pi64, _i64, _pd]
        L.orc_gkb_rs.restype = _i64
        L.orc_gkb_rs.argtypes = [_pd, _pd, _i64, _i64, _d, _d, _pd, _pd, _i64, ctypes.c_int, _pd, _pd, _pd, _pd,
                                 _pint]
        L.orc_jacobi_svd.restype = ctypes.c_int
        L.orc_jacobi_svd.argtypes = [_pd, _i64, _i64, _pd, _pd, _pd]
        L.orc_proj_svd.restype = ctypes.c_int
        L.orc_proj_svd.argtypes = [_pd, _pd, _i64, _pd, _pd, _pd]
        L.orc_lift.restype = None
        L.orc_lift.argtypes = [_pd, _i64, _i64, _pd, _pd]
        L.orc_eval.restype = None
        L.orc_eval.argtypes = [_pd, _i64, _d, _pd, _pd, _i64, _pd]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(_pd)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------
# Kernel, entries, operator (C)
# --------------------------------------------------------------------------


def phi(r: float, eps: float) -> float:
    """MQ kernel sqrt(1 + eps^2 r^2) (eq. (3))."""
    return lib().orc_phi(float(r), float(eps))


def lap_phi(r: float, eps: float) -> float:
    """3-D Laplacian of the MQ kernel, eps^2 (3 + 2 eps^2 r^2) / (1 + eps^2 r^2)^{3/2}."""
    return lib().orc_lap_phi(float(r), float(eps))


def lphi(r: float, kappa: float, eps: float) -> float:
    """Helmholtz-applied kernel Lap(phi) + kappa^2 phi (eq. (8))."""
    return lib().orc_lphi(float(r), float(kappa), float(eps))


def assemble(X: np.ndarray, n_int: int, kappa: float, eps: float) -> np.ndarray:
    """Dense Kansa matrix A = [H; R] (eq. (10)), row-major n x n."""
    X = _c(X)
    n = X.shape[0]
    A = np.empty((n, n))
    lib().orc_assemble(_p(X), n, int(n_int), float(kappa), float(eps), _p(A))
    return A


def interp_matrix(P: np.ndarray, X: np.ndarray, eps: float) -> np.ndarray:
    """B_ij = phi(|P_i - X_j|) (eq. (5))."""
    P, X = _c(P), _c(X)
    B = np.empty((P.shape[0], X.shape[0]))
    lib().orc_interp_matrix(_p(P), P.shape[0], _p(X), X.shape[0], float(eps), _p(B))
    return B


def row_scale(X: np.ndarray, n_int: int, kappa: float, eps: float) -> np.ndarray:
    """d_i = 1 / A_ii: the row scaling D = diag(A)^{-1} of the stacked system A c = f (eq. (11)).

    Not in the paper (an opt-in equilibration of the interior and boundary
    rows); the scaled problem is (D A) c = D f."""
    X = _c(X)
    d = np.empty(X.shape[0])
    lib().orc_row_scale(_p(X), X.shape[0], int(n_int), float(kappa), float(eps), _p(d))
    return d


_row_scale_vector = row_scale


def apply(A: Optional[np.ndarray], X: np.ndarray, n_int: int, kappa: float, eps: float,
          x: np.ndarray, trans: bool = False, d: Optional[np.ndarray] = None) -> np.ndarray:
    """y = A x (trans False) or A^T x (trans True); A None evaluates entries on the fly.

    d: row scale of the entry-by-entry operator (y = D A x, A^T D x); a stored A
    is passed already scaled."""
    X, x = _c(X), _c(x)
    n = X.shape[0]
    y = np.empty(n)
    Ap = None if A is None else _p(_c(A))
    lib().orc_apply_rs(Ap, _p(X), n, int(n_int), float(kappa), float(eps), _p(None if d is None else _c(d)),
                       int(bool(trans)), _p(x), _p(y))
    return y


def apply_sampled(X: np.ndarray, n_int: int, kappa: float, eps: float, x: np.ndarray,
                  idx: np.ndarray, trans: bool = False, d: Optional[np.ndarray] = None) -> np.ndarray:
    """Selected outputs (A x)_idx or (A^T x)_idx, entry by entry (of D A when d is given)."""
    X, x = _c(X), _c(x)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.empty(idx.shape[0])
    lib().orc_apply_sampled_rs(_p(X), X.shape[0], int(n_int), float(kappa), float(eps),
                               _p(None if d is None else _c(d)), int(bool(trans)), _p(x),
                               idx.ctypes.data_as(_pi64), idx.shape[0], _p(out))
    return out


@dataclasses.dataclass
class GKBResult:
    W: np.ndarray  # n x (ell+1), columns w_1..w_{ell+1}
    Z: np.ndarray  # n x ell, columns z_1..z_ell
    alpha: np.ndarray  # alpha_1..alpha_ell
    beta: np.ndarray  # beta_1..beta_{ell+1}
    ell: int  # steps kept (ell_eff)
    flag: int  # 0, 1 (alpha breakdown), 2 (beta breakdown)


def gkb(A: Optional[np.ndarray], X: np.ndarray, n_int: int, kappa: float, eps: float, f: np.ndarray,
        ell: int, reorth: bool = True, d: Optional[np.ndarray] = None) -> GKBResult:
    """Algorithm 1 (Golub-Kahan bidiagonalisation) with full CGS2 reorthogonalisation.

    d: row scale of the entry-by-entry operator (the run is on D A; a stored
    A and f are passed already scaled)."""
    X, f = _c(X), _c(f)
    n = X.shape[0]
    W = np.zeros((ell + 1, n))  # row k is column w_{k+1} (column-major storage)
    Z = np.zeros((ell, n))
    al = np.zeros(ell)
    be = np.zeros(ell + 1)
    flag = ctypes.c_int(0)
    Ap = None if A is None else _p(_c(A))
    le = lib().orc_gkb_rs(Ap, _p(X), n, int(n_int), float(kappa), float(eps), _p(None if d is None else _c(d)),
                          _p(f), int(ell), int(bool(reorth)), _p(W), _p(Z), _p(al), _p(be), ctypes.byref(flag))
    le = int(le)
    return GKBResult(W[: le + 1].T.copy(), Z[:le].T.copy(), al[:le].copy(), be[: le + 1].copy(), le,
                     int(flag.value))


def jacobi_svd(M: np.ndarray):
    """One-sided Jacobi SVD of a dense m x n matrix (m >= n): returns (s, U, V), s descending."""
    M = np.asarray(M, dtype=np.float64)
    m, n = M.shape
    assert m >= n
    Mc = np.ascontiguousarray(M.T)  # column-major copy (row k = column k)
    s = np.empty(n)
    U = np.empty((n, m))
    V = np.empty((n, n))
    sw = lib().orc_jacobi_svd(_p(Mc), m, n, _p(s), _p(U), _p(V))
    if sw < 0:
        raise RuntimeError("Jacobi SVD did not converge")
    return s, U.T.copy(), V.T.copy()


def bidiag_matrix(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """The (ell+1) x ell lower bidiagonal C_ell: diagonal alpha_1..alpha_ell, subdiagonal beta_2..beta_{ell+1}."""
    ell = len(alpha)
    C = np.zeros((ell + 1, ell))
    for j in range(ell):
        C[j, j] = alpha[j]
        C[j + 1, j] = beta[j + 1]
    return C


def proj_svd(alpha: np.ndarray, beta: np.ndarray):
    """SVD of C_ell and projected data f~ = U~^T(beta_1 e_1) (Algorithm 4 step 2).

    Returns (s[ell] descending, ftil[ell+1], V[ell x ell], columns v~_i)."""
    alpha, beta = _c(alpha), _c(beta)
    ell = alpha.shape[0]
    assert beta.shape[0] == ell + 1
    s = np.empty(ell)
    ft = np.empty(ell + 1)
    V = np.empty((ell, ell))
    sw = lib().orc_proj_svd(_p(alpha), _p(beta), ell, _p(s), _p(ft), _p(V))
    if sw < 0:
        raise RuntimeError("projected Jacobi SVD did not converge")
    return s, ft, V.T.copy()


def lift(Z: np.ndarray, y: np.ndarray) -> np.ndarray:
    """alpha = Z_ell y (Algorithm 2 step 5, Algorithm 4 last step)."""
    Zc = np.ascontiguousarray(np.asarray(Z, dtype=np.float64).T)  # column-major
    n, ell = Z.shape
    y = _c(y)
    out = np.empty(n)
    lib().orc_lift(_p(Zc), n, ell, _p(y), _p(out))
    return out


def eval_u(X: np.ndarray, eps: float, coef: np.ndarray, P: np.ndarray) -> np.ndarray:
    """u(P) = sum_j coef_j phi(|P - X_j|) (eq. (18))."""
    X, coef, P = _c(X), _c(coef), _c(P)
    u = np.empty(P.shape[0])
    lib().orc_eval(_p(X), X.shape[0], float(eps), _p(coef), _p(P), P.shape[0], _p(u))
    return u


# --------------------------------------------------------------------------
# Projected problem: filters, norms, GCV, L-curve (numpy)
# --------------------------------------------------------------------------


def tikh_filter(s: np.ndarray, lam: float) -> np.ndarray:
    """phi_i(lambda) = s_i^2 / (s_i^2 + lambda^2)  (Tikhonov filter factors, Section 3.2)."""
    s2 = s * s
    return s2 / (s2 + lam * lam)


def tikh_filter_complement(s: np.ndarray, lam: float) -> np.ndarray:
    """1 - phi_i(lambda), computed directly as lambda^2 / (s_i^2 + lambda^2)."""
    l2 = lam * lam
    return l2 / (s * s + l2)


def rho2_proj(s: np.ndarray, ftil: np.ndarray, lam: float) -> float:
    """rho_l^2 = sum_i (1 - phi_i)^2 f~_i^2 + f~_{l+1}^2  (eq. (28))."""
    ell = s.shape[0]
    c = tikh_filter_complement(s, lam)
    return float(np.sum((c * ftil[:ell]) ** 2) + ftil[ell] ** 2)


def eta2_proj(s: np.ndarray, ftil: np.ndarray, lam: float) -> float:
    """eta_l^2 = sum_i (phi_i / s_i)^2 f~_i^2  (eq. (29))."""
    ell = s.shape[0]
    ph = tikh_filter(s, lam)
    return float(np.sum((ph / s * ftil[:ell]) ** 2))


def gcv_proj(s: np.ndarray, ftil: np.ndarray, lam: float) -> float:
    """GCV_l(lambda) = rho_l^2 / ((l+1) - sum_i phi_i)^2  (eq. (30))."""
    ell = s.shape[0]
    den = (ell + 1) - float(np.sum(tikh_filter(s, lam)))
    return rho2_proj(s, ftil, lam) / (den * den)


def gcv_proj_weighted(s: np.ndarray, ftil: np.ndarray, lam: float, omega: float) -> float:
    """Weighted projected GCV: rho_l^2 / ((l+1) - omega sum_i phi_i)^2 (omega = 1 gives eq. (30))."""
    ell = s.shape[0]
    den = (ell + 1) - omega * float(np.sum(tikh_filter(s, lam)))
    return rho2_proj(s, ftil, lam) / (den * den)


def gcv_full(s: np.ndarray, fhat: np.ndarray, s_perp: float, n: int, lam: float) -> float:
    """GCV(lambda) of the full problem in SVD variables (eq. (25), Algorithm 3)."""
    c = tikh_filter_complement(s, lam)
    rho2 = float(np.sum((c * fhat) ** 2)) + s_perp
    den = n - float(np.sum(tikh_filter(s, lam)))
    return rho2 / (den * den)


def lcurve_curvature(s: np.ndarray, ftil: np.ndarray, lam: float) -> float:
    """Signed curvature of (x, y) = (log rho_l, log eta_l) as a function of t = log lambda.

    With phi_i' = d phi_i / dt = -2 phi_i psi_i (psi_i = 1 - phi_i):
      R  = rho^2,  R'  = sum 4 phi psi^2 f^2,       R'' = sum 8 f^2 phi psi^2 (2 phi - psi)
      E  = eta^2,  E'  = -sum 4 phi^2 psi f^2/s^2,  E'' = sum 8 f^2/s^2 phi^2 psi (2 psi - phi)
      x' = R'/(2R), x'' = (R''R - R'^2)/(2R^2), same for y from E, and
      kappa = (x' y'' - x'' y') / (x'^2 + y'^2)^{3/2}."""
    ell = s.shape[0]
    f2 = ftil[:ell] ** 2
    ph = tikh_filter(s, lam)
    ps = tikh_filter_complement(s, lam)
    R = float(np.sum(ps * ps * f2) + ftil[ell] ** 2)
    R1 = float(np.sum(4.0 * ph * ps * ps * f2))
    R2 = float(np.sum(8.0 * f2 * ph * ps * ps * (2.0 * ph - ps)))
    g2 = f2 / (s * s)
    E = float(np.sum(ph * ph * g2))
    E1 = float(np.sum(-4.0 * ph * ph * ps * g2))
    E2 = float(np.sum(8.0 * g2 * ph * ph * ps * (2.0 * ps - ph)))
    x1, x2 = R1 / (2 * R), (R2 * R - R1 * R1) / (2 * R * R)
    y1, y2 = E1 / (2 * E), (E2 * E - E1 * E1) / (2 * E * E)
    return (x1 * y2 - x2 * y1) / (x1 * x1 + y1 * y1) ** 1.5


def lambda_grid(s: np.ndarray, n_grid: int) -> np.ndarray:
    """Ascending log-spaced grid on [max(s_min, 16 eps_mach s_1), s_1].

    If that interval is empty (all s equal, e.g. ell = 1), the lower end is
    16 eps_mach s_1."""
    hi = float(s[0])
    lo = max(float(s[-1]), 16.0 * EPS_MACH * hi)
    if not lo < hi:
        lo = 16.0 * EPS_MACH * hi
    return np.exp(np.linspace(math.log(lo), math.log(hi), n_grid))


def golden_min(fun, a: float, b: float, tol: float = 1e-10, max_it: int = 200) -> float:
    """Golden-section search for a minimiser of fun on [a, b] (to |b - a| <= tol)."""
    g = (math.sqrt(5.0) - 1.0) / 2.0
    c = b - g * (b - a)
    d = a + g * (b - a)
    fc, fd = fun(c), fun(d)
    it = 0
    while abs(b - a) > tol and it < max_it:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = fun(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = fun(d)
        it += 1
    return 0.5 * (a + b)


def choose_lambda_gcv(s: np.ndarray, ftil: np.ndarray, n_grid: int = 200, refine: bool = True,
                      omega: float = 1.0):
    """lambda* = argmin_{lambda > 0} GCV_l(lambda) (Algorithm 4, GCV branch); with omega != 1
    the weighted GCV.

    Grid minimum first (ties -> larger lambda), then golden-section refinement
    of log(lambda) on the two cells around it.  Returns (lambda, gcv, at_edge, grid, values)."""
    def gcv_proj(s_, f_, lam_):  # noqa: F811 - the weighted form, eq. (30) at omega = 1
        return gcv_proj_weighted(s_, f_, lam_, omega)

    grid = lambda_grid(s, n_grid)
    vals = np.array([gcv_proj(s, ftil, lam) for lam in grid])
    k = n_grid - 1 - int(np.argmin(vals[::-1]))
    if k == 0 or k == n_grid - 1 or not refine:
        return float(grid[k]), float(vals[k]), (k == 0 or k == n_grid - 1), grid, vals
    t = golden_min(lambda tt: gcv_proj(s, ftil, math.exp(tt)), math.log(grid[k - 1]), math.log(grid[k + 1]))
    lam = math.exp(t)
    g = gcv_proj(s, ftil, lam)
    if g > vals[k]:  # refinement cannot be worse than the grid point
        lam, g = float(grid[k]), float(vals[k])
    return lam, g, False, grid, vals


def choose_lambda_lcurve(s: np.ndarray, ftil: np.ndarray, n_grid: int = 200):
    """L-curve corner: lambda of maximum signed curvature on the log grid, end points excluded.

    Returns (lambda, curvature, at_edge, grid, curvatures); at_edge is set
    when the maximum sits next to an excluded end point."""
    grid = lambda_grid(s, n_grid)
    kap = np.array([lcurve_curvature(s, ftil, lam) for lam in grid])
    inner = kap[1:-1]
    k = 1 + (len(inner) - 1 - int(np.argmax(inner[::-1])))
    return float(grid[k]), float(kap[k]), (k == 1 or k == n_grid - 2), grid, kap


def tsvd_gcv(s: np.ndarray, ftil: np.ndarray, k: int, omega: float = 1.0) -> float:
    """Projected TSVD-GCV: (sum_{i>k} f~_i^2 + f~_{l+1}^2) / ((l+1) - omega k)^2 (omega = 1 unless weighted)."""
    ell = s.shape[0]
    res = float(np.sum(ftil[k:ell] ** 2) + ftil[ell] ** 2)
    den = (ell + 1) - omega * k
    return res / (den * den)


def choose_rank(s: np.ndarray, ftil: np.ndarray, omega: float = 1.0) -> int:
    """Ine-TSVD rank k* (Algorithm 2 step 4): argmin of the projected TSVD-GCV over k = 1..max(1, floor(l/2))."""
    ell = s.shape[0]
    kmax = max(1, ell // 2)
    vals = [tsvd_gcv(s, ftil, k, omega) for k in range(1, kmax + 1)]
    return 1 + int(np.argmin(vals))


# --------------------------------------------------------------------------
# LSQR iterates and early stopping (Section 3.4)
# --------------------------------------------------------------------------


def lsqr_path(alpha: np.ndarray, beta: np.ndarray):
    """For k = 1..l: y_k = argmin_y ||C_k y - beta_1 e_1||_2 with C_k the leading (k+1) x k block of
    C_l, so that Z_k y_k is the k-th LSQR iterate and ||A Z_k y_k - f|| = ||C_k y_k - beta_1 e_1||
    (Section 3.4; eq. (26)).  Plain definition: one dense least-squares solve per k.

    Returns (rho[l], eta[l], Y) with rho_k = ||C_k y_k - beta_1 e_1||, eta_k = ||y_k|| and row k-1
    of Y holding y_k padded with zeros to length l."""
    alpha, beta = _c(alpha), _c(beta)
    ell = alpha.shape[0]
    C = bidiag_matrix(alpha, beta)
    rho = np.empty(ell)
    eta = np.empty(ell)
    Y = np.zeros((ell, ell))
    for k in range(1, ell + 1):
        Ck = C[: k + 1, :k]
        rhs = np.zeros(k + 1)
        rhs[0] = beta[0]
        y = np.linalg.lstsq(Ck, rhs, rcond=None)[0]
        rho[k - 1] = float(np.linalg.norm(Ck @ y - rhs))
        eta[k - 1] = float(np.linalg.norm(y))
        Y[k - 1, :k] = y
    return rho, eta, Y


def krylov_gcv(rho: np.ndarray, n: int) -> np.ndarray:
    """G(k) = rho_k^2 / (n - k)^2 for k = 1..len(rho) (trace of the rank-k projector A Z_k C_k^+ W_{k+1}^T is k)."""
    k = np.arange(1, rho.shape[0] + 1, dtype=np.float64)
    return rho * rho / ((n - k) ** 2)


def choose_k_lsqr_gcv(rho: np.ndarray, n: int) -> int:
    """Stopping index: argmin_k G(k) over k = 1..min(l, n-1), ties to the smaller k."""
    kmax = min(rho.shape[0], n - 1)
    if kmax < 1:
        return 1
    return 1 + int(np.argmin(krylov_gcv(rho[:kmax], n)))


def menger_curvature(a, b, c) -> float:
    """Signed curvature of the circle through the points a, b, c (visited in that order)."""
    ab, bc, ac = b - a, c - b, c - a
    la, lb, lc = np.linalg.norm(ab), np.linalg.norm(bc), np.linalg.norm(ac)
    cross = ab[0] * bc[1] - ab[1] * bc[0]
    return 2.0 * cross / (la * lb * lc)


def lcurve_discrete_corner(rho: np.ndarray, eta: np.ndarray):
    """Corner of the discrete L-curve p_k = (log rho_k, log eta_k): argmax over k = 2..l-1 of the
    signed curvature of (p_{k+1}, p_k, p_{k-1}), ties to the smaller k.  Triples with a side shorter
    than 1e-12 times the extent of the point set are skipped.  Returns (k, curvature, at_edge, curvatures)
    (k = l and at_edge when no triple qualifies)."""
    ell = rho.shape[0]
    tiny = np.finfo(np.float64).tiny
    P = np.stack([np.log(np.maximum(rho, tiny)), np.log(np.maximum(eta, tiny))], axis=1)
    kap = np.full(ell, -np.inf)
    if ell < 3:
        return ell, float("nan"), True, kap
    ext = float(np.max(np.max(P, axis=0) - np.min(P, axis=0)))
    tol = 1e-12 * ext
    for k in range(2, ell):  # 1-based k, inner points
        a, b, c = P[k], P[k - 1], P[k - 2]  # p_{k+1}, p_k, p_{k-1}
        if min(np.linalg.norm(b - a), np.linalg.norm(c - b), np.linalg.norm(c - a)) <= tol:
            continue
        kap[k - 1] = menger_curvature(a, b, c)
    if not np.any(np.isfinite(kap)):
        return ell, float("nan"), True, kap
    k = 1 + int(np.argmax(kap))
    return k, float(kap[k - 1]), (k == 2 or k == ell - 1), kap


def y_tikhonov(s: np.ndarray, ftil: np.ndarray, V: np.ndarray, lam: float) -> np.ndarray:
    """Projected Tikhonov solution y = sum_i s_i/(s_i^2 + lambda^2) f~_i v~_i (Algorithm 4 step 8, SVD form)."""
    ell = s.shape[0]
    w = s / (s * s + lam * lam) * ftil[:ell]
    return V @ w


def y_tsvd(s: np.ndarray, ftil: np.ndarray, V: np.ndarray, k: int) -> np.ndarray:
    """Projected TSVD solution y_k = V_k S_k^{-1} U_k^T (beta_1 e_1) (Algorithm 2 step 5)."""
    return V[:, :k] @ (ftil[:k] / s[:k])


# --------------------------------------------------------------------------
# End-to-end solve (Algorithm 2 / Algorithm 4)
# --------------------------------------------------------------------------


@dataclasses.dataclass
class SolveResult:
    coef: np.ndarray
    ell: int
    k: int
    lam: float
    crit: float  # GCV value (GCV rule) or curvature (L-curve rule) at the choice
    resid_norm: float  # rho_l at the choice (Tikhonov) or projected TSVD residual
    sol_norm: float
    flags: int
    alpha: np.ndarray
    beta: np.ndarray
    s: np.ndarray
    ftil: np.ndarray
    gkb: GKBResult


def solve(X: np.ndarray, n_int: int, kappa: float, eps: float, f: np.ndarray, ell: int,
          method: int = METHOD_HKT, rule: int = RULE_GCV, k_trunc: int = 0, lambda_fixed: float = 0.0,
          n_grid: int = 200, stored: bool = True, reorth: bool = True, gcv_weight: float = 1.0,
          row_scale: int = 0) -> SolveResult:
    """Ine-TSVD (Algorithm 2), HKT (Algorithm 4) or LSQR with early stopping (Section 3.4) from
    nodes and data to RBF coefficients.

    row_scale = 1 runs the method on the row-scaled system (D A) c = D f,
    D = diag(A)^{-1} (see row_scale()); every projected quantity then refers
    to that system, and the coefficients are its regularised solution."""
    X = _c(X)
    d = _row_scale_vector(X, n_int, kappa, eps) if row_scale else None
    A = assemble(X, n_int, kappa, eps) if stored else None
    if d is not None:
        f = d * _c(f)
        if A is not None:
            A *= d[:, None]
    g = gkb(A, X, n_int, kappa, eps, f, ell, reorth, d=None if A is not None else d)
    del A
    flags = FLAG_BREAKDOWN if g.flag else 0
    le = g.ell
    s, ft, V = proj_svd(g.alpha, g.beta)
    lam, k, crit = 0.0, 0, float("nan")
    omega = float(gcv_weight) if rule == RULE_WGCV else 1.0
    if method == METHOD_LSQR:
        rho, eta, Y = lsqr_path(g.alpha, g.beta)
        if rule == RULE_LCURVE:
            k, crit, edge, _ = lcurve_discrete_corner(rho, eta)
            if edge:
                flags |= FLAG_LCURVE_AT_EDGE
        elif rule == RULE_FIXED:
            k = min(max(int(k_trunc), 1), le)
            crit = float(krylov_gcv(rho, X.shape[0])[k - 1]) if k < X.shape[0] else float("nan")
        else:
            k = choose_k_lsqr_gcv(rho, X.shape[0])
            crit = float(krylov_gcv(rho, X.shape[0])[k - 1])
        y = Y[k - 1]
        coef = lift(g.Z, y)
        return SolveResult(coef, le, k, 0.0, crit, float(rho[k - 1]), float(eta[k - 1]), flags, g.alpha, g.beta,
                           s, ft, g)
    if method == METHOD_HKT:
        if rule in (RULE_GCV, RULE_WGCV):
            lam, crit, edge, _, _ = choose_lambda_gcv(s, ft, n_grid, omega=omega)
            if edge:
                flags |= FLAG_GCV_AT_EDGE
        elif rule == RULE_LCURVE:
            lam, crit, edge, _, _ = choose_lambda_lcurve(s, ft, n_grid)
            if edge:
                flags |= FLAG_LCURVE_AT_EDGE
        else:
            lam = float(lambda_fixed)
        y = y_tikhonov(s, ft, V, lam)
        rn = math.sqrt(rho2_proj(s, ft, lam))
        sn = math.sqrt(eta2_proj(s, ft, lam))
    else:
        k = int(k_trunc) if rule == RULE_FIXED and k_trunc > 0 else choose_rank(s, ft, omega)
        k = min(k, le)
        crit = tsvd_gcv(s, ft, k, omega)
        y = y_tsvd(s, ft, V, k)
        rn = math.sqrt(float(np.sum(ft[k:] ** 2)))
        sn = float(np.linalg.norm(ft[:k] / s[:k]))
    coef = lift(g.Z, y)
    return SolveResult(coef, le, k, lam, crit, rn, sn, flags, g.alpha, g.beta, s, ft, g)


# --------------------------------------------------------------------------
# Full-matrix references (tiny N only): TSVD and Tikhonov in SVD form
# --------------------------------------------------------------------------


def full_svd(A: np.ndarray):
    """Economy SVD of A by LAPACK (library routine; Algorithm 3 step 1)."""
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    return U, s, Vt.T


def full_tsvd(A: np.ndarray, f: np.ndarray, k: int) -> np.ndarray:
    """alpha_k = sum_{i<=k} v_i (u_i^T f) / s_i  (eq. (14))."""
    U, s, V = full_svd(A)
    return V[:, :k] @ ((U[:, :k].T @ f) / s[:k])


def full_tikhonov(A: np.ndarray, f: np.ndarray, lam: float) -> np.ndarray:
    """alpha_lambda = sum_i s_i/(s_i^2+lambda^2) (u_i^T f) v_i  (eq. (17))."""
    U, s, V = full_svd(A)
    return V @ (s / (s * s + lam * lam) * (U.T @ f))


def choose_lambda_full(s: np.ndarray, fhat: np.ndarray, s_perp: float, n: int, n_grid: int = 200) -> float:
    """Algorithm 3's lambda: the minimiser of the full-problem GCV (eq. (25)) over a log grid on
    [max(s_min, 16 eps_mach s_1), s_1], refined by golden section over the two cells around the
    grid minimum (ties to the larger lambda; a minimum at a grid end is kept)."""
    grid = lambda_grid(s, n_grid)
    vals = np.array([gcv_full(s, fhat, s_perp, n, lam) for lam in grid])
    k = n_grid - 1 - int(np.argmin(vals[::-1]))
    lam = float(grid[k])
    if 0 < k < n_grid - 1:
        t = golden_min(lambda tt: gcv_full(s, fhat, s_perp, n, math.exp(tt)), math.log(grid[k - 1]),
                       math.log(grid[k + 1]))
        if gcv_full(s, fhat, s_perp, n, math.exp(t)) <= vals[k]:
            lam = math.exp(t)
    return lam


def full_tikh_gcv(A: np.ndarray, f: np.ndarray, n_grid: int = 200):
    """Tikh-Reg via GCV (Algorithm 3) with grid refinement; returns (alpha, lambda)."""
    U, s, V = full_svd(A)
    n = A.shape[0]
    fhat = U.T @ f
    s_perp = max(0.0, float(f @ f) - float(fhat @ fhat))
    lam = choose_lambda_full(s, fhat, s_perp, n, n_grid)
    alpha = V @ (s / (s * s + lam * lam) * fhat)
    return alpha, lam


def gcv_tsvd_full(s: np.ndarray, fhat: np.ndarray, s_perp: float, n: int, k: int) -> float:
    """GCV of the full-problem TSVD solution of rank k: eq. (25) with the filter factors
    phi_i = 1 for i <= k and 0 otherwise, i.e. (sum_{i>k} fhat_i^2 + s_perp) / (n - k)^2."""
    d = n - k
    return (float(np.sum(fhat[k:] ** 2)) + s_perp) / (d * d)


def choose_rank_full(s: np.ndarray, fhat: np.ndarray, s_perp: float, n: int) -> int:
    """The TSVD rank minimising the full-problem GCV with 0/1 filter factors over
    k = 1 .. min(r, n - 1), r the number of non-zero singular values, ties to the smaller k."""
    r = int(np.count_nonzero(s > 0.0))
    kmax = min(r, n - 1)
    best, kb = None, 1
    for k in range(1, kmax + 1):
        g = gcv_tsvd_full(s[:r], fhat[:r], s_perp, n, k)
        if best is None or g < best:
            best, kb = g, k
    return kb


def full_tsvd_gcv(A: np.ndarray, f: np.ndarray):
    """Full TSVD (eq. (14)) with the rank chosen by the full-problem GCV (choose_rank_full);
    returns (alpha, k)."""
    U, s, V = full_svd(A)
    n = A.shape[0]
    fhat = U.T @ f
    s_perp = max(0.0, float(f @ f) - float(fhat @ fhat))
    kb = choose_rank_full(s, fhat, s_perp, n)
    alpha = V[:, :kb] @ (fhat[:kb] / s[:kb])
    return alpha, kb


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_linf(a: np.ndarray, b: np.ndarray) -> float:
    """Re = ||u - u_a||_inf / ||u||_inf (eq. (31))."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
