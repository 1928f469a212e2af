"""Block Golub-Kahan bidiagonalisation and block Tikhonov solutions for s
right-hand sides that share one Krylov space: Algorithm 1 and Algorithm 4
with the starting vector f replaced by the n x s block F.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's checks,
never by the library.  It shares no code with the HIP implementation.  Plain
numpy; a QR factorisation (numpy's Householder QR) and a dense SVD (LAPACK)
serve as library steps.

The paper has one right-hand side per problem; these readings make the
block form concrete:
* recurrence: W_1 E_1 = F; for j = 1 .. l
      Z_j D_j^T     = A^T W_j - Z_{j-1} E_j^T,
      W_{j+1} E_{j+1} = A Z_j - W_j D_j,
  each right side reorthogonalised against every earlier block of its basis
  by classical Gram-Schmidt twice (as reading 4 for one source), then
  factored by a QR with a non-negative diagonal in R (D_j^T and E_{j+1} are
  those R factors).  Hence A Z_l = W_{l+1} C_l, where C_l is the lower block
  bidiagonal (l + 1) s x l s matrix with D_j on the diagonal blocks and
  E_{j+1} below them, and A^T W_l = Z_l (C_l)_{1:ls, :}^T.  For s = 1 this
  is Algorithm 1 with alpha_j = D_j and beta_{j+1} = E_{j+1};
* breakdown: a QR whose R has a diagonal entry at most n eps_mach times the
  largest diagonal entry of the D and E blocks so far (E_1, the data's
  scale, left out) ends the process: at a D_j, l = j - 1 steps are kept; at
  an E_{j+1}, l = j steps with E_{j+1} = 0 (as reading 7 for one source);
* the sources must be linearly independent to working precision: E_1 with a
  diagonal entry at most n eps_mach times its largest (a zero or repeated
  source) is rejected, since W_1 would carry a direction of rounding noise;
* projected problem of source k: min ||C_l y - b_k||^2 + lambda^2 ||y||^2
  with b_k = (E_1 e_k; 0), solved through the SVD C_l = U S V^T:
  f~ = U^T b_k, y = V diag(s / (s^2 + lambda^2)) f~, coefficients Z_l y;
* GCV of source k in the full-problem form of eq. (25) with m = (l + 1) s
  rows: (sum_i (lambda^2 / (s_i^2 + lambda^2))^2 f~_i^2 + s_perp) /
  (m - sum_i s_i^2 / (s_i^2 + lambda^2))^2, s_perp = ||b_k||^2 - ||f~||^2;
  for s = 1, s_perp = f~_{l+1}^2 and this is eq. (30).  lambda by the grid
  and refinement of reading 9 on [max(s_min, 16 eps s_1), s_1], per source.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import oracle as O

EPS_MACH = np.finfo(np.float64).eps


def qr_pos(P: np.ndarray):
    """Thin QR of P (n x s, n >= s) with a non-negative diagonal in R."""
    Q, R = np.linalg.qr(P, mode="reduced")
    sg = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    return Q * sg[None, :], R * sg[:, None]


def cgs2(V: np.ndarray, P: np.ndarray) -> np.ndarray:
    """P with its components along the orthonormal columns of V removed, twice."""
    if V.shape[1] == 0:
        return P
    P = P - V @ (V.T @ P)
    return P - V @ (V.T @ P)


@dataclasses.dataclass
class BlockGKB:
    W: np.ndarray  # n x (l + 1) s
    Z: np.ndarray  # n x l s
    C: np.ndarray  # (l + 1) s x l s lower block bidiagonal
    E1: np.ndarray  # s x s, W_1 E_1 = F
    ell: int  # block steps kept
    flag: int  # 0, 1 (breakdown at a D block), 2 (at an E block)


def block_gkb(A: np.ndarray, F: np.ndarray, ell: int) -> BlockGKB:
    """The block recurrence of the module docstring, with full reorthogonalisation."""
    n, s = F.shape
    W1, E1 = qr_pos(F)
    d = np.abs(np.diag(E1))
    if not float(d.min()) > n * EPS_MACH * float(d.max()):
        raise ValueError("the sources are zero or linearly dependent")
    Ws, Zs, Ds, Es = [W1], [], [], []
    scale = 0.0
    tau = n * EPS_MACH
    flag, kept = 0, ell
    for j in range(1, ell + 1):
        P = A.T @ Ws[-1]
        if j > 1:
            P = P - Zs[-1] @ Es[-1].T
        P = cgs2(np.hstack(Zs) if Zs else np.zeros((n, 0)), P)
        Zj, R = qr_pos(P)
        scale = max(scale, float(np.max(np.abs(np.diag(R)))))
        if float(np.min(np.diag(R))) <= tau * scale:
            flag, kept = 1, j - 1
            break
        Dj = R.T
        Q = A @ Zj - Ws[-1] @ Dj
        Q = cgs2(np.hstack(Ws), Q)
        Wn, R2 = qr_pos(Q)
        scale = max(scale, float(np.max(np.abs(np.diag(R2)))))
        Zs.append(Zj)
        Ds.append(Dj)
        if float(np.min(np.diag(R2))) <= tau * scale:
            flag, kept = 2, j
            Es.append(np.zeros((s, s)))
            Ws.append(np.zeros((n, s)))
            break
        Es.append(R2)
        Ws.append(Wn)
    l = kept
    C = np.zeros(((l + 1) * s, l * s))
    for j in range(l):
        C[j * s:(j + 1) * s, j * s:(j + 1) * s] = Ds[j]
        C[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s] = Es[j]
    W = np.hstack(Ws[: l + 1])
    Z = np.hstack(Zs[:l]) if l > 0 else np.zeros((n, 0))
    return BlockGKB(W, Z, C, E1, l, flag)


@dataclasses.dataclass
class BlockSolve:
    coef: np.ndarray  # n x s
    lam: np.ndarray  # s
    sv: np.ndarray  # singular values of C_l, descending
    ftil: np.ndarray  # (l s) x s, U^T b_k
    s_perp: np.ndarray  # s
    gkb: BlockGKB


def block_solve(A: np.ndarray, F: np.ndarray, ell: int, lambda_fixed=None, n_grid: int = 200) -> BlockSolve:
    """Block HKT: per source the Tikhonov solution on the shared block Krylov space, lambda by the
    GCV of the module docstring, or lambda_fixed (a scalar or one value per source)."""
    g = block_gkb(A, F, ell)
    s = F.shape[1]
    m = (g.ell + 1) * s
    U, sv, Vt = np.linalg.svd(g.C, full_matrices=False)
    B = np.zeros((m, s))
    B[:s, :] = g.E1
    Ft = U.T @ B
    sp = np.maximum(0.0, np.sum(B * B, axis=0) - np.sum(Ft * Ft, axis=0))
    lams = np.zeros(s)
    coef = np.zeros((F.shape[0], s))
    for k in range(s):
        if lambda_fixed is None:
            lam = O.choose_lambda_full(sv, Ft[:, k], float(sp[k]), m, n_grid)
        else:
            lam = float(np.broadcast_to(np.asarray(lambda_fixed, dtype=float), (s,))[k])
        lams[k] = lam
        y = Vt.T @ (sv / (sv * sv + lam * lam) * Ft[:, k])
        coef[:, k] = g.Z @ y
    return BlockSolve(coef, lams, sv, Ft, sp, g)
