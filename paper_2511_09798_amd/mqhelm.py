"""Python binding of libmqhelm.so (include/mqhelm.h): argument marshalling only.

Every array argument is either a C-contiguous float64 numpy array (host
pointer) or a contiguous float64 torch tensor on the GPU (device pointer);
one call never mixes the two kinds.  Every computation runs in the HIP
library; importing this module fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Any, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmqhelm.so")

# constants (mirror include/mqhelm.h)
MQH_OK = 0
MQH_EINVAL = -1
MQH_ENOMEM = -2
MQH_EDEVICE = -3
MQH_WBREAKDOWN = 1
MQH_WEDGE = 2
MQH_WNOCONV = 3
MQH_OP_STORED_FP64 = 0
MQH_OP_MATFREE_FP64 = 1
MQH_OP_MATFREE_FP32 = 2
MQH_METHOD_INE_TSVD = 0
MQH_METHOD_HKT = 1
MQH_METHOD_LSQR = 2
MQH_RULE_GCV = 0
MQH_RULE_LCURVE = 1
MQH_RULE_FIXED = 2
MQH_RULE_WGCV = 3
MQH_FLAG_DEVICE_PTRS = 1
MQH_FLAG_TIME_PRODUCTS = 2
MQH_FLAG_FIXED_SHAPES = 4
MQH_FLAG_GRAPH = 8
MQH_FLAG_ROW_SCALE = 16
MQH_FLAG_PROJ_QR = 32
MQH_FLAG_PROJ_NO_FALLBACK = 64
MQH_FLAG_BLOCK_JACOBI = 128
MQH_INFO_BREAKDOWN = 1
MQH_INFO_GCV_AT_EDGE = 2
MQH_INFO_LCURVE_AT_EDGE = 4
MQH_INFO_SOLVE_NOCONV = 8
MQH_INFO_SVD_QR = 16
MQH_INFO_BLOCK_JACOBI = 32
MQH_MAX_ELL = 1024
MQH_NOALLOC_MAX_ELL = 512
MQH_NOALLOC_SCRATCH_BYTES = 6332800
MQH_FULL_MAX_N = 32768
MQH_FULL_CG_MAX = 1024
MQH_BLOCK_MAX_DIM = 4096
MQH_BLOCK_RHS = 16
MQH_MLP_IN = 24
MQH_MLP_WIDTH = 128
MQH_MLP_OUT = 2
MQH_MLP_PROBE = 10
MQH_MLP_NPARAMS = 36482

OP_MODES = {"stored_fp64": MQH_OP_STORED_FP64, "matfree_fp64": MQH_OP_MATFREE_FP64,
            "matfree_fp32": MQH_OP_MATFREE_FP32}


class MQHError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: status {code} ({msg})")
        self.code = code


class mqh_solve_opts(ctypes.Structure):
    _fields_ = [("ell", ctypes.c_int32), ("reorth", ctypes.c_int32), ("method", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("k_trunc", ctypes.c_int32), ("n_grid", ctypes.c_int32),
                ("lambda_fixed", ctypes.c_double), ("flags", ctypes.c_uint32), ("row_scale", ctypes.c_int32),
                ("gcv_weight", ctypes.c_double)]


class mqh_solve_info(ctypes.Structure):
    _fields_ = [("ell_done", ctypes.c_int32), ("k_chosen", ctypes.c_int32), ("lambda_chosen", ctypes.c_double),
                ("crit", ctypes.c_double), ("resid_norm", ctypes.c_double), ("sol_norm", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32), ("t_ms", ctypes.c_double * 8)]


class mqh_sweep_item(ctypes.Structure):
    _fields_ = [("p", ctypes.c_void_p), ("F", ctypes.c_void_p), ("ldf", ctypes.c_int64), ("nrhs", ctypes.c_int32),
                ("status", ctypes.c_int32), ("coef", ctypes.c_void_p), ("ldc", ctypes.c_int64),
                ("info", ctypes.c_void_p)]


class mqh_predictor(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("in_mean", ctypes.c_float * 24), ("in_std", ctypes.c_float * 24),
                ("out_mean", ctypes.c_float * 2), ("out_std", ctypes.c_float * 2), ("h", ctypes.c_double),
                ("ell_step", ctypes.c_int32), ("reserved", ctypes.c_int32), ("judge_ratio", ctypes.c_double)]


class mqh_learned_info(ctypes.Structure):
    _fields_ = [("ell_pred", ctypes.c_int32), ("used_net_lambda", ctypes.c_int32), ("lambda_net", ctypes.c_double),
                ("lambda_gcv", ctypes.c_double), ("gcv_net", ctypes.c_double), ("gcv_min", ctypes.c_double),
                ("out", ctypes.c_double * 2)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_d = ctypes.c_double

_SIGNATURES = {
    "mqh_version": (ctypes.c_int, []),
    "mqh_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "mqh_last_error": (ctypes.c_char_p, []),
    "mqh_problem_create": (ctypes.c_int, [_vp, _i64, _vp, _i64, _d, _d, _i32, _vp, _u32, ctypes.POINTER(_vp)]),
    "mqh_problem_destroy": (ctypes.c_int, [_vp]),
    "mqh_problem_size": (_i64, [_vp]),
    "mqh_device_bytes": (_i64, []),
    "mqh_apply": (ctypes.c_int, [_vp, _i32, _vp, _d, _vp, _vp, _u32]),
    "mqh_matrix_rows": (ctypes.c_int, [_vp, _i64, _i64, _vp, _u32]),
    "mqh_gkb": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp, ctypes.POINTER(_i32), _u32]),
    "mqh_proj_svd": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp, _vp, _u32]),
    "mqh_proj_svd_noalloc": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "mqh_param_choice": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32, _i32, _d, _i32, _d, ctypes.POINTER(_d),
                                        ctypes.POINTER(_i32), ctypes.POINTER(_d), ctypes.POINTER(_u32), _vp, _vp,
                                        _u32]),
    "mqh_lsqr": (ctypes.c_int, [_vp, _vp, _i32, _i64, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_d),
                                ctypes.POINTER(_u32), _vp, _vp, _vp, _vp, _u32]),
    "mqh_proj_solution": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i32, _d, _i32, _vp, _vp, _u32]),
    "mqh_lift": (ctypes.c_int, [_vp, _i64, _i32, _vp, _vp, _vp, _u32]),
    "mqh_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(mqh_solve_opts), _vp, _vp, _vp, _vp,
                                 ctypes.POINTER(mqh_solve_info)]),
    "mqh_apply_multi": (ctypes.c_int, [_vp, _i32, _vp, _i64, _i32, _vp, _vp, _i64, _vp, _i64, _u32]),
    "mqh_gkb_multi": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _u32]),
    "mqh_solve_multi": (ctypes.c_int, [_vp, _vp, _i64, _i32, ctypes.POINTER(mqh_solve_opts), _vp, _i64,
                                       ctypes.POINTER(mqh_solve_info)]),
    "mqh_solve_sweep": (ctypes.c_int, [ctypes.POINTER(mqh_sweep_item), _i32, ctypes.POINTER(mqh_solve_opts), _i32]),
    "mqh_full_svd": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_d), _u32]),
    "mqh_gkb_block": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp, ctypes.POINTER(_i32),
                                     ctypes.POINTER(_i32), _u32]),
    "mqh_solve_block": (ctypes.c_int, [_vp, _vp, _i64, _i32, ctypes.POINTER(mqh_solve_opts), _vp, _i64, _vp,
                                       ctypes.POINTER(mqh_solve_info)]),
    "mqh_full_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(mqh_solve_opts), _vp, _vp,
                                      ctypes.POINTER(mqh_solve_info)]),
    "mqh_eval": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _u32]),
    "mqh_mlp_forward": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp, _u32]),
    "mqh_mlp_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _u32]),
    "mqh_mlp_loss": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _u32]),
    "mqh_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, _i32, _vp, _u32]),
    "mqh_solve_learned": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(mqh_solve_opts), ctypes.POINTER(mqh_predictor),
                                         _vp, ctypes.POINTER(mqh_solve_info), ctypes.POINTER(mqh_learned_info)]),
}


def _load():
    # One HIP runtime per process: torch ships its own libamdhip64 (loaded
    # under the unversioned name), so when torch is importable it is loaded
    # first and this library binds to that runtime (its soname matches);
    # torch streams and device pointers are then valid in every call.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_09798_amd.build` "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def _check(code: int, where: str, warn_ok: bool = True) -> int:
    if code < 0 or (code > 0 and not warn_ok):
        raise MQHError(code, where, lib.mqh_last_error().decode() or lib.mqh_status_str(code).decode())
    return code


# --------------------------------------------------------------------------
# array marshalling
# --------------------------------------------------------------------------

def _is_torch(a: Any) -> bool:
    return type(a).__module__.startswith("torch")


def _ptr(a: Any):
    """(pointer, is_device) of a float64 contiguous array; None -> (None, None)."""
    if a is None:
        return None, None
    if _is_torch(a):
        if a.dtype.is_floating_point and a.element_size() != 8:
            raise TypeError("torch tensors must be float64")
        if not a.is_contiguous():
            raise TypeError("torch tensors must be contiguous")
        return ctypes.c_void_p(a.data_ptr()), bool(a.is_cuda)
    if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags.c_contiguous:
        raise TypeError("numpy arrays must be C-contiguous float64")
    return ctypes.c_void_p(a.ctypes.data), False


def _flags(*arrays) -> int:
    kinds = {d for (_, d) in (_ptr(a) for a in arrays if a is not None)}
    if len(kinds) > 1:
        raise TypeError("a call must use only host (numpy) or only device (torch) arrays")
    return MQH_FLAG_DEVICE_PTRS if kinds == {True} else 0


def _empty_like_kind(ref: Any, shape) -> Any:
    if ref is not None and _is_torch(ref) and ref.is_cuda:
        import torch

        return torch.empty(shape, dtype=torch.float64, device=ref.device)
    return np.empty(shape, dtype=np.float64)


def _zeros_like_kind(ref: Any, shape) -> Any:
    if ref is not None and _is_torch(ref) and ref.is_cuda:
        import torch

        return torch.zeros(shape, dtype=torch.float64, device=ref.device)
    return np.zeros(shape, dtype=np.float64)


def _stream_of(stream: Any) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


# --------------------------------------------------------------------------
# C-ABI names
# --------------------------------------------------------------------------

def mqh_version() -> int:
    return int(lib.mqh_version())


def mqh_status_str(code: int) -> str:
    return lib.mqh_status_str(code).decode()


def mqh_last_error() -> str:
    return lib.mqh_last_error().decode()


def mqh_problem_create(x_int, x_bnd, kappa: float, eps: float, op_mode: int, stream=None,
                       fixed_shapes: bool = False) -> ctypes.c_void_p:
    fl = _flags(x_int, x_bnd) | (MQH_FLAG_FIXED_SHAPES if fixed_shapes else 0)
    pi, _ = _ptr(x_int)
    pb, _ = _ptr(x_bnd)
    n_int = 0 if x_int is None else int(x_int.shape[0])
    n_bnd = 0 if x_bnd is None else int(x_bnd.shape[0])
    h = ctypes.c_void_p()
    _check(lib.mqh_problem_create(pi, n_int, pb, n_bnd, float(kappa), float(eps), int(op_mode), _stream_of(stream),
                                  fl, ctypes.byref(h)), "mqh_problem_create")
    return h


def mqh_device_bytes() -> int:
    """Bytes of device memory the library holds (compared with MQH_DEVICE_MEM_CAP)."""
    return int(lib.mqh_device_bytes())


def mqh_problem_destroy(h) -> None:
    lib.mqh_problem_destroy(h)


def mqh_apply(h, trans: int, x, shift: float = 0.0, z=None, y=None, row_scale: int = 0):
    fl = _flags(x, z, y) | (MQH_FLAG_ROW_SCALE if row_scale else 0)
    if y is None:
        y = _empty_like_kind(x, (x.shape[0],))
    _check(lib.mqh_apply(h, int(trans), _ptr(x)[0], float(shift), _ptr(z)[0], _ptr(y)[0], fl), "mqh_apply")
    return y


def mqh_matrix_rows(h, row0: int, count: int, out=None, n: Optional[int] = None, row_scale: int = 0):
    if out is None:
        out = np.empty((count, int(lib.mqh_problem_size(h))), dtype=np.float64)
    fl = _flags(out) | (MQH_FLAG_ROW_SCALE if row_scale else 0)
    _check(lib.mqh_matrix_rows(h, int(row0), int(count), _ptr(out)[0], fl), "mqh_matrix_rows")
    return out


def mqh_gkb(h, f, ell: int, reorth: int = 1, want_bases: bool = True, row_scale: int = 0):
    n = int(lib.mqh_problem_size(h))
    W = _empty_like_kind(f, (ell + 1, n)) if want_bases else None  # row k = column k of the n x (ell+1) basis
    Z = _empty_like_kind(f, (ell, n)) if want_bases else None
    al = _empty_like_kind(f, (ell,))
    be = _empty_like_kind(f, (ell + 1,))
    fl = _flags(f, W, Z, al, be) | (MQH_FLAG_ROW_SCALE if row_scale else 0)
    done = _i32(0)
    st = _check(lib.mqh_gkb(h, _ptr(f)[0], int(ell), int(reorth), _ptr(W)[0], _ptr(Z)[0], _ptr(al)[0], _ptr(be)[0],
                            ctypes.byref(done), fl), "mqh_gkb")
    return dict(W=W, Z=Z, alpha=al, beta=be, ell_done=int(done.value), status=st)


def mqh_proj_svd(alpha, beta, want_v: bool = True, stream=None, path: str = "auto"):
    """path: "auto" (fast path, QR iteration for rejected problems), "qr" (QR iteration only) or
    "fast" (fast path only; MQHError if it rejects the problem)."""
    ell = int(alpha.shape[0])
    sv = _empty_like_kind(alpha, (ell,))
    ft = _empty_like_kind(alpha, (ell + 1,))
    V = _empty_like_kind(alpha, (ell, ell)) if want_v else None  # row i = v~_i
    fl = _flags(alpha, beta, sv, ft, V) | {"auto": 0, "qr": MQH_FLAG_PROJ_QR, "fast": MQH_FLAG_PROJ_NO_FALLBACK}[path]
    _check(lib.mqh_proj_svd(_ptr(alpha)[0], _ptr(beta)[0], ell, _ptr(sv)[0], _ptr(ft)[0], _ptr(V)[0],
                            _stream_of(stream), fl), "mqh_proj_svd")
    return sv, ft, V


def mqh_proj_svd_noalloc(alpha, beta, sv, ftil, V=None, stream=None):
    """mqh_proj_svd into caller-provided device arrays with no device allocation (all torch CUDA tensors):
    sv (ell), ftil (ell + 1), V (ell x ell, row i = v~_i) or None."""
    ell = int(alpha.shape[0])
    arrays = [a for a in (alpha, beta, sv, ftil, V) if a is not None]
    if _flags(*arrays) != MQH_FLAG_DEVICE_PTRS:
        raise TypeError("mqh_proj_svd_noalloc takes device (torch CUDA) arrays only")
    _check(lib.mqh_proj_svd_noalloc(_ptr(alpha)[0], _ptr(beta)[0], ell, _ptr(sv)[0], _ptr(ftil)[0], _ptr(V)[0],
                                    _stream_of(stream)), "mqh_proj_svd_noalloc")
    return sv, ftil, V


def mqh_param_choice(sv, ftil, method: int, rule: int, n_grid: int = 200, lambda_fixed: float = 0.0,
                     k_trunc: int = 0, want_curve: bool = False, stream=None, gcv_weight: float = 1.0):
    ell = int(sv.shape[0])
    J = 200 if n_grid == 0 else n_grid
    curve = _empty_like_kind(sv, (J,)) if want_curve else None
    fl = _flags(sv, ftil, curve)
    lam, k, crit, inf = _d(0), _i32(0), _d(0), _u32(0)
    st = _check(lib.mqh_param_choice(_ptr(sv)[0], _ptr(ftil)[0], ell, int(method), int(rule), int(n_grid),
                                     float(lambda_fixed), int(k_trunc), float(gcv_weight), ctypes.byref(lam),
                                     ctypes.byref(k),
                                     ctypes.byref(crit), ctypes.byref(inf), _ptr(curve)[0], _stream_of(stream), fl),
                "mqh_param_choice")
    return dict(lambda_=lam.value, k=int(k.value), crit=crit.value, flags=int(inf.value), curve=curve, status=st)


def mqh_lsqr(alpha, beta, n: int, rule: int = MQH_RULE_GCV, k_trunc: int = 0, want_path: bool = True, stream=None):
    """LSQR iterates on the projected problem and the stopping index (Section 3.4)."""
    ell = int(alpha.shape[0])
    y = _empty_like_kind(alpha, (ell,))
    rho = _empty_like_kind(alpha, (ell,)) if want_path else None
    eta = _empty_like_kind(alpha, (ell,)) if want_path else None
    fl = _flags(alpha, beta, y, rho, eta)
    k, crit, inf = _i32(0), _d(0), _u32(0)
    st = _check(lib.mqh_lsqr(_ptr(alpha)[0], _ptr(beta)[0], ell, int(n), int(rule), int(k_trunc), ctypes.byref(k),
                             ctypes.byref(crit), ctypes.byref(inf), _ptr(y)[0], _ptr(rho)[0], _ptr(eta)[0],
                             _stream_of(stream), fl), "mqh_lsqr")
    return dict(k=int(k.value), crit=crit.value, flags=int(inf.value), y=y, rho=rho, eta=eta, status=st)


def mqh_proj_solution(sv, ftil, V, method: int, lam: float = 0.0, k: int = 0, stream=None):
    ell = int(sv.shape[0])
    y = _empty_like_kind(sv, (ell,))
    fl = _flags(sv, ftil, V, y)
    _check(lib.mqh_proj_solution(_ptr(sv)[0], _ptr(ftil)[0], _ptr(V)[0], ell, int(method), float(lam), int(k),
                                 _ptr(y)[0], _stream_of(stream), fl), "mqh_proj_solution")
    return y


def mqh_lift(Z, y, stream=None):
    """coef = Z y with Z given as an (ell, n) array whose row k is column k."""
    ell, n = int(Z.shape[0]), int(Z.shape[1])
    coef = _empty_like_kind(Z, (n,))
    fl = _flags(Z, y, coef)
    _check(lib.mqh_lift(_ptr(Z)[0], n, ell, _ptr(y)[0], _ptr(coef)[0], _stream_of(stream), fl), "mqh_lift")
    return coef


@dataclasses.dataclass
class SolveOutput:
    coef: Any
    alpha: Any
    beta: Any
    sv: Any
    status: int
    ell_done: int
    k: int
    lam: float
    crit: float
    resid_norm: float
    sol_norm: float
    flags: int
    t_ms: list


def mqh_solve(h, f_int, g_bnd, ell: int, method: int = MQH_METHOD_HKT, rule: int = MQH_RULE_GCV,
              k_trunc: int = 0, lambda_fixed: float = 0.0, n_grid: int = 200, reorth: int = 1,
              time_products: bool = False, coef=None, gcv_weight: float = 1.0, want_sv: bool = True,
              row_scale: int = 0) -> SolveOutput:
    n = int(lib.mqh_problem_size(h))
    ref = f_int if f_int is not None else g_bnd
    if coef is None:
        coef = _empty_like_kind(ref, (n,))
    al = _zeros_like_kind(ref, (ell,))
    be = _zeros_like_kind(ref, (ell + 1,))
    sv = _zeros_like_kind(ref, (ell,)) if want_sv else None
    fl = _flags(f_int, g_bnd, coef, al, be, sv)
    opts = mqh_solve_opts(ell=int(ell), reorth=int(reorth), method=int(method), rule=int(rule),
                          k_trunc=int(k_trunc), n_grid=int(n_grid), lambda_fixed=float(lambda_fixed),
                          flags=fl | (MQH_FLAG_TIME_PRODUCTS if time_products else 0), row_scale=int(row_scale),
                          gcv_weight=float(gcv_weight))
    info = mqh_solve_info()
    st = _check(lib.mqh_solve(h, _ptr(f_int)[0], _ptr(g_bnd)[0], ctypes.byref(opts), _ptr(coef)[0], _ptr(al)[0],
                              _ptr(be)[0], _ptr(sv)[0], ctypes.byref(info)), "mqh_solve")
    return SolveOutput(coef, al, be, sv, st, info.ell_done, info.k_chosen, info.lambda_chosen, info.crit,
                       info.resid_norm, info.sol_norm, info.flags, list(info.t_ms))


def mqh_apply_multi(h, trans: int, X, shifts=None, Z=None, Y=None, row_scale: int = 0):
    """Rows of Y (nrhs x n): Y[k] = op(A) X[k] - shifts[k] Z[k]."""
    n = int(lib.mqh_problem_size(h))
    nrhs = int(X.shape[0])
    if X.shape[1] != n or (Z is not None and tuple(Z.shape) != tuple(X.shape)):
        raise ValueError("X and Z must be nrhs x n")
    if Y is None:
        Y = _empty_like_kind(X, (nrhs, n))
    fl = _flags(X, Z, Y) | (MQH_FLAG_ROW_SCALE if row_scale else 0)
    sh = None
    if shifts is not None:
        sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64).reshape(nrhs))
    _check(lib.mqh_apply_multi(h, int(trans), _ptr(X)[0], n, nrhs, None if sh is None else ctypes.c_void_p(sh.ctypes.data),
                               _ptr(Z)[0], n, _ptr(Y)[0], n, fl), "mqh_apply_multi", warn_ok=False)
    return Y


def mqh_gkb_multi(h, F, ell: int, reorth: int = 1, want_bases: bool = True, row_scale: int = 0):
    """Lockstep runs of Algorithm 1 for the rows of F (nrhs x n): per run k,
    W[k] (ell+1 x n, row j = w_{j+1}), Z[k], alpha[k], beta[k], ell_done[k]."""
    n = int(lib.mqh_problem_size(h))
    nrhs = int(F.shape[0])
    if F.shape[1] != n:
        raise ValueError("F must be nrhs x n")
    W = _empty_like_kind(F, (nrhs, ell + 1, n)) if want_bases else None
    Z = _empty_like_kind(F, (nrhs, ell, n)) if want_bases else None
    al = _empty_like_kind(F, (nrhs, ell))
    be = _empty_like_kind(F, (nrhs, ell + 1))
    fl = _flags(F, W, Z, al, be) | (MQH_FLAG_ROW_SCALE if row_scale else 0)
    done = np.zeros(nrhs, dtype=np.int32)
    st = _check(lib.mqh_gkb_multi(h, _ptr(F)[0], n, nrhs, int(ell), int(reorth), _ptr(W)[0], _ptr(Z)[0], _ptr(al)[0],
                                  _ptr(be)[0], ctypes.c_void_p(done.ctypes.data), fl), "mqh_gkb_multi")
    return dict(W=W, Z=Z, alpha=al, beta=be, ell_done=done, status=st)


@dataclasses.dataclass
class MultiSolveOutput:
    coef: Any          # nrhs x n
    status: int
    ell_done: np.ndarray
    k: np.ndarray
    lam: np.ndarray
    crit: np.ndarray
    resid_norm: np.ndarray
    sol_norm: np.ndarray
    flags: np.ndarray
    t_ms: np.ndarray   # nrhs x 8 (each run reports its group's times)


def mqh_solve_multi(h, F, ell: int, method: int = MQH_METHOD_HKT, rule: int = MQH_RULE_GCV, k_trunc: int = 0,
                    lambda_fixed: float = 0.0, n_grid: int = 200, reorth: int = 1, time_products: bool = False,
                    coef=None, gcv_weight: float = 1.0, graph: bool = False, row_scale: int = 0) -> MultiSolveOutput:
    """Algorithm 4 for every row of F (nrhs x n, rows [f_int; g_bnd])."""
    n = int(lib.mqh_problem_size(h))
    nrhs = int(F.shape[0])
    if F.shape[1] != n:
        raise ValueError("F must be nrhs x n")
    if coef is None:
        coef = _empty_like_kind(F, (nrhs, n))
    fl = _flags(F, coef) | (MQH_FLAG_GRAPH if graph else 0)
    opts = mqh_solve_opts(ell=int(ell), reorth=int(reorth), method=int(method), rule=int(rule),
                          k_trunc=int(k_trunc), n_grid=int(n_grid), lambda_fixed=float(lambda_fixed),
                          flags=fl | (MQH_FLAG_TIME_PRODUCTS if time_products else 0), row_scale=int(row_scale),
                          gcv_weight=float(gcv_weight))
    infos = (mqh_solve_info * nrhs)()
    st = _check(lib.mqh_solve_multi(h, _ptr(F)[0], n, nrhs, ctypes.byref(opts), _ptr(coef)[0], n, infos),
                "mqh_solve_multi")
    get = lambda f, dt: np.array([getattr(i, f) for i in infos], dtype=dt)  # noqa: E731
    return MultiSolveOutput(coef, st, get("ell_done", np.int32), get("k_chosen", np.int32),
                            get("lambda_chosen", np.float64), get("crit", np.float64),
                            get("resid_norm", np.float64), get("sol_norm", np.float64), get("flags", np.uint32),
                            np.array([list(i.t_ms) for i in infos], dtype=np.float64))


def mqh_gkb_block(h, F, ell: int, want_bases: bool = False) -> dict:
    """Block Golub-Kahan from the rows of F (nrhs x n, rows [f_int; g_bnd]): C ((ell + 1) nrhs x
    ell nrhs), E1 (nrhs x nrhs), the bases W ((ell + 1) nrhs x n) and Z (ell nrhs x n) as rows if
    want_bases, ell_done, flag, status."""
    n = int(lib.mqh_problem_size(h))
    s = int(F.shape[0])
    if F.shape[1] != n:
        raise ValueError("F must be nrhs x n")
    C = _zeros_like_kind(F, ((ell + 1) * s, ell * s))
    E1 = _zeros_like_kind(F, (s, s))
    W = _zeros_like_kind(F, ((ell + 1) * s, n)) if want_bases else None
    Z = _zeros_like_kind(F, (ell * s, n)) if want_bases else None
    fl = _flags(F, C, E1, W, Z)
    ld, flag = ctypes.c_int32(0), ctypes.c_int32(0)
    st = _check(lib.mqh_gkb_block(h, _ptr(F)[0], n, s, int(ell), _ptr(C)[0], _ptr(E1)[0], _ptr(W)[0], _ptr(Z)[0],
                                  ctypes.byref(ld), ctypes.byref(flag), fl), "mqh_gkb_block")
    return dict(C=C, E1=E1, W=W, Z=Z, ell_done=ld.value, flag=flag.value, status=st)


def mqh_solve_block(h, F, ell: int, rule: int = MQH_RULE_GCV, lambda_fixed: float = 0.0, n_grid: int = 200,
                    coef=None, want_sv: bool = False, jacobi: bool = False) -> MultiSolveOutput:
    """Block HKT: every row of F (nrhs x n) solved by Tikhonov on the block Krylov space of all rows
    (ell block steps); the returned record's sv holds the projected singular values if want_sv.
    jacobi: the projected problem through the Jacobi full SVD only (MQH_FLAG_BLOCK_JACOBI)."""
    n = int(lib.mqh_problem_size(h))
    s = int(F.shape[0])
    if F.shape[1] != n:
        raise ValueError("F must be nrhs x n")
    if coef is None:
        coef = _empty_like_kind(F, (s, n))
    sv = _zeros_like_kind(F, (ell * s,)) if want_sv else None
    fl = _flags(F, coef, sv) | (MQH_FLAG_BLOCK_JACOBI if jacobi else 0)
    opts = mqh_solve_opts(ell=int(ell), reorth=1, method=MQH_METHOD_HKT, rule=int(rule), k_trunc=0,
                          n_grid=int(n_grid), lambda_fixed=float(lambda_fixed), flags=fl, row_scale=0, gcv_weight=1.0)
    infos = (mqh_solve_info * s)()
    st = _check(lib.mqh_solve_block(h, _ptr(F)[0], n, s, ctypes.byref(opts), _ptr(coef)[0], n, _ptr(sv)[0], infos),
                "mqh_solve_block")
    get = lambda f, dt: np.array([getattr(i, f) for i in infos], dtype=dt)  # noqa: E731
    out = MultiSolveOutput(coef, st, get("ell_done", np.int32), get("k_chosen", np.int32),
                           get("lambda_chosen", np.float64), get("crit", np.float64), get("resid_norm", np.float64),
                           get("sol_norm", np.float64), get("flags", np.uint32),
                           np.array([list(i.t_ms) for i in infos], dtype=np.float64))
    out.sv = sv
    return out


def mqh_solve_sweep(problems, Fs, ell: int, workers: int = 2, coefs=None, method: int = MQH_METHOD_HKT,
                    rule: int = MQH_RULE_GCV, k_trunc: int = 0, lambda_fixed: float = 0.0, n_grid: int = 200,
                    reorth: int = 1, time_products: bool = False, gcv_weight: float = 1.0, graph: bool = False,
                    row_scale: int = 0):
    """Solve every problem of a sweep (Problem objects, each with its own right-hand sides Fs[i],
    nrhs_i x n_i) side by side on `workers` host threads; returns a list of MultiSolveOutput."""
    if len(problems) != len(Fs) or not problems:
        raise ValueError("one F per problem")
    count = len(problems)
    if coefs is None:
        coefs = [_empty_like_kind(F, tuple(F.shape)) for F in Fs]
    fl = _flags(*Fs, *coefs) | (MQH_FLAG_GRAPH if graph else 0)
    infos = [(mqh_solve_info * int(F.shape[0]))() for F in Fs]
    items = (mqh_sweep_item * count)()
    for i, (pr, F, C) in enumerate(zip(problems, Fs, coefs)):
        if F.shape[1] != pr.n or tuple(C.shape) != tuple(F.shape):
            raise ValueError("F and coef must be nrhs x n of their problem")
        items[i] = mqh_sweep_item(p=pr.h.value, F=_ptr(F)[0].value, ldf=pr.n, nrhs=int(F.shape[0]), status=0,
                                  coef=_ptr(C)[0].value, ldc=pr.n, info=ctypes.cast(infos[i], ctypes.c_void_p).value)
    opts = mqh_solve_opts(ell=int(ell), reorth=int(reorth), method=int(method), rule=int(rule),
                          k_trunc=int(k_trunc), n_grid=int(n_grid), lambda_fixed=float(lambda_fixed),
                          flags=fl | (MQH_FLAG_TIME_PRODUCTS if time_products else 0), row_scale=int(row_scale),
                          gcv_weight=float(gcv_weight))
    _check(lib.mqh_solve_sweep(items, count, ctypes.byref(opts), int(workers)), "mqh_solve_sweep")
    outs = []
    for i in range(count):
        inf = infos[i]
        get = lambda f, dt: np.array([getattr(x, f) for x in inf], dtype=dt)  # noqa: E731
        outs.append(MultiSolveOutput(coefs[i], int(items[i].status), get("ell_done", np.int32),
                                     get("k_chosen", np.int32), get("lambda_chosen", np.float64),
                                     get("crit", np.float64), get("resid_norm", np.float64),
                                     get("sol_norm", np.float64), get("flags", np.uint32),
                                     np.array([list(x.t_ms) for x in inf], dtype=np.float64)))
    return outs


def mqh_full_svd(h, f=None, ref=None):
    """Full SVD of A (one-sided block Jacobi): dict(sv descending, fhat = U^T f, sweeps, off, status)."""
    n = int(lib.mqh_problem_size(h))
    like = f if f is not None else ref
    sv = _empty_like_kind(like, (n,))
    fh = _empty_like_kind(like, (n,)) if f is not None else None
    fl = _flags(f, sv, fh)
    sw = _i32(0)
    off = _d(0.0)
    st = _check(lib.mqh_full_svd(h, _ptr(f)[0], _ptr(sv)[0], _ptr(fh)[0], ctypes.byref(sw), ctypes.byref(off), fl),
                "mqh_full_svd")
    return dict(sv=sv, fhat=fh, sweeps=int(sw.value), off=float(off.value), status=st)


def mqh_full_solve(h, f_int, g_bnd, method: int = MQH_METHOD_HKT, rule: int = MQH_RULE_GCV, k_trunc: int = 0,
                   lambda_fixed: float = 0.0, n_grid: int = 200, coef=None, want_sv: bool = True) -> SolveOutput:
    """Algorithm 3 (method MQH_METHOD_HKT: Tikhonov filter) or the full TSVD (MQH_METHOD_INE_TSVD) on the
    full SVD of A.  SolveOutput.ell_done holds the Jacobi sweeps, t_ms[6] the last sweep's off-diagonal."""
    n = int(lib.mqh_problem_size(h))
    ref = f_int if f_int is not None else g_bnd
    if coef is None:
        coef = _empty_like_kind(ref, (n,))
    sv = _zeros_like_kind(ref, (n,)) if want_sv else None
    fl = _flags(f_int, g_bnd, coef, sv)
    opts = mqh_solve_opts(ell=1, reorth=1, method=int(method), rule=int(rule), k_trunc=int(k_trunc),
                          n_grid=int(n_grid), lambda_fixed=float(lambda_fixed), flags=fl, row_scale=0, gcv_weight=1.0)
    info = mqh_solve_info()
    st = _check(lib.mqh_full_solve(h, _ptr(f_int)[0], _ptr(g_bnd)[0], ctypes.byref(opts), _ptr(coef)[0],
                                   _ptr(sv)[0], ctypes.byref(info)), "mqh_full_solve")
    return SolveOutput(coef, None, None, sv, st, info.ell_done, info.k_chosen, info.lambda_chosen, info.crit,
                       info.resid_norm, info.sol_norm, info.flags, list(info.t_ms))


def mqh_eval(h, coef, x_eval, u=None):
    m = int(x_eval.shape[0])
    if u is None:
        u = _empty_like_kind(coef, (m,))
    fl = _flags(coef, x_eval, u)
    _check(lib.mqh_eval(h, _ptr(coef)[0], _ptr(x_eval)[0], m, _ptr(u)[0], fl), "mqh_eval")
    return u


# --------------------------------------------------------------------------
# Predictor network (FP32 torch tensors on the GPU)
# --------------------------------------------------------------------------

def _fptr(t) -> ctypes.c_void_p:
    """Device pointer of a contiguous float32 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not (_is_torch(t) and t.is_cuda and t.dtype.itemsize == 4 and t.dtype.is_floating_point and t.is_contiguous()):
        raise TypeError("the network calls take contiguous float32 GPU tensors")
    return ctypes.c_void_p(t.data_ptr())


def mqh_mlp_forward(params, x, y, hidden, stream=None):
    _check(lib.mqh_mlp_forward(_fptr(params), _fptr(x), int(x.shape[0]), _fptr(y), _fptr(hidden), _stream_of(stream),
                               MQH_FLAG_DEVICE_PTRS), "mqh_mlp_forward")


def mqh_mlp_backward(params, x, hidden, dy, grad, work, stream=None):
    _check(lib.mqh_mlp_backward(_fptr(params), _fptr(x), _fptr(hidden), _fptr(dy), int(x.shape[0]), _fptr(grad),
                                _fptr(work), _stream_of(stream), MQH_FLAG_DEVICE_PTRS), "mqh_mlp_backward")


def mqh_mlp_loss(y, t, w, loss=None, dy=None, stream=None):
    _check(lib.mqh_mlp_loss(_fptr(y), _fptr(t), _fptr(w), int(y.shape[0]), _fptr(loss), _fptr(dy), _stream_of(stream),
                            MQH_FLAG_DEVICE_PTRS), "mqh_mlp_loss")


def mqh_mlp_adam(params, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, stream=None):
    _check(lib.mqh_mlp_adam(_fptr(params), _fptr(grad), _fptr(m), _fptr(v), int(params.numel()), float(lr),
                            float(beta1), float(beta2), float(eps), int(step), _stream_of(stream),
                            MQH_FLAG_DEVICE_PTRS), "mqh_mlp_adam")


def make_predictor(params, in_mean, in_std, out_mean, out_std, h: float, ell_step: int = 5,
                   judge_ratio: float = 0.0) -> mqh_predictor:
    pr = mqh_predictor()
    pr.params = _fptr(params)
    for i in range(MQH_MLP_IN):
        pr.in_mean[i] = float(in_mean[i])
        pr.in_std[i] = float(in_std[i])
    for i in range(MQH_MLP_OUT):
        pr.out_mean[i] = float(out_mean[i])
        pr.out_std[i] = float(out_std[i])
    pr.h = float(h)
    pr.ell_step = int(ell_step)
    pr.judge_ratio = float(judge_ratio)
    return pr


@dataclasses.dataclass
class LearnedOutput:
    coef: Any
    status: int
    ell_done: int
    lam: float
    ell_pred: int
    used_net_lambda: bool
    lambda_net: float
    lambda_gcv: float
    gcv_net: float
    gcv_min: float
    out: tuple
    t_ms: list


def mqh_solve_learned(h, f_int, g_bnd, ell: int, predictor: mqh_predictor, coef=None, n_grid: int = 200,
                      reorth: int = 1, row_scale: int = 0) -> LearnedOutput:
    n = int(lib.mqh_problem_size(h))
    ref = f_int if f_int is not None else g_bnd
    if coef is None:
        coef = _empty_like_kind(ref, (n,))
    fl = _flags(f_int, g_bnd, coef)
    opts = mqh_solve_opts(ell=int(ell), reorth=int(reorth), method=MQH_METHOD_HKT, rule=MQH_RULE_GCV, k_trunc=0,
                          n_grid=int(n_grid), lambda_fixed=0.0, flags=fl, row_scale=int(row_scale), gcv_weight=1.0)
    info, li = mqh_solve_info(), mqh_learned_info()
    st = _check(lib.mqh_solve_learned(h, _ptr(f_int)[0], _ptr(g_bnd)[0], ctypes.byref(opts), ctypes.byref(predictor),
                                      _ptr(coef)[0], ctypes.byref(info), ctypes.byref(li)), "mqh_solve_learned")
    return LearnedOutput(coef, st, info.ell_done, info.lambda_chosen, li.ell_pred, bool(li.used_net_lambda),
                         li.lambda_net, li.lambda_gcv, li.gcv_net, li.gcv_min, (li.out[0], li.out[1]),
                         list(info.t_ms))


# --------------------------------------------------------------------------
# Convenience wrapper
# --------------------------------------------------------------------------

class Problem:
    """Owns one mqh_problem handle (nodes, kappa, eps, operator mode, stream)."""

    def __init__(self, x_int, x_bnd, kappa: float, eps: float, op_mode="matfree_fp64", stream=None,
                 fixed_shapes: bool = False):
        mode = OP_MODES[op_mode] if isinstance(op_mode, str) else int(op_mode)
        self.mode = mode
        self.n_int = 0 if x_int is None else int(x_int.shape[0])
        self.n_bnd = 0 if x_bnd is None else int(x_bnd.shape[0])
        self.n = self.n_int + self.n_bnd
        self.h = mqh_problem_create(x_int, x_bnd, kappa, eps, mode, stream, fixed_shapes)

    def close(self):
        if self.h is not None and self.h.value:
            mqh_problem_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def apply(self, x, trans=False, shift=0.0, z=None, y=None, row_scale=0):
        return mqh_apply(self.h, int(bool(trans)), x, shift, z, y, row_scale)

    def matrix_rows(self, row0, count, out=None, row_scale=0):
        return mqh_matrix_rows(self.h, row0, count, out, row_scale=row_scale)

    def gkb(self, f, ell, reorth=True, want_bases=True, row_scale=0):
        return mqh_gkb(self.h, f, ell, int(bool(reorth)), want_bases, row_scale)

    def apply_multi(self, X, trans=False, shifts=None, Z=None, Y=None, row_scale=0):
        return mqh_apply_multi(self.h, int(bool(trans)), X, shifts, Z, Y, row_scale)

    def gkb_multi(self, F, ell, reorth=True, want_bases=True, row_scale=0):
        return mqh_gkb_multi(self.h, F, ell, int(bool(reorth)), want_bases, row_scale)

    def solve_multi(self, F, ell, **kw) -> MultiSolveOutput:
        return mqh_solve_multi(self.h, F, ell, **kw)

    def gkb_block(self, F, ell, **kw):
        return mqh_gkb_block(self.h, F, ell, **kw)

    def solve_block(self, F, ell, **kw) -> MultiSolveOutput:
        return mqh_solve_block(self.h, F, ell, **kw)

    def full_svd(self, f=None, ref=None):
        return mqh_full_svd(self.h, f, ref)

    def full_solve(self, f_int, g_bnd, **kw) -> SolveOutput:
        return mqh_full_solve(self.h, f_int, g_bnd, **kw)

    def solve_learned(self, f_int, g_bnd, ell, predictor, **kw) -> LearnedOutput:
        return mqh_solve_learned(self.h, f_int, g_bnd, ell, predictor, **kw)

    def solve(self, f_int, g_bnd, ell, **kw) -> SolveOutput:
        return mqh_solve(self.h, f_int, g_bnd, ell, **kw)

    def eval(self, coef, x_eval, u=None):
        return mqh_eval(self.h, coef, x_eval, u)
