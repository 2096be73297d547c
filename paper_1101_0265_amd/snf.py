"""Thin ctypes binding of libsnf (the C ABI declared in include/snf.h).

Argument marshalling only: tensors are passed as raw device pointers together with the
current HIP stream; every step of the computation runs in the library's HIP kernels.  The
binding refuses to work (raises) when the compiled library is missing -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsnf.so")

# ---- status codes, schemes, precisions (mirror include/snf.h) ----------------------------
OK, PENDING, OK_FLOOR = 0, 1, 2
EINVAL, ENOMEM, ENOCONV, ENONFINITE, EMIXED, EDEVICE = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {OK: "ok", PENDING: "pending", OK_FLOOR: "ok_floor", EINVAL: "einval",
                ENOMEM: "enomem", ENOCONV: "noconv", ENONFINITE: "nonfinite", EMIXED: "mixed",
                EDEVICE: "edevice"}

SCHEMES = {"sp2": 0, "tc2": 1, "snf_varmu": 2, "mcweeny": 3, "snf_fixmu": 4}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_ref64": 2, "bf16_ref64": 3}
BRANCH_LETTERS = {0: "S", 1: "F", 2: "M"}
LOG_MAX = 256
FLAG_TIME_PRODUCTS = 1


class Params(ctypes.Structure):
    _fields_ = [("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("mu", ctypes.c_double), ("xi", ctypes.c_double),
                ("homo", ctypes.c_double), ("lumo", ctypes.c_double),
                ("n_occ", ctypes.c_int64), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("gap_switch", ctypes.c_double), ("lowp_floor", ctypes.c_double)]


class LogRec(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int32), ("branch", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("betabar", ctypes.c_double), ("e", ctypes.c_double),
                ("t1", ctypes.c_double), ("t2", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("products", ctypes.c_int32), ("products_fp64", ctypes.c_int32),
                ("products_lowp", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("idem_err", ctypes.c_double), ("trace", ctypes.c_double),
                ("trace_err", ctypes.c_double), ("alpha_last", ctypes.c_double),
                ("beta_last", ctypes.c_double), ("betabar_last", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("product_ms", ctypes.c_double),
                ("branch", ctypes.c_uint8 * LOG_MAX)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsnf.so (built by ``build_lib``); raise if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1101_0265_amd.build_lib` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.snf_purify_dense.argtypes = [vp, i64, i64, ctypes.POINTER(Params), i32, i32, vp,
                                   ctypes.POINTER(Result), ctypes.POINTER(LogRec), i32, vp]
    L.snf_purify_dense.restype = ctypes.c_int
    L.snf_step_dense.argtypes = [vp, vp, i64, i64, dbl, dbl, dbl, i32, vp,
                                 ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), vp]
    L.snf_step_dense.restype = ctypes.c_int
    L.snf_workspace_bytes.argtypes = [i64, i32]
    L.snf_workspace_bytes.restype = ctypes.c_size_t
    L.snf_release_workspace.argtypes = []
    L.snf_release_workspace.restype = ctypes.c_int
    L.snf_strerror.argtypes = [ctypes.c_int]
    L.snf_strerror.restype = ctypes.c_char_p
    L.snf_version.argtypes = []
    L.snf_version.restype = ctypes.c_char_p
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().snf_strerror(status).decode()


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _check_dense(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA (HIP) tensor")
    if t.dim() != 2 or t.shape[0] != t.shape[1] or t.stride(1) != 1:
        raise ValueError(f"{name} must be a square row-major matrix")


def make_params(*, lambda_min, lambda_max, mu=float("nan"), xi=float("nan"),
                homo=float("nan"), lumo=float("nan"), n_occ=-1, tol=1e-10, max_iter=200,
                flags=0, gap_switch=0.0, lowp_floor=0.0) -> Params:
    return Params(float(lambda_min), float(lambda_max),
                  float("nan") if mu is None else float(mu),
                  float("nan") if xi is None else float(xi),
                  float("nan") if homo is None else float(homo),
                  float("nan") if lumo is None else float(lumo),
                  -1 if n_occ is None else int(n_occ), float(tol), int(max_iter), int(flags),
                  float(gap_switch), float(lowp_floor))


def result_dict(res: Result, log_arr=None) -> dict:
    nrec = min(res.iterations + 1, LOG_MAX)
    d = dict(status=STATUS_NAMES.get(res.status, str(res.status)), code=res.status,
             iterations=res.iterations, products=res.products,
             products_fp64=res.products_fp64, products_lowp=res.products_lowp,
             idem_err=res.idem_err, trace=res.trace, trace_err=res.trace_err,
             alpha_last=res.alpha_last, beta_last=res.beta_last,
             betabar_last=res.betabar_last, device_ms=res.device_ms,
             product_ms=res.product_ms,
             branches="".join(BRANCH_LETTERS.get(res.branch[i], "")
                              for i in range(res.iterations)))
    if log_arr is not None:
        d["log"] = [dict(i=r.i, branch=BRANCH_LETTERS.get(r.branch), precision=r.precision,
                         phase=r.reserved, alpha=r.alpha, beta=r.beta, betabar=r.betabar,
                         e=r.e, t1=r.t1, t2=r.t2)
                    for r in list(log_arr)[:nrec]]
    return d


def purify_dense(F, scheme: str = "snf_varmu", precision: str = "fp64", *, out=None,
                 stream=None, want_log: bool = True, **params) -> tuple:
    """Purify the symmetric float64 CUDA tensor ``F``.  Returns (D, result-dict).

    ``params``: lambda_min, lambda_max, and per scheme mu/xi (fixed-mu), homo/lumo
    (varying-mu), n_occ, tol, max_iter, flags, gap_switch, lowp_floor (see snf_params).
    """
    import torch
    _check_dense(F, "F")
    n = F.shape[0]
    D = out if out is not None else torch.empty_like(F)
    _check_dense(D, "out")
    p = make_params(**params)
    res = Result()
    logs = (LogRec * LOG_MAX)() if want_log else None
    rc = lib().snf_purify_dense(F.data_ptr(), n, F.stride(0), ctypes.byref(p),
                                SCHEMES[scheme], PRECISIONS[precision], D.data_ptr(),
                                ctypes.byref(res), logs, LOG_MAX if want_log else 0,
                                _stream_handle(stream))
    if rc in (EINVAL, EDEVICE, ENOMEM) and res.iterations == 0 and res.products == 0:
        raise RuntimeError(f"snf_purify_dense: {strerror(rc)} ({rc})")
    return D, result_dict(res, logs)


def step_dense(A, B, c2: float, c1: float, c0: float, precision: str = "fp64", *, out=None,
               stream=None) -> tuple:
    """Y = c2 A.B + c1 A + c0 I with FP64 sums (||A.B - A||_F^2, tr Y, ||Y||_F^2).
    Returns (Y, sums tuple, product-kernel milliseconds)."""
    import torch
    _check_dense(A, "A")
    _check_dense(B, "B")
    if A.shape != B.shape or A.stride(0) != B.stride(0):
        raise ValueError("A and B must have the same shape and row stride")
    Y = out if out is not None else torch.empty_like(A)
    sums = (ctypes.c_double * 3)()
    ms = ctypes.c_double(0.0)
    rc = lib().snf_step_dense(A.data_ptr(), B.data_ptr(), A.shape[0], A.stride(0), c2, c1,
                              c0, PRECISIONS[precision], Y.data_ptr(), sums,
                              ctypes.byref(ms), _stream_handle(stream))
    if rc != OK:
        raise RuntimeError(f"snf_step_dense: {strerror(rc)} ({rc})")
    return Y, (sums[0], sums[1], sums[2]), ms.value


def workspace_bytes(n: int, precision: str = "fp64") -> int:
    return int(lib().snf_workspace_bytes(n, PRECISIONS[precision]))


def release_workspace() -> None:
    lib().snf_release_workspace()


def version() -> str:
    return lib().snf_version().decode()
