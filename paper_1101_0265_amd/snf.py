"""Thin ctypes binding of libsnf (the C ABI declared in include/snf.h).

Argument marshalling only: tensors are passed as raw device pointers together with the
current HIP stream; every step of the computation runs in the library's HIP kernels.  The
binding refuses to work (raises) when the compiled library is missing -- there is no
fallback implementation.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsnf.so")

# ---- status codes, schemes, precisions (mirror include/snf.h) ----------------------------
OK, PENDING, OK_FLOOR = 0, 1, 2
EINVAL, ENOMEM, ENOCONV, ENONFINITE, EMIXED, EDEVICE, ESIZE = -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {OK: "ok", PENDING: "pending", OK_FLOOR: "ok_floor", EINVAL: "einval",
                ENOMEM: "enomem", ENOCONV: "noconv", ENONFINITE: "nonfinite", EMIXED: "mixed",
                EDEVICE: "edevice", ESIZE: "esize"}
NOALLOC_MAX_N = 896

SCHEMES = {"sp2": 0, "tc2": 1, "snf_varmu": 2, "mcweeny": 3, "snf_fixmu": 4,
           "snf_fixmu3": 5, "snf_fixmu5": 6, "pmm3": 7, "pmm5": 8, "snf_pij": 9, "pij": 10}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_ref64": 2, "bf16_ref64": 3}
BRANCH_LETTERS = {0: "S", 1: "F", 2: "M", 3: "3", 4: "5", 5: "P"}
LOG_MAX = 256
FLAG_TIME_PRODUCTS = 1
FLAG_TRUNC_ERROR_CONTROL = 2
FLAG_SUBSPACE_NEWTON = 4


class Params(ctypes.Structure):
    _fields_ = [("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("mu", ctypes.c_double), ("xi", ctypes.c_double),
                ("homo", ctypes.c_double), ("lumo", ctypes.c_double),
                ("n_occ", ctypes.c_int64), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("gap_switch", ctypes.c_double), ("lowp_floor", ctypes.c_double),
                ("poly_i", ctypes.c_int32), ("poly_j", ctypes.c_int32),
                ("screen_tau", ctypes.c_double)]


class LogRec(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int32), ("branch", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("betabar", ctypes.c_double), ("e", ctypes.c_double),
                ("t1", ctypes.c_double), ("t2", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("products", ctypes.c_int32), ("products_fp64", ctypes.c_int32),
                ("products_lowp", ctypes.c_int32), ("products_newton", ctypes.c_int32),
                ("idem_err", ctypes.c_double), ("trace", ctypes.c_double),
                ("trace_err", ctypes.c_double), ("alpha_last", ctypes.c_double),
                ("beta_last", ctypes.c_double), ("betabar_last", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("product_ms", ctypes.c_double),
                ("branch", ctypes.c_uint8 * LOG_MAX), ("flops", ctypes.c_double),
                ("blocks", ctypes.c_int64)]


class Bsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("b", ctypes.c_int32), ("nb", ctypes.c_int32),
                ("nnzb", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


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
    L.snf_purify_dense_noalloc.argtypes = L.snf_purify_dense.argtypes
    L.snf_purify_dense_noalloc.restype = ctypes.c_int
    L.snf_step_dense.argtypes = [vp, vp, i64, i64, dbl, dbl, dbl, i32, vp,
                                 ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), vp]
    L.snf_step_dense.restype = ctypes.c_int
    L.snf_purify_bsr.argtypes = [ctypes.POINTER(Bsr), ctypes.POINTER(Params), i32, dbl,
                                 ctypes.POINTER(ctypes.POINTER(Bsr)), ctypes.POINTER(Result),
                                 ctypes.POINTER(LogRec), i32, vp]
    L.snf_purify_bsr.restype = ctypes.c_int
    L.snf_step_bsr.argtypes = [ctypes.POINTER(Bsr), dbl, dbl, dbl, dbl, dbl,
                               ctypes.POINTER(ctypes.POINTER(Bsr)),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                               vp]
    L.snf_step_bsr.restype = ctypes.c_int
    L.snf_bsr_copy_out.argtypes = [ctypes.POINTER(Bsr), vp, vp, vp, vp]
    L.snf_bsr_copy_out.restype = ctypes.c_int
    L.snf_bsr_free.argtypes = [ctypes.POINTER(Bsr)]
    L.snf_bsr_free.restype = None
    L.snf_serve_create.argtypes = [ctypes.c_size_t, i32, ctypes.POINTER(vp)]
    L.snf_serve_create.restype = ctypes.c_int
    L.snf_serve_request_bytes.argtypes = [i64, i32]
    L.snf_serve_request_bytes.restype = ctypes.c_size_t
    L.snf_serve_submit.argtypes = [vp, vp, i64, ctypes.POINTER(Params), i32, i32, vp,
                                   ctypes.POINTER(ctypes.c_uint64)]
    L.snf_serve_submit.restype = ctypes.c_int
    L.snf_serve_submit_device.argtypes = [vp, vp, i64, ctypes.POINTER(Params), i32, i32, vp,
                                          ctypes.POINTER(ctypes.c_uint64)]
    L.snf_serve_submit_device.restype = ctypes.c_int
    L.snf_serve_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Result)]
    L.snf_serve_poll.restype = ctypes.c_int
    L.snf_serve_timing.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
    L.snf_serve_timing.restype = ctypes.c_int
    L.snf_serve_timeline.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
    L.snf_serve_timeline.restype = ctypes.c_int
    L.snf_shutdown.argtypes = []
    L.snf_shutdown.restype = ctypes.c_int
    L.snf_serve_destroy.argtypes = [vp]
    L.snf_serve_destroy.restype = ctypes.c_int
    L.snf_workspace_bytes.argtypes = [i64, i32]
    L.snf_workspace_bytes.restype = ctypes.c_size_t
    L.snf_release_workspace.argtypes = []
    L.snf_release_workspace.restype = ctypes.c_int
    L.snf_spectral_bounds.argtypes = [vp, i64, i64, i32, vp, ctypes.POINTER(dbl), vp]
    L.snf_spectral_bounds.restype = ctypes.c_int
    L.snf_gap_bounds.argtypes = [vp, vp, i64, i64, dbl, dbl, i32, vp, ctypes.POINTER(dbl), vp]
    L.snf_gap_bounds.restype = ctypes.c_int
    L.snf_strerror.argtypes = [ctypes.c_int]
    L.snf_strerror.restype = ctypes.c_char_p
    L.snf_version.argtypes = []
    L.snf_version.restype = ctypes.c_char_p
    _lib = L
    # free the library's device and pinned memory while the HIP runtime is still up: Python
    # runs atexit handlers before the C runtime's exit handlers, where HIP tears down
    atexit.register(L.snf_shutdown)
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
                flags=0, gap_switch=0.0, lowp_floor=0.0, poly_ij=None,
                screen_tau=0.0) -> Params:
    return Params(float(lambda_min), float(lambda_max),
                  float("nan") if mu is None else float(mu),
                  float("nan") if xi is None else float(xi),
                  float("nan") if homo is None else float(homo),
                  float("nan") if lumo is None else float(lumo),
                  -1 if n_occ is None else int(n_occ), float(tol), int(max_iter), int(flags),
                  float(gap_switch), float(lowp_floor),
                  int(poly_ij[0]) if poly_ij else 0, int(poly_ij[1]) if poly_ij else 0,
                  float(screen_tau))


def result_dict(res: Result, log_arr=None) -> dict:
    nrec = min(res.iterations + 1, LOG_MAX)
    d = dict(status=STATUS_NAMES.get(res.status, str(res.status)), code=res.status,
             iterations=res.iterations, products=res.products,
             products_fp64=res.products_fp64, products_lowp=res.products_lowp,
             products_newton=res.products_newton, idem_err=res.idem_err, trace=res.trace, trace_err=res.trace_err,
             alpha_last=res.alpha_last, beta_last=res.beta_last,
             betabar_last=res.betabar_last, device_ms=res.device_ms,
             product_ms=res.product_ms, flops=res.flops, blocks=res.blocks,
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
    (varying-mu), n_occ, tol, max_iter, flags, gap_switch, lowp_floor, poly_ij = (i, j) for
    the P_{i,j} schemes (see snf_params).
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


# ---- block-sparse path -------------------------------------------------------------------

def _bsr_struct(row_ptr, col_idx, val, n: int, b: int = 32) -> Bsr:
    import torch
    for t, dt, nm in ((row_ptr, torch.int32, "row_ptr"), (col_idx, torch.int32, "col_idx"),
                      (val, torch.float32, "val")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError(f"{nm} must be a contiguous {dt} CUDA (HIP) tensor")
    nb = n // b
    return Bsr(int(n), int(b), int(nb), int(col_idx.numel()), row_ptr.data_ptr(),
               col_idx.data_ptr(), val.data_ptr())


def _take_bsr(ptr, stream) -> tuple:
    """Copy a library-allocated snf_bsr into torch tensors and free it."""
    import torch
    m = ptr.contents
    dev = torch.device("cuda", torch.cuda.current_device())
    rp = torch.empty(m.nb + 1, dtype=torch.int32, device=dev)
    ci = torch.empty(max(m.nnzb, 1), dtype=torch.int32, device=dev)
    va = torch.empty((max(m.nnzb, 1), m.b, m.b), dtype=torch.float32, device=dev)
    rc = lib().snf_bsr_copy_out(ptr, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), stream)
    lib().snf_bsr_free(ptr)
    if rc != OK:
        raise RuntimeError(f"snf_bsr_copy_out: {strerror(rc)}")
    return rp, ci[:m.nnzb], va[:m.nnzb]


def spectral_bounds(F, steps: int = 40, start=None, stream=None) -> tuple:
    """(lambda_min, lambda_max, gershgorin_min, gershgorin_max) of the symmetric float64 CUDA
    tensor F (see snf_spectral_bounds)."""
    _check_dense(F, "F")
    n = F.shape[0]
    if start is not None:
        _check_vec(start, n)
    out = (ctypes.c_double * 4)()
    rc = lib().snf_spectral_bounds(F.data_ptr(), n, F.stride(0), int(steps),
                                   start.data_ptr() if start is not None else None, out,
                                   _stream_handle(stream))
    if rc != OK:
        raise RuntimeError(f"snf_spectral_bounds: {strerror(rc)} ({rc})")
    return tuple(out)


def gap_bounds(F, D, lambda_min: float, lambda_max: float, steps: int = 40, start=None,
               stream=None) -> tuple:
    """(homo, lumo) bounds of the gap edges from a projector D (see snf_gap_bounds)."""
    _check_dense(F, "F")
    _check_dense(D, "D")
    n = F.shape[0]
    if D.shape != F.shape or D.stride(0) != F.stride(0):
        raise ValueError("D must match F in shape and row stride")
    if start is not None:
        _check_vec(start, n)
    out = (ctypes.c_double * 2)()
    rc = lib().snf_gap_bounds(F.data_ptr(), D.data_ptr(), n, F.stride(0), float(lambda_min),
                              float(lambda_max), int(steps),
                              start.data_ptr() if start is not None else None, out,
                              _stream_handle(stream))
    if rc != OK:
        raise RuntimeError(f"snf_gap_bounds: {strerror(rc)} ({rc})")
    return tuple(out)


def _check_vec(v, n):
    import torch
    if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64 and
            v.dim() == 1 and v.numel() == n and v.is_contiguous()):
        raise ValueError(f"start must be a contiguous float64 CUDA vector of length {n}")


def purify_bsr(row_ptr, col_idx, val, n: int, scheme: str = "snf_varmu", *, trunc_tau=1e-6,
               stream=None, want_log: bool = True, **params) -> tuple:
    """Purify a symmetric block-sparse F (32x32 FP32 blocks, device tensors).
    Returns ((row_ptr, col_idx, val) of D as torch tensors, result-dict)."""
    m = _bsr_struct(row_ptr, col_idx, val, n)
    p = make_params(**params)
    res = Result()
    logs = (LogRec * LOG_MAX)() if want_log else None
    out = ctypes.POINTER(Bsr)()
    sh = _stream_handle(stream)
    rc = lib().snf_purify_bsr(ctypes.byref(m), ctypes.byref(p), SCHEMES[scheme],
                              float(trunc_tau), ctypes.byref(out), ctypes.byref(res), logs,
                              LOG_MAX if want_log else 0, sh)
    if not out:
        raise RuntimeError(f"snf_purify_bsr: {strerror(rc)} ({rc})")
    D = _take_bsr(out, sh)
    d = result_dict(res, logs)
    d["nnzb"] = int(D[1].numel())
    return D, d


def step_bsr(row_ptr, col_idx, val, n: int, c2: float, c1: float, c0: float,
             trunc_tau: float = 0.0, screen_tau: float = 0.0, stream=None) -> tuple:
    """Y = truncation of (c2 X.X + c1 X + c0 I), X.X norm-screened at ``screen_tau``.
    Returns ((row_ptr, col_idx, val), sums, product-kernel ms)."""
    m = _bsr_struct(row_ptr, col_idx, val, n)
    out = ctypes.POINTER(Bsr)()
    sums = (ctypes.c_double * 3)()
    ms = ctypes.c_double(0.0)
    sh = _stream_handle(stream)
    rc = lib().snf_step_bsr(ctypes.byref(m), c2, c1, c0, float(trunc_tau), float(screen_tau),
                            ctypes.byref(out), sums, ctypes.byref(ms), sh)
    if rc != OK:
        raise RuntimeError(f"snf_step_bsr: {strerror(rc)} ({rc})")
    return _take_bsr(out, sh), (sums[0], sums[1], sums[2]), ms.value


# ---- serving -----------------------------------------------------------------------------

class Server:
    """Continuous-batching purification server (snf_serve_*): host matrices in, host D out."""

    def __init__(self, budget_bytes: int, max_slots: int = 64):
        self._h = ctypes.c_void_p()
        rc = lib().snf_serve_create(int(budget_bytes), int(max_slots), ctypes.byref(self._h))
        if rc != OK:
            raise RuntimeError(f"snf_serve_create: {strerror(rc)} ({rc})")
        self._out = {}

    @staticmethod
    def request_bytes(n: int, precision: str = "fp64") -> int:
        return int(lib().snf_serve_request_bytes(n, PRECISIONS[precision]))

    def submit(self, F, scheme: str = "snf_varmu", precision: str = "fp64", **params) -> int:
        import numpy as np
        F = np.ascontiguousarray(F, dtype=np.float64)
        n = F.shape[0]
        D = np.empty((n, n), dtype=np.float64)
        p = make_params(**params)
        t = ctypes.c_uint64(0)
        rc = lib().snf_serve_submit(self._h, F.ctypes.data, n, ctypes.byref(p), SCHEMES[scheme],
                                    PRECISIONS[precision], D.ctypes.data, ctypes.byref(t))
        if rc != OK:
            raise RuntimeError(f"snf_serve_submit: {strerror(rc)} ({rc})")
        self._out[t.value] = D
        return t.value

    def submit_device(self, F, scheme: str = "snf_varmu", precision: str = "fp64",
                      out=None, **params) -> int:
        """Submit a float64 CUDA tensor F (kept alive until completion); D is written to
        ``out`` (allocated if None), returned by poll/wait."""
        import torch
        _check_dense(F, "F")
        if not F.is_contiguous():
            raise ValueError("F must be contiguous")
        n = F.shape[0]
        D = out if out is not None else torch.empty_like(F)
        p = make_params(**params)
        t = ctypes.c_uint64(0)
        rc = lib().snf_serve_submit_device(self._h, F.data_ptr(), n, ctypes.byref(p),
                                           SCHEMES[scheme], PRECISIONS[precision],
                                           D.data_ptr(), ctypes.byref(t))
        if rc != OK:
            raise RuntimeError(f"snf_serve_submit_device: {strerror(rc)} ({rc})")
        self._out[t.value] = D
        self._keep = getattr(self, "_keep", {})
        self._keep[t.value] = F
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (D, result-dict)."""
        res = Result()
        rc = lib().snf_serve_poll(self._h, ticket, ctypes.byref(res))
        if rc == PENDING:
            return None
        if rc == EINVAL and ticket not in self._out:
            raise KeyError(ticket)
        return self._out[ticket], result_dict(res)

    def timing(self, ticket: int) -> tuple:
        ms = (ctypes.c_double * 3)()
        rc = lib().snf_serve_timing(self._h, ticket, ms)
        if rc != OK:
            raise RuntimeError(f"snf_serve_timing: {strerror(rc)} ({rc})")
        return ms[0], ms[1], ms[2]

    def timeline(self, ticket: int) -> tuple:
        """(submitted, admitted, finished, done) in ms since the server was created."""
        t = (ctypes.c_double * 4)()
        rc = lib().snf_serve_timeline(self._h, ticket, t)
        if rc != OK:
            raise RuntimeError(f"snf_serve_timeline: {strerror(rc)} ({rc})")
        return t[0], t[1], t[2], t[3]

    def wait(self, ticket: int, timeout_s: float = 120.0, sleep_s: float = 2e-4):
        import time
        t0 = time.monotonic()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() - t0 > timeout_s:
                raise TimeoutError(f"request {ticket} not done after {timeout_s} s")
            time.sleep(sleep_s)

    def close(self) -> None:
        if self._h:
            lib().snf_serve_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
