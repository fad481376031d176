"""ctypes binding of liblsrn.so (include/lsrn.h) for torch device tensors.

Argument marshalling only: every step of LSRN runs in the HIP kernels of the
library.  Arrays are torch float64 tensors on the current HIP device; work
is ordered on torch's current stream.  If the library has not been built
this module raises at first use (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsrn.so")

LSQR, CHEBYSHEV = 0, 1
ROW_MAJOR, COL_MAJOR = 0, 1
STATUS = {0: "ok", 1: "invalid argument", 2: "out of device memory", 3: "HIP runtime error",
          4: "not converged", 5: "unsupported"}


class LSRNError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Options(C.Structure):
    _fields_ = [("gamma", C.c_double), ("lambda_", C.c_double), ("tol", C.c_double),
                ("rcond", C.c_double), ("t_margin", C.c_double), ("refine_tol", C.c_double),
                ("seed", C.c_uint64), ("max_iter", C.c_int64), ("method", C.c_int32),
                ("refine", C.c_int32), ("profile", C.c_int32), ("precond", C.c_int32),
                ("precision", C.c_int32), ("autotune", C.c_int32), ("keep_sketch", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("s", C.c_int64), ("d", C.c_int64), ("rank", C.c_int64), ("iters", C.c_int64),
                ("refine_steps", C.c_int64), ("refine_iters", C.c_int64), ("sweeps", C.c_int64),
                ("tall", C.c_int32), ("converged", C.c_int32), ("sigma_l", C.c_double),
                ("sigma_u", C.c_double), ("sigma_max", C.c_double), ("sigma_min_kept", C.c_double),
                ("t_sketch_ms", C.c_double), ("t_svd_ms", C.c_double), ("t_iter_ms", C.c_double),
                ("t_refine_ms", C.c_double), ("t_total_ms", C.c_double),
                ("t_sketch_kernel_ms", C.c_double), ("t_sweep_kernel_ms", C.c_double),
                ("sketch_kernels", C.c_int64), ("sweep_kernels", C.c_int64),
                ("t_jacobi_kernel_ms", C.c_double), ("jacobi_kernels", C.c_int64),
                ("fp64_refine_steps", C.c_int64), ("cs_fallbacks", C.c_int64),
                ("precond_used", C.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None

EXPORTS = ["lsrn_default_options", "lsrn_status_string", "lsrn_last_error", "lsrn_solve_dense",
           "lsrn_workspace_bytes", "lsrn_solve_csr", "lsrn_workspace_bytes_csr",
           "lsrn_philox_words", "lsrn_gauss_fill", "lsrn_sketch_dense", "lsrn_sketch_dense_bf16",
           "lsrn_sketch_csr",
           "lsrn_precond", "lsrn_precond_qr", "lsrn_iterate_dense", "lsrn_iterate_csr"]
EXPORTS = EXPORTS + ["lsrn_solve_batch", "lsrn_solve_batch_opts"]
SERVER_EXPORTS = ["lsrn_server_create", "lsrn_server_submit_dense", "lsrn_server_submit_csr",
                  "lsrn_server_wait", "lsrn_server_stats", "lsrn_server_last_error",
                  "lsrn_server_destroy"]
EXPORTS = EXPORTS + SERVER_EXPORTS
PLAN_EXPORTS = ["lsrn_plan_create_dense", "lsrn_plan_create_csr", "lsrn_plan_solve",
                "lsrn_plan_destroy", "lsrn_plan_set_lambda", "lsrn_tune_gamma"]
EXPORTS = EXPORTS + PLAN_EXPORTS + ["lsrn_solve_op", "lsrn_tune_export", "lsrn_tune_import",
                                     "lsrn_tune_clear", "lsrn_solve_dense_f32",
                                     "lsrn_sketch_dense_noalloc"]
NOALLOC_SCRATCH_BYTES = 64 << 20    # LSRN_NOALLOC_SCRATCH_BYTES
# lsrn_apply_fn: (ctx, trans, k, in, ldin, out, ldout, stream) -> int
APPLY_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int64,
                       C.c_void_p, C.c_int64, C.c_void_p)
PRECOND = {"auto": 0, "svd": 1, "qr": 2}
PRECISION = {"fp64": 0, "mixed": 1}
_SIZE_FNS = ("lsrn_default_options", "lsrn_status_string", "lsrn_last_error",
             "lsrn_workspace_bytes", "lsrn_workspace_bytes_csr", "lsrn_server_last_error",
             "lsrn_server_destroy", "lsrn_plan_destroy", "lsrn_tune_export", "lsrn_tune_clear")


class ServerTiming(C.Structure):
    _fields_ = [("queue_ms", C.c_double), ("run_ms", C.c_double), ("latency_ms", C.c_double),
                ("footprint_bytes", C.c_int64), ("batch_size", C.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1109_5981_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, I64, I32, U64, D = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_double
        L.lsrn_default_options.argtypes = [C.POINTER(Options)]
        L.lsrn_status_string.argtypes = [C.c_int]
        L.lsrn_status_string.restype = C.c_char_p
        L.lsrn_last_error.restype = C.c_char_p
        L.lsrn_solve_dense.argtypes = [I64, I64, P, I64, I32, P, P, C.POINTER(Options),
                                       C.POINTER(Info), P]
        L.lsrn_workspace_bytes.argtypes = [I64, I64, I32, C.POINTER(Options)]
        L.lsrn_workspace_bytes.restype = C.c_size_t
        L.lsrn_philox_words.argtypes = [U64, I64, I64, I64, I64, P, P]
        L.lsrn_gauss_fill.argtypes = [U64, I64, I64, I64, I64, P, P]
        L.lsrn_sketch_dense.argtypes = [I64, I64, P, I64, I32, D, I64, U64, P, P]
        L.lsrn_sketch_dense_bf16.argtypes = [I64, I64, P, I64, I32, D, I64, U64, P, P]
        L.lsrn_sketch_dense_noalloc.argtypes = [I64, I64, P, I64, I32, D, I64, U64, P, P]
        L.lsrn_precond.argtypes = [I64, I64, P, D, P, P, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64), P]
        L.lsrn_iterate_dense.argtypes = [I64, I64, P, I64, I32, P, P, I64, I64, I64, P,
                                         C.POINTER(Options), C.POINTER(Info), P]
        L.lsrn_solve_csr.argtypes = [I64, I64, I64, P, P, P, P, P, C.POINTER(Options),
                                     C.POINTER(Info), P]
        L.lsrn_workspace_bytes_csr.argtypes = [I64, I64, I64, C.POINTER(Options)]
        L.lsrn_workspace_bytes_csr.restype = C.c_size_t
        L.lsrn_sketch_csr.argtypes = [I64, I64, I64, P, P, P, D, I64, U64, P, P]
        L.lsrn_precond_qr.argtypes = [I64, I64, P, D, P, P, P]
        L.lsrn_iterate_csr.argtypes = [I64, I64, I64, P, P, P, P, P, I64, I64, I64, P,
                                       C.POINTER(Options), C.POINTER(Info), P]
        L.lsrn_solve_batch.argtypes = [I32, P, P, P, P, P, P, C.POINTER(Options), P, P]
        L.lsrn_solve_batch_opts.argtypes = [I32, P, P, P, P, P, P, P, P, P]
        L.lsrn_server_create.argtypes = [I64, I32, C.POINTER(C.c_void_p)]
        L.lsrn_server_submit_dense.argtypes = [P, I64, I64, P, I64, I32, P, P, C.POINTER(Options),
                                               C.POINTER(C.c_int64)]
        L.lsrn_server_submit_csr.argtypes = [P, I64, I64, I64, P, P, P, P, P, C.POINTER(Options),
                                             C.POINTER(C.c_int64)]
        L.lsrn_server_wait.argtypes = [P, I64, C.POINTER(Info), C.POINTER(ServerTiming)]
        L.lsrn_server_stats.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                        C.POINTER(C.c_int64)]
        L.lsrn_server_last_error.restype = C.c_char_p
        L.lsrn_server_destroy.argtypes = [P]
        L.lsrn_server_destroy.restype = None
        L.lsrn_plan_create_dense.argtypes = [I64, I64, P, I64, I32, C.POINTER(Options),
                                             C.POINTER(C.c_void_p), C.POINTER(Info), P]
        L.lsrn_plan_create_csr.argtypes = [I64, I64, I64, P, P, P, C.POINTER(Options),
                                           C.POINTER(C.c_void_p), C.POINTER(Info), P]
        L.lsrn_plan_solve.argtypes = [P, P, P, C.POINTER(Options), C.POINTER(Info), P]
        L.lsrn_plan_destroy.argtypes = [P]
        L.lsrn_plan_set_lambda.argtypes = [P, D, C.POINTER(Info), P]
        L.lsrn_tune_gamma.argtypes = [C.POINTER(Info), D, D, D, C.POINTER(C.c_double)]
        L.lsrn_plan_destroy.restype = None
        L.lsrn_solve_op.argtypes = [I64, I64, APPLY_FN, P, P, P, C.POINTER(Options),
                                    C.POINTER(Info), P]
        L.lsrn_solve_dense_f32.argtypes = [I64, I64, P, I64, I32, P, P, C.POINTER(Options),
                                           C.POINTER(Info), P]
        L.lsrn_tune_export.argtypes = [C.c_char_p, C.c_size_t]
        L.lsrn_tune_export.restype = C.c_size_t
        L.lsrn_tune_import.argtypes = [C.c_char_p]
        L.lsrn_tune_clear.argtypes = []
        L.lsrn_tune_clear.restype = None
        for name in EXPORTS:
            if name not in _SIZE_FNS:
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise LSRNError(st, lib().lsrn_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a float64 tensor on the GPU")
    return t


def options(**kw) -> Options:
    o = Options()
    lib().lsrn_default_options(C.byref(o))
    alias = {"lam": "lambda_", "lambda": "lambda_"}
    for k, v in kw.items():
        k = alias.get(k, k)
        if k == "method" and isinstance(v, str):
            v = {"lsqr": LSQR, "chebyshev": CHEBYSHEV, "cs": CHEBYSHEV}[v.lower()]
        if k == "precond" and isinstance(v, str):
            v = PRECOND[v.lower()]
        if k == "precision" and isinstance(v, str):
            v = PRECISION[v.lower()]
        setattr(o, k, v)
    return o


def _layout_dims(A: torch.Tensor, layout: int):
    """(m, n, lda) of the least-squares matrix stored in A.  Row-major: A has
    shape (m, n).  Column-major: A holds A^T with shape (n, m)."""
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D tensor with unit stride in its last dimension")
    rows, cols = A.shape
    lda = A.stride(0) if rows > 1 else cols
    return (rows, cols, lda) if layout == ROW_MAJOR else (cols, rows, lda)


def solve_dense(A: torch.Tensor, b: torch.Tensor, x: torch.Tensor | None = None, *,
                layout: int = ROW_MAJOR, allow_not_converged: bool = False, **opts):
    """Min-length least-squares solution of min ||A x - b|| (Alg. 1 / Alg. 2).
    Returns (x, info dict).  With allow_not_converged, LSRN_E_NOT_CONVERGED
    returns the last iterate with info["status"] = 4 instead of raising."""
    _dev_f64(A, "A")
    _dev_f64(b, "b")
    m, n, lda = _layout_dims(A, layout)
    if b.numel() != m or not b.is_contiguous():
        raise ValueError("b must be contiguous with m entries")
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=A.device)
    o, info = options(**opts), Info()
    st = lib().lsrn_solve_dense(m, n, A.data_ptr(), lda, layout, b.data_ptr(), x.data_ptr(),
                                C.byref(o), C.byref(info), _stream())
    if not (allow_not_converged and st == 4):
        _check(st)
    out = info.as_dict()
    out["status"] = int(st)
    return x, out


def solve_dense_f32(A: torch.Tensor, b: torch.Tensor, x: torch.Tensor | None = None, *,
                    layout: int = ROW_MAJOR, allow_not_converged: bool = False, **opts):
    """lsrn_solve_dense_f32: A stored in FP32 (b, x FP64).  Returns (x, info)."""
    if not (isinstance(A, torch.Tensor) and A.is_cuda and A.dtype == torch.float32):
        raise TypeError("A must be a float32 tensor on the GPU")
    _dev_f64(b, "b")
    m, n, lda = _layout_dims(A, layout)
    if b.numel() != m or not b.is_contiguous():
        raise ValueError("b must be contiguous with m entries")
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=A.device)
    o, info = options(**opts), Info()
    st = lib().lsrn_solve_dense_f32(m, n, A.data_ptr(), lda, layout, b.data_ptr(), x.data_ptr(),
                                    C.byref(o), C.byref(info), _stream())
    if not (allow_not_converged and st == 4):
        _check(st)
    out = info.as_dict()
    out["status"] = int(st)
    return x, out


def workspace_bytes(m: int, n: int, layout: int = ROW_MAJOR, **opts) -> int:
    o = options(**opts)
    return int(lib().lsrn_workspace_bytes(m, n, layout, C.byref(o)))


def philox_words(seed: int, row0: int, nrows: int, q0: int, nq: int, device="cuda") -> torch.Tensor:
    """int32 tensor (nrows, nq, 4) holding the uint32 Philox words bit for bit."""
    out = torch.empty((nrows, nq, 4), dtype=torch.int32, device=device)
    _check(lib().lsrn_philox_words(seed, row0, nrows, q0, nq, out.data_ptr(), _stream()))
    return out


def gauss_fill(seed: int, row0: int, nrows: int, col0: int, ncols: int, device="cuda"):
    out = torch.empty((nrows, ncols), dtype=torch.float64, device=device)
    _check(lib().lsrn_gauss_fill(seed, row0, nrows, col0, ncols, out.data_ptr(), _stream()))
    return out


def sketch_dense(A: torch.Tensor, s: int, seed: int = 0, lam: float = 0.0,
                 layout: int = ROW_MAJOR) -> torch.Tensor:
    """The sketch X = G T (s x d) of Alg. 1/2 step 3, returned as a (d, s)
    tensor holding X column-major (so `.T` is X)."""
    _dev_f64(A, "A")
    m, n, lda = _layout_dims(A, layout)
    d = n if m >= n else m
    X = torch.empty((d, s), dtype=torch.float64, device=A.device)
    _check(lib().lsrn_sketch_dense(m, n, A.data_ptr(), lda, layout, lam, s, seed, X.data_ptr(),
                                   _stream()))
    return X


def sketch_dense_noalloc(A: torch.Tensor, s: int, seed: int = 0, lam: float = 0.0,
                         layout: int = ROW_MAJOR, X: torch.Tensor | None = None) -> torch.Tensor:
    """lsrn_sketch_dense_noalloc: sketch_dense with the library's static
    scratch instead of device allocations; enqueued on the current stream
    without a synchronisation.  X (d, s) may be given (else allocated here
    by torch, outside the call)."""
    _dev_f64(A, "A")
    m, n, lda = _layout_dims(A, layout)
    d = n if m >= n else m
    if X is None:
        X = torch.empty((d, s), dtype=torch.float64, device=A.device)
    if tuple(X.shape) != (d, s) or not X.is_contiguous():
        raise ValueError("X must be a contiguous (d, s) tensor")
    _check(lib().lsrn_sketch_dense_noalloc(m, n, A.data_ptr(), lda, layout, lam, s, seed,
                                           X.data_ptr(), _stream()))
    return X


def sketch_dense_bf16(A: torch.Tensor, s: int, seed: int = 0, lam: float = 0.0,
                      layout: int = ROW_MAJOR) -> torch.Tensor:
    """The precision form's sketch bf16(G) fl32(T), as sketch_dense."""
    _dev_f64(A, "A")
    m, n, lda = _layout_dims(A, layout)
    d = n if m >= n else m
    X = torch.empty((d, s), dtype=torch.float64, device=A.device)
    _check(lib().lsrn_sketch_dense_bf16(m, n, A.data_ptr(), lda, layout, lam, s, seed,
                                        X.data_ptr(), _stream()))
    return X


def precond(Xcm: torch.Tensor, rcond: float = 0.0):
    """Steps 4-5 on a sketch given column-major as a (d, s) tensor.
    Returns (rank, sigma (d,), P (d, r), sweeps)."""
    _dev_f64(Xcm, "X")
    d, s = Xcm.shape
    Xcm = Xcm.contiguous()
    sigma = torch.empty(d, dtype=torch.float64, device=Xcm.device)
    P = torch.empty((d, d), dtype=torch.float64, device=Xcm.device)
    r, sw = C.c_int64(), C.c_int64()
    _check(lib().lsrn_precond(s, d, Xcm.data_ptr(), rcond, sigma.data_ptr(), P.data_ptr(),
                              C.byref(r), C.byref(sw), _stream()))
    return int(r.value), sigma, P[:, : r.value], int(sw.value)


def iterate_dense(A: torch.Tensor, b: torch.Tensor, P: torch.Tensor, s: int, *,
                  layout: int = ROW_MAJOR, **opts):
    """Steps 6-7 with a given preconditioner P (d x r, row-major rows)."""
    _dev_f64(A, "A")
    _dev_f64(b, "b")
    _dev_f64(P, "P")
    if P.stride(1) != 1:
        raise ValueError("P must have unit stride in its last dimension")
    m, n, lda = _layout_dims(A, layout)
    x = torch.empty(n, dtype=torch.float64, device=A.device)
    o, info = options(**opts), Info()
    r = P.shape[1]
    _check(lib().lsrn_iterate_dense(m, n, A.data_ptr(), lda, layout, b.data_ptr(), P.data_ptr(),
                                    P.stride(0), r, s, x.data_ptr(), C.byref(o), C.byref(info),
                                    _stream()))
    return x, info.as_dict()


class Csr:
    """Device CSR matrix for the sparse entry points: rowptr int64 (m + 1),
    colind int32 (nnz), val float64 (nnz), all contiguous on the GPU."""

    def __init__(self, m: int, n: int, rowptr: torch.Tensor, colind: torch.Tensor,
                 val: torch.Tensor):
        for t, dt, name in ((rowptr, torch.int64, "rowptr"), (colind, torch.int32, "colind"),
                            (val, torch.float64, "val")):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise TypeError(f"{name} must be a contiguous {dt} tensor on the GPU")
        if rowptr.numel() != m + 1 or colind.numel() != val.numel():
            raise ValueError("CSR arrays have inconsistent sizes")
        self.m, self.n, self.nnz = int(m), int(n), int(val.numel())
        self.rowptr, self.colind, self.val = rowptr, colind, val

    @classmethod
    def from_host(cls, m, n, rowptr, colind, val, device="cuda"):
        import numpy as np
        return cls(m, n, torch.from_numpy(np.ascontiguousarray(rowptr, dtype=np.int64)).to(device),
                   torch.from_numpy(np.ascontiguousarray(colind, dtype=np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(val, dtype=np.float64)).to(device))

    def args(self):
        return (self.m, self.n, self.nnz, self.rowptr.data_ptr(), self.colind.data_ptr(),
                self.val.data_ptr())


def solve_csr(A: Csr, b: torch.Tensor, x: torch.Tensor | None = None, *,
              allow_not_converged: bool = False, **opts):
    """lsrn_solve_csr: min-length LS solution for CSR A.  Returns (x, info).
    With allow_not_converged, LSRN_E_NOT_CONVERGED returns the last iterate
    with info["status"] = 4 instead of raising."""
    _dev_f64(b, "b")
    if b.numel() != A.m or not b.is_contiguous():
        raise ValueError("b must be contiguous with m entries")
    if x is None:
        x = torch.empty(A.n, dtype=torch.float64, device=b.device)
    o, info = options(**opts), Info()
    st = lib().lsrn_solve_csr(*A.args(), b.data_ptr(), x.data_ptr(), C.byref(o), C.byref(info), _stream())
    if not (allow_not_converged and st == 4):
        _check(st)
    out = info.as_dict()
    out["status"] = int(st)
    return x, out


def workspace_bytes_csr(m: int, n: int, nnz: int, **opts) -> int:
    o = options(**opts)
    return int(lib().lsrn_workspace_bytes_csr(m, n, nnz, C.byref(o)))


def sketch_csr(A: Csr, s: int, seed: int = 0, lam: float = 0.0) -> torch.Tensor:
    """X = G T for CSR A as a (d, s) tensor holding X column-major."""
    d = min(A.m, A.n)
    X = torch.empty((d, s), dtype=torch.float64, device=A.val.device)
    _check(lib().lsrn_sketch_csr(*A.args(), lam, s, seed, X.data_ptr(), _stream()))
    return X


def precond_qr(Xcm: torch.Tensor, rcond: float = 0.0):
    """The QR-inverse preconditioner of a sketch given column-major as (d, s).
    Returns (|diag R| descending, P = R^-1 (d, d))."""
    _dev_f64(Xcm, "X")
    d, s = Xcm.shape
    Xcm = Xcm.contiguous()
    sigma = torch.empty(d, dtype=torch.float64, device=Xcm.device)
    P = torch.empty((d, d), dtype=torch.float64, device=Xcm.device)
    _check(lib().lsrn_precond_qr(s, d, Xcm.data_ptr(), rcond, sigma.data_ptr(), P.data_ptr(),
                                 _stream()))
    return sigma, P


def iterate_csr(A: Csr, b: torch.Tensor, P: torch.Tensor, s: int, **opts):
    """Steps 6-7 for CSR A with a given preconditioner P (d x r)."""
    _dev_f64(b, "b")
    _dev_f64(P, "P")
    if P.stride(1) != 1:
        raise ValueError("P must have unit stride in its last dimension")
    x = torch.empty(A.n, dtype=torch.float64, device=b.device)
    o, info = options(**opts), Info()
    _check(lib().lsrn_iterate_csr(*A.args(), b.data_ptr(), P.data_ptr(), P.stride(0), P.shape[1], s,
                                  x.data_ptr(), C.byref(o), C.byref(info), _stream()))
    return x, info.as_dict()


def tune_export() -> str:
    """The launch-shape tuning table as text (lsrn_tune_export)."""
    need = lib().lsrn_tune_export(None, 0)
    buf = C.create_string_buffer(need)
    lib().lsrn_tune_export(buf, need)
    return buf.value.decode()


def tune_import(text: str) -> None:
    _check(lib().lsrn_tune_import(text.encode()))


def tune_clear() -> None:
    lib().lsrn_tune_clear()


class _DeviceArray:
    """A device pointer described by the CUDA array interface."""

    def __init__(self, ptr: int, shape, strides):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": "<f8",
                                         "data": (int(ptr), False), "version": 2,
                                         "strides": tuple(strides)}


def device_view(ptr: int, rows: int, cols: int, ld: int) -> torch.Tensor:
    """A column-major rows x cols FP64 array at a device pointer (leading
    dimension ld) as a torch tensor of shape (rows, cols), without a copy."""
    if cols == 0 or rows == 0:
        return torch.empty((rows, cols), dtype=torch.float64, device="cuda")
    t = torch.as_tensor(_DeviceArray(ptr, (cols, rows), (ld * 8, 8)), device="cuda")
    return t.T


def solve_op(m: int, n: int, apply, b: torch.Tensor, x: torch.Tensor | None = None, *,
             allow_not_converged: bool = False, **opts):
    """lsrn_solve_op: A (m x n) given by apply(trans, k, in_ptr, ldin, out_ptr,
    ldout, stream) -> 0 on success, which writes out = A in (trans 0) or
    A^T in (trans 1) for k column-major columns.  Returns (x, info)."""
    _dev_f64(b, "b")
    if b.numel() != m or not b.is_contiguous():
        raise ValueError("b must be contiguous with m entries")
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=b.device)

    def trampoline(ctx, trans, k, pin, ldin, pout, ldout, stream):
        try:
            return int(apply(int(trans), int(k), pin, int(ldin), pout, int(ldout), stream) or 0)
        except Exception:  # an error must not cross the C boundary as a silent 0
            import traceback
            traceback.print_exc()
            return 1

    cb = APPLY_FN(trampoline)
    o, info = options(**opts), Info()
    st = lib().lsrn_solve_op(m, n, cb, None, b.data_ptr(), x.data_ptr(), C.byref(o), C.byref(info),
                             _stream())
    if not (allow_not_converged and st == 4):
        _check(st)
    out = info.as_dict()
    out["status"] = int(st)
    return x, out


class Plan:
    """lsrn_plan_*: the sketch and preconditioner of one matrix (steps 1-5)
    made once, then solves for many right-hand sides (steps 6-7).  Build
    with Plan.dense(A, ...) or Plan.csr(A, ...); keeps A alive."""

    def __init__(self, handle, m: int, n: int, keep, info: dict, opts: dict):
        self._h, self.m, self.n, self._keep, self.info = handle, m, n, keep, info
        self._opts = dict(opts)

    @classmethod
    def dense(cls, A: torch.Tensor, *, layout: int = ROW_MAJOR, **opts) -> "Plan":
        _dev_f64(A, "A")
        m, n, lda = _layout_dims(A, layout)
        h, o, info = C.c_void_p(), options(**opts), Info()
        _check(lib().lsrn_plan_create_dense(m, n, A.data_ptr(), lda, layout, C.byref(o),
                                            C.byref(h), C.byref(info), _stream()))
        return cls(h, m, n, (A,), info.as_dict(), opts)

    @classmethod
    def csr(cls, A: "Csr", **opts) -> "Plan":
        h, o, info = C.c_void_p(), options(**opts), Info()
        _check(lib().lsrn_plan_create_csr(*A.args(), C.byref(o), C.byref(h), C.byref(info),
                                          _stream()))
        return cls(h, A.m, A.n, (A,), info.as_dict(), opts)

    def solve(self, b: torch.Tensor, x: torch.Tensor | None = None, *,
              allow_not_converged: bool = False, **opts):
        """Steps 6-7 for b; opts update the plan's per-solve settings (tol,
        max_iter, method, refine, ...).  Returns (x, info)."""
        if self._h is None:
            raise RuntimeError("plan is closed")
        _dev_f64(b, "b")
        if b.numel() != self.m or not b.is_contiguous():
            raise ValueError("b must be contiguous with m entries")
        if x is None:
            x = torch.empty(self.n, dtype=torch.float64, device=b.device)
        info = Info()
        o = C.byref(options(**{**self._opts, **opts})) if opts else None
        st = lib().lsrn_plan_solve(self._h, b.data_ptr(), x.data_ptr(), o, C.byref(info), _stream())
        if not (allow_not_converged and st == 4):
            _check(st)
        out = info.as_dict()
        out["status"] = int(st)
        return x, out

    def set_lambda(self, lam: float) -> dict:
        """lsrn_plan_set_lambda: the preconditioner for a new Tikhonov weight
        from the kept sketch (the plan needs keep_sketch=1).  Returns info."""
        if self._h is None:
            raise RuntimeError("plan is closed")
        info = Info()
        _check(lib().lsrn_plan_set_lambda(self._h, float(lam), C.byref(info), _stream()))
        self._opts["lam"] = float(lam)
        self._opts.pop("lambda", None)
        self._opts.pop("lambda_", None)
        self.info = info.as_dict()
        return self.info

    def close(self):
        if self._h is not None:
            lib().lsrn_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_gamma(info: dict, tol: float = 1e-14, gamma_min: float = 1.25,
               gamma_max: float = 4.0) -> float:
    """lsrn_tune_gamma: the modelled best oversampling factor from the info
    of a measured solve (host arithmetic only)."""
    inf = Info()
    for name, _ in Info._fields_:
        if name in info:
            setattr(inf, name, info[name])
    g = C.c_double()
    _check(lib().lsrn_tune_gamma(C.byref(inf), tol, gamma_min, gamma_max, C.byref(g)))
    return g.value


class Server:
    """The serving runtime (lsrn_server_*): submit solves as they arrive,
    wait for them by ticket.  Tensors of a request are kept referenced until
    it has been waited for."""

    def __init__(self, hbm_budget_bytes: int, streams: int = 8):
        h = C.c_void_p()
        st = lib().lsrn_server_create(int(hbm_budget_bytes), int(streams), C.byref(h))
        if st != 0:
            raise LSRNError(st, lib().lsrn_server_last_error().decode())
        self._h = h
        self._keep = {}

    def submit_dense(self, A: torch.Tensor, b: torch.Tensor, x: torch.Tensor | None = None, *,
                     layout: int = ROW_MAJOR, **opts) -> int:
        _dev_f64(A, "A")
        _dev_f64(b, "b")
        m, n, lda = _layout_dims(A, layout)
        if b.numel() != m or not b.is_contiguous():
            raise ValueError("b must be contiguous with m entries")
        if x is None:
            x = torch.empty(n, dtype=torch.float64, device=A.device)
        o = options(**opts)
        t = C.c_int64()
        # the request's inputs must be complete before a worker stream reads them
        torch.cuda.current_stream().synchronize()
        st = lib().lsrn_server_submit_dense(self._h, m, n, A.data_ptr(), lda, layout, b.data_ptr(),
                                            x.data_ptr(), C.byref(o), C.byref(t))
        if st != 0:
            raise LSRNError(st, lib().lsrn_server_last_error().decode())
        self._keep[t.value] = (A, b, x)
        return t.value

    def submit_csr(self, A: "Csr", b: torch.Tensor, x: torch.Tensor | None = None, **opts) -> int:
        _dev_f64(b, "b")
        if x is None:
            x = torch.empty(A.n, dtype=torch.float64, device=b.device)
        o = options(**opts)
        t = C.c_int64()
        torch.cuda.current_stream().synchronize()
        st = lib().lsrn_server_submit_csr(self._h, *A.args(), b.data_ptr(), x.data_ptr(),
                                          C.byref(o), C.byref(t))
        if st != 0:
            raise LSRNError(st, lib().lsrn_server_last_error().decode())
        self._keep[t.value] = (A, b, x)
        return t.value

    def wait(self, ticket: int, allow_not_converged: bool = False):
        """(x, info dict, timing dict) of a submitted request."""
        info, tm = Info(), ServerTiming()
        st = lib().lsrn_server_wait(self._h, ticket, C.byref(info), C.byref(tm))
        _, _, x = self._keep.pop(ticket)
        if st != 0 and not (allow_not_converged and st == 4):
            raise LSRNError(st, lib().lsrn_server_last_error().decode())
        out = info.as_dict()
        out["status"] = int(st)
        return x, out, {"queue_ms": tm.queue_ms, "run_ms": tm.run_ms,
                        "latency_ms": tm.latency_ms, "footprint_bytes": tm.footprint_bytes,
                        "batch_size": tm.batch_size}

    def stats(self):
        p, r, b = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().lsrn_server_stats(self._h, C.byref(p), C.byref(r), C.byref(b)))
        return {"pending": p.value, "running": r.value, "bytes_in_use": b.value}

    def close(self):
        if self._h:
            lib().lsrn_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def solve_batch(As, bs, xs=None, allow_not_converged: bool = False, per_problem=None, **opts):
    """lsrn_solve_batch over lists of row-major tall A (n <= 512) and b, or
    with per_problem (a list of option dicts, one per problem, each merged
    over **opts) lsrn_solve_batch_opts.  Returns (list of x, list of info
    dicts)."""
    count = len(As)
    if len(bs) != count:
        raise ValueError("As and bs differ in length")
    ms, ns, ldas = [], [], []
    for A, b in zip(As, bs):
        _dev_f64(A, "A")
        _dev_f64(b, "b")
        m, n, lda = _layout_dims(A, ROW_MAJOR)
        if b.numel() != m or not b.is_contiguous():
            raise ValueError("b must be contiguous with m entries")
        ms.append(m); ns.append(n); ldas.append(lda)
    if xs is None:
        xs = [torch.empty(n, dtype=torch.float64, device=A.device) for A, n in zip(As, ns)]
    I64A = C.c_int64 * max(count, 1)
    PA = C.c_void_p * max(count, 1)
    infos = (Info * max(count, 1))()
    args = (count, I64A(*ms), I64A(*ns), PA(*[A.data_ptr() for A in As]), I64A(*ldas),
            PA(*[b.data_ptr() for b in bs]), PA(*[x.data_ptr() for x in xs]))
    if per_problem is None:
        o = options(**opts)
        st = lib().lsrn_solve_batch(*args, C.byref(o), infos, _stream())
    else:
        if len(per_problem) != count:
            raise ValueError("per_problem needs one option dict per problem")
        oa = (Options * max(count, 1))(*[options(**dict(opts, **d)) for d in per_problem])
        st = lib().lsrn_solve_batch_opts(*args, oa, infos, _stream())
    if not (allow_not_converged and st == 4):
        _check(st)
    return xs, [infos[i].as_dict() for i in range(count)]
