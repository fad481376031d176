"""Python access to the plain CPU LSRN oracle (oracle/lsrn_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The GPU library never imports this
package and this package never imports the GPU library.

All arrays are numpy float64 / int64 / int32 / uint32, C-contiguous.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lsrn_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblsrn_oracle.so")

ORC_DENSE_ROW, ORC_DENSE_COL, ORC_CSR = 0, 1, 2
LSQR, CS = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP on).  Returns the library path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Matrix(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("kind", C.c_int32), ("pad_", C.c_int32),
                ("a", C.c_void_p), ("lda", C.c_int64), ("rowptr", C.c_void_p),
                ("colind", C.c_void_p), ("val", C.c_void_p), ("lam", C.c_double)]


class _Options(C.Structure):
    _fields_ = [("gamma", C.c_double), ("tol", C.c_double), ("rcond", C.c_double),
                ("t_margin", C.c_double), ("seed", C.c_uint64), ("max_iter", C.c_int64),
                ("method", C.c_int32), ("refine", C.c_int32), ("precond", C.c_int32),
                ("pad_", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("s", C.c_int64), ("d", C.c_int64), ("rank", C.c_int64), ("iters", C.c_int64),
                ("sweeps", C.c_int64), ("refine_steps", C.c_int64),
                ("sigma_l", C.c_double), ("sigma_u", C.c_double),
                ("t_sketch", C.c_double), ("t_svd", C.c_double), ("t_iter", C.c_double),
                ("t_refine", C.c_double), ("tall", C.c_int32), ("converged", C.c_int32),
                ("cs_fallbacks", C.c_int64)]


_MV = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double))


class _Linop(C.Structure):
    _fields_ = [("rows", C.c_int64), ("cols", C.c_int64), ("mv", _MV), ("mvt", _MV),
                ("ctx", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        hdr = os.path.join(os.path.dirname(_SRC), "lsrn_oracle.h")
        if (not os.path.exists(_LIB_PATH)
                or os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(_SRC), os.path.getmtime(hdr))):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_philox_block.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, P]
        L.orc_box_muller.argtypes = [C.c_uint32, C.c_uint32, P, P]
        L.orc_gauss.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        L.orc_gauss.restype = C.c_double
        L.orc_gauss_fill.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int64, C.c_int64, P]
        L.orc_matvec.argtypes = [P, P, P]
        L.orc_matvec_t.argtypes = [P, P, P]
        L.orc_sketch.argtypes = [P, C.c_int64, C.c_uint64, P]
        L.orc_sketch.restype = C.c_int64
        L.orc_sketch_bf16.argtypes = [P, C.c_int64, C.c_uint64, P]
        L.orc_sketch_bf16.restype = C.c_int64
        L.orc_bf16_round.argtypes = [C.c_float]
        L.orc_bf16_round.restype = C.c_float
        L.orc_qr_r.argtypes = [C.c_int64, C.c_int64, P, P]
        L.orc_jacobi_rt.argtypes = [C.c_int64, P, P, C.c_int]
        L.orc_precond.argtypes = [C.c_int64, C.c_int64, P, C.c_double, P, P, P]
        L.orc_precond.restype = C.c_int64
        L.orc_precond_qr.argtypes = [C.c_int64, C.c_int64, P, C.c_double, P, P]
        L.orc_precond_qr.restype = C.c_int64
        L.orc_lsqr.argtypes = [C.POINTER(_Linop), P, C.c_double, C.c_int64, P]
        L.orc_lsqr.restype = C.c_int64
        L.orc_cs.argtypes = [C.POINTER(_Linop), P, C.c_double, C.c_double, C.c_double, P]
        L.orc_cs.restype = C.c_int64
        L.orc_cs_iterations.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_cs_iterations.restype = C.c_int64
        L.orc_cs_bounds.argtypes = [C.c_int64, C.c_int64, C.c_double, P, P]
        L.orc_lsrn_solve.argtypes = [P, P, P, P, P, P, P]
        L.orc_lsrn_iterate.argtypes = [P, P, P, C.c_int64, C.c_int64, C.c_int64, P, P, P]
        L.orc_pinv_solve.argtypes = [P, P, C.c_double, P]
        L.orc_pinv_solve.restype = C.c_int64
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- problems

@dataclass
class Matrix:
    """A least-squares matrix for the oracle.

    kind ORC_DENSE_ROW: `a` is m x n row-major.  ORC_DENSE_COL: `a` holds A
    column-major, i.e. `a` is the n x m row-major array of A^T.  ORC_CSR:
    rowptr/colind/val.  lam > 0 selects the Tikhonov problem (Sec. 5)."""
    m: int
    n: int
    kind: int = ORC_DENSE_ROW
    a: np.ndarray | None = None
    rowptr: np.ndarray | None = None
    colind: np.ndarray | None = None
    val: np.ndarray | None = None
    lam: float = 0.0

    @staticmethod
    def dense(A: np.ndarray, lam: float = 0.0) -> "Matrix":
        A = _f64(A)
        return Matrix(A.shape[0], A.shape[1], ORC_DENSE_ROW, a=A, lam=lam)

    @staticmethod
    def dense_colmajor(At: np.ndarray, lam: float = 0.0) -> "Matrix":
        """A given through the row-major array of A^T (n x m)."""
        At = _f64(At)
        return Matrix(At.shape[1], At.shape[0], ORC_DENSE_COL, a=At, lam=lam)

    @staticmethod
    def csr(m, n, rowptr, colind, val, lam: float = 0.0) -> "Matrix":
        return Matrix(m, n, ORC_CSR, rowptr=np.ascontiguousarray(rowptr, np.int64),
                      colind=np.ascontiguousarray(colind, np.int32), val=_f64(val), lam=lam)

    def _struct(self) -> _Matrix:
        s = _Matrix()
        s.m, s.n, s.kind, s.lam = self.m, self.n, self.kind, float(self.lam)
        if self.kind == ORC_CSR:
            s.rowptr, s.colind, s.val = (self.rowptr.ctypes.data, self.colind.ctypes.data,
                                         self.val.ctypes.data)
            s.a, s.lda = None, 0
        else:
            s.a = self.a.ctypes.data
            s.lda = self.n if self.kind == ORC_DENSE_ROW else self.m
        return s

    def to_dense(self) -> np.ndarray:
        if self.kind == ORC_DENSE_ROW:
            return self.a.copy()
        if self.kind == ORC_DENSE_COL:
            return self.a.T.copy()
        A = np.zeros((self.m, self.n))
        for i in range(self.m):
            for p in range(self.rowptr[i], self.rowptr[i + 1]):
                A[i, self.colind[p]] += self.val[p]
        return A


# ---------------------------------------------------------------- RNG

def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox_block(seed: int, row: int, q: int) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().orc_philox_block(seed, row, q, _ptr(out))
    return out


def box_muller(w0: int, w1: int):
    g0, g1 = C.c_double(), C.c_double()
    lib().orc_box_muller(w0, w1, C.byref(g0), C.byref(g1))
    return g0.value, g1.value


def gauss(seed: int, row: int, col: int) -> float:
    return lib().orc_gauss(seed, row, col)


def gauss_fill(seed: int, row0: int, nrows: int, col0: int, ncols: int) -> np.ndarray:
    out = np.zeros((nrows, ncols))
    lib().orc_gauss_fill(seed, row0, nrows, col0, ncols, _ptr(out))
    return out


# ---------------------------------------------------------------- steps

def matvec(M: Matrix, x) -> np.ndarray:
    x = _f64(x)
    y = np.zeros(M.m)
    s = M._struct()
    lib().orc_matvec(C.byref(s), _ptr(x), _ptr(y))
    return y


def matvec_t(M: Matrix, y) -> np.ndarray:
    y = _f64(y)
    x = np.zeros(M.n)
    s = M._struct()
    lib().orc_matvec_t(C.byref(s), _ptr(y), _ptr(x))
    return x


def is_tall(M: Matrix) -> bool:
    """Alg. 1 when m >= n, Alg. 2 otherwise (with lambda > 0 the latter is
    the under-determined Tikhonov form [A, lambda I_m] of Sec. 5)."""
    return M.m >= M.n


def sketch(M: Matrix, s: int, seed: int) -> np.ndarray:
    """X = G T (s x d), the sketch of Alg. 1 (tall) or its transpose (Alg. 2)."""
    d = M.n if is_tall(M) else M.m
    X = np.zeros((s, d))
    st = M._struct()
    rc = lib().orc_sketch(C.byref(st), s, seed, _ptr(X))
    if rc < 0:
        raise ValueError("orc_sketch rejected the input")
    return X


def sketch_bf16(M: "Matrix", s: int, seed: int = 0) -> np.ndarray:
    """The precision form's sketch bf16(G) fl32(T) (s x d), exact products in FP64."""
    d = M.n if is_tall(M) else M.m
    X = np.zeros((s, d))
    st = M._struct()
    lib().orc_sketch_bf16(C.byref(st), s, seed, _ptr(X))
    return X


def bf16_round(f: float) -> float:
    return float(lib().orc_bf16_round(f))


def qr_r(X) -> np.ndarray:
    X = _f64(X)
    s, d = X.shape
    R = np.zeros((d, d))
    if lib().orc_qr_r(s, d, _ptr(X), _ptr(R)) != 0:
        raise ValueError("orc_qr_r rejected the input")
    return R


def jacobi_rt(R, max_sweeps: int = 60):
    R = _f64(R)
    d = R.shape[0]
    W = np.zeros((d, d))
    sweeps = lib().orc_jacobi_rt(d, _ptr(R), _ptr(W), max_sweeps)
    return W, sweeps   # row c of W is column c of the orthogonalised R^T


def precond(X, rcond: float = 0.0):
    """(rank r, sigma (d,), P (d x r), sweeps) for the sketch X (s x d)."""
    X = _f64(X)
    s, d = X.shape
    sigma = np.zeros(d)
    P = np.zeros((d, d))
    sw = C.c_int()
    r = lib().orc_precond(s, d, _ptr(X), rcond, _ptr(sigma), _ptr(P), C.byref(sw))
    return int(r), sigma, P[:, :r].copy(), sw.value


def precond_qr(X, rcond: float = 0.0):
    """(|diag R| descending, P = R^-1 (d x d)) for the sketch X (s x d);
    raises ValueError when the sketch is numerically rank-deficient."""
    X = _f64(X)
    s, d = X.shape
    dg = np.zeros(d)
    P = np.zeros((d, d))
    r = lib().orc_precond_qr(s, d, _ptr(X), rcond, _ptr(dg), _ptr(P))
    if r < 0:
        raise ValueError("rank-deficient sketch")
    return dg, P


def cs_iterations(sigma_l: float, sigma_u: float, eps: float) -> int:
    return int(lib().orc_cs_iterations(sigma_l, sigma_u, eps))


def cs_bounds(s: int, r: int, t: float = 1.0):
    lo, hi = C.c_double(), C.c_double()
    rc = lib().orc_cs_bounds(s, r, t, C.byref(lo), C.byref(hi))
    if rc != 0:
        raise ValueError("sqrt(s) - sqrt(r) - t <= 0")
    return lo.value, hi.value


class _PyLinop:
    """Wrap numpy callables mv(x)->y, mvt(y)->x as an orc_linop."""

    def __init__(self, rows, cols, mv, mvt):
        def _mv(_ctx, x, y):
            xa = np.ctypeslib.as_array(x, shape=(cols,))
            ya = np.ctypeslib.as_array(y, shape=(rows,))
            ya[:] = mv(xa.copy())

        def _mvt(_ctx, y, x):
            ya = np.ctypeslib.as_array(y, shape=(rows,))
            xa = np.ctypeslib.as_array(x, shape=(cols,))
            xa[:] = mvt(ya.copy())

        self._cb = (_MV(_mv), _MV(_mvt))
        self.s = _Linop(rows, cols, self._cb[0], self._cb[1], None)


def lsqr(rows, cols, mv, mvt, b, tol, maxiter):
    """Oracle LSQR on a Python operator.  Returns (x, iters, converged)."""
    op = _PyLinop(rows, cols, mv, mvt)
    b = _f64(b)
    x = np.zeros(cols)
    it = lib().orc_lsqr(C.byref(op.s), _ptr(b), tol, maxiter, _ptr(x))
    return x, abs(int(it)), it >= 0


def cs(rows, cols, mv, mvt, b, sigma_l, sigma_u, eps):
    """Oracle Chebyshev semi-iteration (Alg. 3).  Returns (x, iters)."""
    op = _PyLinop(rows, cols, mv, mvt)
    b = _f64(b)
    x = np.zeros(cols)
    it = lib().orc_cs(C.byref(op.s), _ptr(b), sigma_l, sigma_u, eps, _ptr(x))
    return x, int(it)


# ---------------------------------------------------------------- LSRN

@dataclass
class Result:
    x: np.ndarray
    s: int
    d: int
    rank: int
    iters: int
    sweeps: int
    refine_steps: int
    sigma_l: float
    sigma_u: float
    t_sketch: float
    t_svd: float
    t_iter: float
    t_refine: float
    tall: bool
    converged: bool
    sigma: np.ndarray
    P: np.ndarray
    cs_fallbacks: int = 0


PRECOND_SVD, PRECOND_QR = 0, 1


def lsrn_solve(M: Matrix, b, *, gamma=2.0, tol=1e-14, method=LSQR, seed=0, rcond=0.0,
               t_margin=1.0, max_iter=0, refine=0, precond=PRECOND_SVD) -> Result:
    """LSRN (Alg. 1 / Alg. 2) in the oracle; refine > 0 selects reference mode;
    precond = PRECOND_QR uses N = R^-1 (full-rank sketches only)."""
    b = _f64(b)
    if b.shape[0] != M.m:
        raise ValueError("b has the wrong length")
    o = _Options(gamma, tol, rcond, t_margin, seed, max_iter, method, refine, precond, 0)
    info = _Info()
    x = np.zeros(M.n)
    d = M.n if is_tall(M) else M.m
    sigma = np.zeros(d)
    P = np.zeros((d, d))
    st = M._struct()
    rc = lib().orc_lsrn_solve(C.byref(st), _ptr(b), C.byref(o), _ptr(x), C.byref(info),
                              _ptr(sigma), _ptr(P))
    if rc != 0:
        raise ValueError(f"orc_lsrn_solve failed ({rc})")
    r = int(info.rank)
    return Result(x, info.s, info.d, r, info.iters, info.sweeps, info.refine_steps,
                  info.sigma_l, info.sigma_u, info.t_sketch, info.t_svd, info.t_iter,
                  info.t_refine, bool(info.tall), bool(info.converged), sigma,
                  P[:, :r].copy(), int(info.cs_fallbacks))


def lsrn_iterate(M: Matrix, b, P, s: int, *, tol=1e-14, method=LSQR, t_margin=1.0,
                 max_iter=0, refine=0):
    """Steps 6-7 (and refinement) with a given preconditioner P (d x r).
    Returns (x, iters, converged, info dict of timings)."""
    b = _f64(b)
    P = _f64(P)
    d, r = P.shape
    o = _Options(2.0, tol, 0.0, t_margin, 0, max_iter, method, refine, 0, 0)
    info = _Info()
    x = np.zeros(M.n)
    st = M._struct()
    rc = lib().orc_lsrn_iterate(C.byref(st), _ptr(b), _ptr(P), r, r, s, C.byref(o), _ptr(x),
                                C.byref(info))
    if rc != 0:
        raise ValueError(f"orc_lsrn_iterate failed ({rc})")
    return x, int(info.iters), bool(info.converged), {"t_iter": info.t_iter,
                                                     "t_refine": info.t_refine,
                                                     "refine_steps": int(info.refine_steps),
                                                     "cs_fallbacks": int(info.cs_fallbacks)}


def pinv_solve(M: Matrix, b, rcond: float = 0.0):
    """Brute-force x = A^+ b (long-double Jacobi SVD).  Returns (x, rank)."""
    b = _f64(b)
    x = np.zeros(M.n)
    st = M._struct()
    r = lib().orc_pinv_solve(C.byref(st), _ptr(b), rcond, _ptr(x))
    return x, int(r)


def num_threads() -> int:
    return int(lib().orc_num_threads())
