"""Seeded synthetic inputs shaped like the paper's workloads.

Both the oracle side and the GPU side of every test draw their inputs from
here.  Nothing in this module computes any part of LSRN: it only builds
matrices and right-hand sides whose spectra and sparsity the tests need.

Recipes (Sec. 6 of the paper uses random dense matrices with a chosen
condition number, rank-deficient variants, and sprandn-like sparse matrices):

* dense_problem: A = U diag(sigma) V^T, U (m x k) and V (n x k) Haar-distributed
  with orthonormal columns (QR of a Gaussian with the signs of diag(R) fixed,
  Mezzadri 2007), sigma log-spaced from 1 down to sigma_min, k = rank.
* rhs: b = A x_gen + noise * N(0,1), or b ~ N(0,1).
* sparse_problem: CSR with `per_row` distinct uniform-random columns per row plus
  `n_dense` chosen columns each filled with probability `fill`, values N(0,1),
  column indices sorted in each row.
* Under-determined inputs are the transpose construction: the row-major array
  of a tall matrix read as the column-major storage of its transpose.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def haar_columns(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """rows x cols with orthonormal columns, Haar-distributed."""
    Z = rng.standard_normal((rows, cols))
    Q, R = np.linalg.qr(Z)
    Q *= np.sign(np.diag(R))
    return Q


def logspaced(k: int, smin: float) -> np.ndarray:
    if k == 1:
        return np.ones(1)
    return 10.0 ** np.linspace(0.0, np.log10(smin), k)


@dataclass
class Dense:
    A: np.ndarray        # m x n, row-major
    U: np.ndarray        # m x k
    sigma: np.ndarray    # k
    V: np.ndarray        # n x k


def dense_problem(m: int, n: int, rank: int | None = None, smin: float = 1e-6,
                  seed: int = 0) -> Dense:
    """A = U diag(sigma) V^T (m x n) with the given rank (default min(m, n))."""
    k = min(m, n) if rank is None else rank
    rng = np.random.default_rng(seed)
    U = haar_columns(rng, m, k)
    V = haar_columns(rng, n, k)
    sigma = logspaced(k, smin)
    A = (U * sigma) @ V.T
    return Dense(np.ascontiguousarray(A), U, sigma, V)


CHUNK_ELEMS = 1 << 28  # every torch BLAS / solver call stays far below 2^31 elements


def _row_chunks(rows: int, cols: int):
    step = max(1, CHUNK_ELEMS // max(cols, 1))
    for r0 in range(0, rows, step):
        yield r0, min(rows, r0 + step)


def haar_device(rows: int, k: int, g, device="cuda"):
    """Haar-distributed rows x k orthonormal columns: Z R^-1 with R the
    Cholesky factor of Z^T Z, Z Gaussian (the Q factor of Z with positive
    diag R), formed in row chunks."""
    import torch
    Z = torch.empty(rows, k, dtype=torch.float64, device=device)
    for r0, r1 in _row_chunks(rows, k):
        Z[r0:r1] = torch.randn(r1 - r0, k, generator=g, dtype=torch.float64, device=device)
    if rows * k <= CHUNK_ELEMS:
        Q, R = torch.linalg.qr(Z)
        return Q * torch.sign(torch.diagonal(R))
    # kappa(Z) is about (sqrt(rows) + sqrt(k)) / (sqrt(rows) - sqrt(k)), so
    # one Cholesky QR pass is orthonormal to rounding; a second pass removes
    # what is left
    for _ in range(2):
        C = torch.zeros(k, k, dtype=torch.float64, device=device)
        for r0, r1 in _row_chunks(rows, k):
            C += Z[r0:r1].T @ Z[r0:r1]
        R = torch.linalg.cholesky(C, upper=True)
        # kappa(R) ~ 1: multiply by the explicit inverse (a plain GEMM per chunk)
        Rinv = torch.linalg.solve_triangular(R, torch.eye(k, dtype=R.dtype, device=R.device),
                                             upper=True)
        for r0, r1 in _row_chunks(rows, k):
            Z[r0:r1] = Z[r0:r1] @ Rinv
    return Z


def dense_problem_device(m: int, n: int, rank: int | None = None, smin: float = 1e-6,
                         seed: int = 0, device="cuda"):
    """The dense_problem recipe built with torch on `device` (for sizes where
    the host QR would dominate set-up).  Returns (A, U, sigma, V) tensors."""
    import torch
    k = min(m, n) if rank is None else rank
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    U = haar_device(m, k, g, device)
    V = haar_device(n, k, g, device)
    sigma = torch.logspace(0.0, float(np.log10(smin)), k, dtype=torch.float64, device=device)
    A = torch.empty(m, n, dtype=torch.float64, device=device)
    W = (V * sigma).T.contiguous()                     # k x n
    for r0, r1 in _row_chunks(m, max(n, k)):
        A[r0:r1] = U[r0:r1] @ W
    return A, U, sigma, V


def reflected_problem_device(m: int, n: int, cond: float, seed: int, device="cuda",
                             reflectors: int = 4):
    """An m x n (m >= n) matrix with singular values log-spaced from 1 to
    1/cond, built in O(m n): A = H_1 ... H_k [Sigma V^T; 0] with V Haar (n x n)
    and H_i = I - 2 u_i u_i^T for random unit u_i.  The cheap generator of the
    serving workload (a request's matrix is made when it arrives)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    Z = torch.randn(n, n, generator=g, dtype=torch.float64, device=device)
    Q, R = torch.linalg.qr(Z)
    V = Q * torch.sign(torch.diagonal(R))
    sigma = torch.logspace(0.0, -float(np.log10(cond)), n, dtype=torch.float64, device=device)
    A = torch.zeros(m, n, dtype=torch.float64, device=device)
    A[:n] = sigma[:, None] * V.T
    for _ in range(reflectors):
        u = torch.randn(m, generator=g, dtype=torch.float64, device=device)
        u /= torch.linalg.norm(u)
        A -= 2.0 * torch.outer(u, u @ A)
    return A


def matvec_device(A, x, trans: bool = False):
    """A x (or A^T x) in row chunks."""
    import torch
    m, n = A.shape
    dt = x.dtype  # FP32-stored A is widened chunk by chunk
    if not trans:
        out = torch.empty(m, dtype=dt, device=A.device)
        for r0, r1 in _row_chunks(m, n):
            out[r0:r1] = A[r0:r1].to(dt) @ x
        return out
    out = torch.zeros(n, dtype=dt, device=A.device)
    for r0, r1 in _row_chunks(m, n):
        out += A[r0:r1].to(dt).T @ x[r0:r1]
    return out


def rhs_gauss_device(m: int, seed: int, device="cuda"):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed + 104729)
    return torch.randn(m, generator=g, dtype=torch.float64, device=device)


def rhs_model_device(A, noise: float, seed: int):
    """rhs_model's recipe with torch on A's device: (b, x_gen) tensors."""
    import torch
    g = torch.Generator(device=A.device)
    g.manual_seed(seed + 7919)
    xg = torch.randn(A.shape[1], generator=g, dtype=torch.float64, device=A.device)
    b = matvec_device(A, xg) + noise * torch.randn(A.shape[0], generator=g, dtype=torch.float64,
                                                   device=A.device)
    return b, xg


def rhs_model(A: np.ndarray, noise: float, seed: int):
    """b = A x_gen + noise * N(0,1); returns (b, x_gen)."""
    rng = np.random.default_rng(seed + 7919)
    xg = rng.standard_normal(A.shape[1])
    b = A @ xg + noise * rng.standard_normal(A.shape[0])
    return b, xg


def rhs_gauss(m: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed + 104729).standard_normal(m)


@dataclass
class Sparse:
    m: int
    n: int
    rowptr: np.ndarray   # int64, m+1
    colind: np.ndarray   # int32, nnz (sorted within each row)
    val: np.ndarray      # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_dense(self) -> np.ndarray:
        A = np.zeros((self.m, self.n))
        rows = np.repeat(np.arange(self.m), np.diff(self.rowptr))
        A[rows, self.colind] = self.val
        return A


def sparse_problem(m: int, n: int, per_row: int = 20, n_dense: int = 10,
                   fill: float = 0.1, seed: int = 0, chunk: int = 1 << 18) -> Sparse:
    """CSR m x n: per_row distinct uniform columns per row, plus n_dense fixed
    columns each present with probability `fill` (a collision keeps one
    entry); values N(0,1)."""
    rng = np.random.default_rng(seed)
    dense_cols = np.sort(rng.choice(n, size=min(n_dense, n), replace=False)).astype(np.int64)
    counts = np.zeros(m, np.int64)
    cols_parts, val_parts = [], []
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        rows = r1 - r0
        # distinct columns per row: sample with replacement and redraw duplicates
        c = rng.integers(0, n, size=(rows, per_row), dtype=np.int64)
        c.sort(axis=1)
        dup = np.zeros_like(c, dtype=bool)
        dup[:, 1:] = c[:, 1:] == c[:, :-1]
        while dup.any():
            c[dup] = rng.integers(0, n, size=int(dup.sum()), dtype=np.int64)
            c.sort(axis=1)
            dup[:] = False
            dup[:, 1:] = c[:, 1:] == c[:, :-1]
        hit = rng.random((rows, dense_cols.size)) < fill
        full = np.concatenate([c, np.where(hit, dense_cols[None, :], -1)], axis=1)
        full.sort(axis=1)
        keep = full >= 0
        keep[:, 1:] &= full[:, 1:] != full[:, :-1]
        cnt = keep.sum(axis=1)
        counts[r0:r1] = cnt
        cols_parts.append(full[keep].astype(np.int32))
        val_parts.append(rng.standard_normal(int(cnt.sum())))
    rowptr = np.zeros(m + 1, np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return Sparse(m, n, rowptr, np.concatenate(cols_parts), np.concatenate(val_parts))


# The five workloads the build is measured on (sizes of the dense, rank-
# deficient, sparse, precision and serving cases).  Each entry is what the
# generator needs; solver settings live with the tests and the benchmark.
WORKLOADS = {
    "dense_2000x100": dict(m=2000, n=100, rank=100, smin=1e-6, noise=1e-3, seed=11),
    "rankdef_200000x2000": dict(m=200_000, n=2000, rank=1800, smin=1e-6, seed=12),
    "sparse_2000000x20000": dict(m=2_000_000, n=20_000, per_row=20, n_dense=10, fill=0.1,
                                 lam=1e-3, seed=13),
    "dense_1000000x4000": dict(m=1_000_000, n=4000, rank=4000, smin=1e-8, noise=1e-6, seed=14),
}


def tnimg_like(n: int, m: int = 1024, seed: int = 0, chunk: int = 1 << 18) -> Sparse:
    """A synthetic stand-in for the paper's tnimg matrices (Sec. 6.5): m = 1024
    rows (the 32 x 32 two-dimensional DCT frequencies (u, v) of an image,
    row 32 u + v), n columns (images), each column keeping 20 or 21
    coefficients (the largest 2% of 1024; 21 with probability 0.9, so about
    21 n nonzeros as in the paper's tables).  Row 0 (the DC term) is in every
    column with a value in (0.5, 30); the others are drawn without
    replacement with probability proportional to (1 + u + v)^-1.5 and get
    N(0,1) values scaled by 8 / (1 + u + v), as the magnitudes of an image's
    DCT fall with frequency.  Rows that end up empty are removed (as in the
    paper), so m may come out smaller.  Returned in CSR (rows sorted by
    column within each row)."""
    rng = np.random.default_rng(seed)
    u, v = np.divmod(np.arange(m, dtype=np.int64), 32)
    freq = (1 + u + v).astype(np.float64)
    w = freq[1:] ** -1.5
    cdf = np.cumsum(w / w.sum())
    cdf[-1] = 1.0
    rows_parts, cols_parts, val_parts = [], [], []
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        k = c1 - c0
        per = np.where(rng.random(k) < 0.9, 21, 20)
        # 20 draws from rows 1..m-1 per column (distinct), the 21st slot kept
        # only where per == 21; row 0 added separately
        draw = 1 + np.searchsorted(cdf, rng.random((k, 20)))
        draw.sort(axis=1)
        dup = np.zeros_like(draw, dtype=bool)
        dup[:, 1:] = draw[:, 1:] == draw[:, :-1]
        while dup.any():
            draw[dup] = 1 + np.searchsorted(cdf, rng.random(int(dup.sum())))
            draw.sort(axis=1)
            dup[:] = False
            dup[:, 1:] = draw[:, 1:] == draw[:, :-1]
        keep = np.ones_like(draw, dtype=bool)
        keep[per == 20, 19] = False                    # 19 draws + row 0 = 20 entries
        cols = np.repeat(np.arange(c0, c1, dtype=np.int64), keep.sum(axis=1))
        rws = draw[keep]
        vals = rng.standard_normal(rws.size) * (8.0 / freq[rws])
        dc = rng.uniform(0.5, 30.0, k)
        rows_parts += [np.zeros(k, np.int64), rws]
        cols_parts += [np.arange(c0, c1, dtype=np.int64), cols]
        val_parts += [dc, vals]
    rows = np.concatenate(rows_parts)
    cols = np.concatenate(cols_parts)
    vals = np.concatenate(val_parts)
    # drop empty rows, renumbering the others in order
    present = np.bincount(rows, minlength=m) > 0
    newid = np.cumsum(present) - 1
    rows = newid[rows]
    m_eff = int(present.sum())
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(m_eff + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=m_eff), out=rowptr[1:])
    return Sparse(m_eff, n, rowptr, cols.astype(np.int32), vals)
