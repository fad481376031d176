"""Pins of the oracle's full-rank preconditioner N = R^-1 and of the sparse
oracle path, against LAPACK and the normal equations (not against itself)."""
import numpy as np
import pytest
import scipy.linalg as sl

import workloads


@pytest.mark.parametrize("s,d", [(60, 25), (200, 100), (33, 33)])
def test_precond_qr_is_inverse_of_lapack_r(orc, s, d):
    rng = np.random.default_rng(s * 3 + d)
    X = rng.standard_normal((s, d)) @ np.diag(10.0 ** np.linspace(0, -3, d))
    dg, P = orc.precond_qr(X)
    R = sl.qr(X, mode="r")[0][:d]
    # LAPACK's R equals the oracle's up to the sign of each row: |R P| = I
    np.testing.assert_allclose(np.abs(R @ P), np.eye(d), atol=1e-10)
    assert np.all(np.tril(P, -1) == 0.0)
    Q = X @ P
    np.testing.assert_allclose(Q.T @ Q, np.eye(d), atol=1e-10)
    np.testing.assert_allclose(dg, np.sort(np.abs(np.diag(R)))[::-1], rtol=1e-12)


def test_precond_qr_rejects_rank_deficient(orc):
    rng = np.random.default_rng(2)
    X = rng.standard_normal((50, 10))
    X[:, 4] = 3.0 * X[:, 1]
    with pytest.raises(ValueError):
        orc.precond_qr(X)


@pytest.mark.parametrize("method", [0, 1])
def test_lsrn_qr_precond_solves_tikhonov_normal_equations(orc, method):
    """With N = R^-1 the oracle LSRN solves (A^T A + lam^2 I) x = A^T b."""
    S = workloads.sparse_problem(3000, 60, per_row=6, n_dense=3, fill=0.2, seed=8)
    A = S.to_dense()
    b = workloads.rhs_gauss(3000, 8)
    lam = 1e-2
    M = orc.Matrix.csr(S.m, S.n, S.rowptr, S.colind, S.val, lam=lam)
    res = orc.lsrn_solve(M, b, seed=4, method=method, tol=1e-14, precond=orc.PRECOND_QR, refine=2)
    assert res.rank == 60 and res.sweeps == 0
    xr = np.linalg.solve(A.T @ A + lam * lam * np.eye(60), A.T @ b)
    assert np.linalg.norm(res.x - xr) / np.linalg.norm(xr) < 1e-12


def test_sparse_fat_oracle_is_min_length(orc):
    """The CSR oracle on an under-determined A returns A^+ b (brute force)."""
    S = workloads.sparse_problem(40, 300, per_row=12, n_dense=2, fill=0.3, seed=9)
    b = workloads.rhs_gauss(40, 9)
    res = orc.lsrn_solve(orc.Matrix.csr(S.m, S.n, S.rowptr, S.colind, S.val), b, seed=2, refine=2)
    xp, r = orc.pinv_solve(orc.Matrix.dense(S.to_dense()), b)
    assert res.rank == r == 40
    assert np.linalg.norm(res.x - xp) / np.linalg.norm(xp) < 1e-12
