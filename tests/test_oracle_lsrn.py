"""Pins for the oracle's full LSRN solve (Alg. 1, Alg. 2, Sec. 5) against the
plain definition x* = A^+ b (Sec. 1-2), optimality invariants and the
paper's theorems."""
import numpy as np
import pytest

import workloads


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _exact_rankdef(m, n, rank, seed):
    """A whose trailing n - rank columns are copies of leading ones scaled by
    powers of two, so the rank deficiency is exact in floating point."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((m, rank)) @ np.diag(10.0 ** np.linspace(0, -3, rank))
    extra = [B[:, j % rank] * 2.0 ** (-(j % 3) - 1) for j in range(n - rank)]
    return np.column_stack([B] + extra) if extra else B


@pytest.mark.parametrize("m,n,rank", [(40, 7, 7), (9, 31, 9), (30, 12, 8), (12, 35, 5)])
def test_pinv_matches_numpy(orc, m, n, rank):
    A = _exact_rankdef(m, n, rank, m + n)
    b = np.random.default_rng(1).standard_normal(m)
    x, r = orc.pinv_solve(orc.Matrix.dense(A), b)
    assert r == rank
    np.testing.assert_allclose(x, np.linalg.pinv(A, rcond=1e-10) @ b, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("m,n,rank", [(64, 10, 10), (64, 10, 6), (10, 64, 10), (10, 64, 6)])
def test_lsrn_matches_bruteforce_tiny(orc, method, m, n, rank):
    A = _exact_rankdef(m, n, rank, 3 * m + n)
    b = np.random.default_rng(2).standard_normal(m)
    M = orc.Matrix.dense(A)
    xp, r = orc.pinv_solve(M, b)
    res = orc.lsrn_solve(M, b, method=method, seed=3, refine=3)
    assert res.rank == rank == r
    assert res.tall == (m >= n)
    assert _rel(res.x, xp) < 1e-11


def test_lsrn_colmajor_storage_is_the_same_problem(orc):
    A = _exact_rankdef(12, 70, 9, 5)
    b = np.random.default_rng(3).standard_normal(12)
    r1 = orc.lsrn_solve(orc.Matrix.dense(A), b, seed=1, refine=2)
    r2 = orc.lsrn_solve(orc.Matrix.dense_colmajor(A.T.copy()), b, seed=1, refine=2)
    assert _rel(r1.x, r2.x) < 1e-12


def test_tikhonov_normal_equations(orc):
    """Sec. 5: with W = lambda I the solution satisfies (A^T A + lambda^2 I) x = A^T b."""
    P = workloads.dense_problem(300, 20, smin=1e-6, seed=8)
    b = workloads.rhs_gauss(300, 8)
    lam = 1e-3
    res = orc.lsrn_solve(orc.Matrix.dense(P.A, lam=lam), b, seed=2, refine=3)
    ref = np.linalg.solve(P.A.T @ P.A + lam * lam * np.eye(20), P.A.T @ b)
    assert _rel(res.x, ref) < 1e-10
    assert res.s == 40 and res.rank == 20


def test_tikhonov_sparse_equals_dense(orc):
    S = workloads.sparse_problem(400, 25, per_row=4, n_dense=2, fill=0.2, seed=9)
    b = workloads.rhs_gauss(400, 9)
    rs = orc.lsrn_solve(orc.Matrix.csr(S.m, S.n, S.rowptr, S.colind, S.val, lam=1e-2), b,
                        seed=4, refine=2)
    rd = orc.lsrn_solve(orc.Matrix.dense(S.to_dense(), lam=1e-2), b, seed=4, refine=2)
    assert _rel(rs.x, rd.x) < 1e-12


def test_theorem2_solution_does_not_depend_on_G(orc):
    P = workloads.dense_problem(2000, 100, smin=1e-6, seed=11)
    b, _ = workloads.rhs_model(P.A, 1e-3, 11)
    M = orc.Matrix.dense(P.A)
    xs = [orc.lsrn_solve(M, b, seed=s, refine=3, method=m).x for s, m in ((1, 0), (2, 1), (3, 0))]
    assert _rel(xs[0], xs[1]) < 1e-12 and _rel(xs[0], xs[2]) < 1e-12
    xp, _ = orc.pinv_solve(M, b)
    assert _rel(xs[0], xp) < 1e-11


def test_invariants_rank_deficient(orc):
    """A^T (b - A x) = 0 and x in range(A^T) for a rank-deficient tall A.

    A = U diag(sigma) V^T is stored in floating point, so its row space is
    only defined to about eps * sigma_1 / sigma_r = 1e-10; the bounds below
    sit at that floor (unrefined FP64 gives ~1e-12 for the first one)."""
    P = workloads.dense_problem(3000, 120, rank=100, smin=1e-6, seed=12)
    b = workloads.rhs_gauss(3000, 12)
    for method in (0, 1):
        res = orc.lsrn_solve(orc.Matrix.dense(P.A), b, seed=5, method=method, refine=3)
        assert res.rank == 100
        Al = P.A.astype(np.longdouble)
        rr = b.astype(np.longdouble) - Al @ res.x.astype(np.longdouble)
        ne = np.linalg.norm((Al.T @ rr).astype(float))
        assert ne / (np.linalg.norm(P.A, 2) * np.linalg.norm(rr.astype(float))) < 5e-13
        out = res.x - P.V @ (P.V.T @ res.x)
        assert np.linalg.norm(out) / np.linalg.norm(res.x) < 1e-9


def test_iteration_counts_follow_theorem4(orc):
    """LSQR stays under the Theorem 4 bound (alpha -> 0); CS takes the count of
    Alg. 3 with Theorem 3's bounds (t = 1)."""
    P = workloads.dense_problem(2000, 100, smin=1e-6, seed=11)
    b, _ = workloads.rhs_model(P.A, 1e-3, 11)
    M = orc.Matrix.dense(P.A)
    lq = orc.lsrn_solve(M, b, seed=9, method=0)
    cs = orc.lsrn_solve(M, b, seed=9, method=1)
    s, r = 200, 100
    bound = (np.log(1e-14) - np.log(2)) / np.log(np.sqrt(r / s))
    assert lq.iters <= bound
    sl, su = orc.cs_bounds(s, r, 1.0)
    assert cs.iters == orc.cs_iterations(sl, su, 1e-14) == 133
    sv = np.linalg.svd(P.A @ cs.P, compute_uv=False)
    assert sl <= sv[-1] and sv[0] <= su


def test_fat_rank_deficient_min_length(orc):
    P = workloads.dense_problem(2500, 60, rank=50, smin=1e-6, seed=13)
    A = P.A.T.copy()                                     # 60 x 2500, rank 50
    b = workloads.rhs_gauss(60, 13)
    for method in (0, 1):
        res = orc.lsrn_solve(orc.Matrix.dense_colmajor(P.A.copy()), b, seed=6, method=method,
                             refine=3)
        assert not res.tall and res.rank == 50
        xp, _ = orc.pinv_solve(orc.Matrix.dense(A), b, rcond=1e-9)
        assert _rel(res.x, xp) < 1e-9


@pytest.mark.parametrize("lam", [1e-2, 0.3])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("storage", ["dense", "colmajor", "csr"])
def test_tikhonov_under_determined_closed_form(orc, lam, method, storage):
    """Sec. 5's under-determined form: for m < n the Tikhonov solution is the
    first n entries of the min-length solution of [A, lambda I_m] x^ = b,
    i.e. x = A^T (A A^T + lambda^2 I)^-1 b (the minimiser of
    ||A x - b||^2 + lambda^2 ||x||^2), for a rank-deficient A as well."""
    rng = np.random.default_rng(int(lam * 1000) + method)
    A = _exact_rankdef(800, 40, 30, 77).T.copy()          # 40 x 800, rank 30
    b = rng.standard_normal(40)
    x_ref = A.T @ np.linalg.solve(A @ A.T + lam * lam * np.eye(40), b)
    if storage == "dense":
        M = orc.Matrix.dense(A, lam=lam)
    elif storage == "colmajor":
        M = orc.Matrix.dense_colmajor(A.T.copy(), lam=lam)
    else:
        rows, cols = np.nonzero(A)
        rowptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=40))])
        M = orc.Matrix.csr(40, 800, rowptr, cols.astype(np.int32), A[rows, cols], lam=lam)
    res = orc.lsrn_solve(M, b, seed=4, method=method, refine=2)
    assert not res.tall and res.rank == 40 and res.s == 80
    assert _rel(res.x, x_ref) < 1e-11
    # the stationarity condition of the regularised problem
    g = A.T @ (A @ res.x - b) + lam * lam * res.x
    assert np.linalg.norm(g) <= 1e-11 * np.linalg.norm(A.T @ b)
