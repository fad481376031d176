"""Pins for the oracle's sketch (Alg. 1/2 step 3) and its SVD-based
preconditioner (steps 4-5), against brute-force numpy / LAPACK and the
paper's Lemma 2."""
import math

import numpy as np
import pytest

import workloads


def _explicit_T(M, orc):
    """The tall view T (rows x d) built explicitly with numpy."""
    A = M.to_dense()
    if orc.is_tall(M):
        return np.vstack([A, M.lam * np.eye(M.n)]) if M.lam > 0 else A
    return A.T


@pytest.mark.parametrize("shape,kind,lam", [((60, 7), "row", 0.0), ((9, 80), "col", 0.0),
                                            ((50, 12), "row", 0.5), ((33, 5), "csr", 0.0),
                                            ((7, 40), "csr", 0.0), ((40, 6), "csr", 0.25)])
def test_sketch_matches_exact_sum(orc, shape, kind, lam):
    """Entries of A are 0, +-1, +-2, so every product G(i,k) T(k,j) is exact and
    math.fsum gives the correctly rounded X(i,j); the oracle's ascending sum
    must lie within the recursive-summation bound K u sum|G T|."""
    m, n = shape
    rng = np.random.default_rng(m * 100 + n)
    A = rng.integers(-2, 3, size=(m, n)).astype(float)
    A[rng.random((m, n)) < 0.4] = 0.0
    if kind == "row":
        M = orc.Matrix.dense(A, lam=lam)
    elif kind == "col":
        M = orc.Matrix.dense_colmajor(A.T.copy(), lam=lam)
    else:
        rows, cols = np.nonzero(A)
        rowptr = np.zeros(m + 1, np.int64)
        np.add.at(rowptr, rows + 1, 1)
        M = orc.Matrix.csr(m, n, np.cumsum(rowptr), cols.astype(np.int32), A[rows, cols], lam=lam)
    T = _explicit_T(M, orc)
    K, d = T.shape
    s = 2 * d + 1
    X = orc.sketch(M, s, seed=99)
    G = orc.gauss_fill(99, 0, s, 0, K)
    for i in range(s):
        for j in range(d):
            terms = G[i] * T[:, j]
            exact = math.fsum(terms)
            bound = K * np.finfo(float).eps * np.abs(terms).sum()
            assert abs(X[i, j] - exact) <= bound + 1e-300


def test_sketch_csr_equals_dense(orc):
    S = workloads.sparse_problem(300, 40, per_row=5, n_dense=3, fill=0.3, seed=5)
    D = S.to_dense()
    Xs = orc.sketch(orc.Matrix.csr(S.m, S.n, S.rowptr, S.colind, S.val, lam=0.1), 81, 4)
    Xd = orc.sketch(orc.Matrix.dense(D, lam=0.1), 81, 4)
    np.testing.assert_allclose(Xs, Xd, rtol=0, atol=1e-12 * np.abs(Xd).max())


def test_qr_r_against_lapack(orc):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((90, 40)) @ np.diag(10.0 ** np.linspace(0, -6, 40))
    R = orc.qr_r(X)
    assert np.allclose(np.tril(R, -1), 0.0)
    np.testing.assert_allclose(R.T @ R, X.T @ X, atol=1e-13 * np.linalg.norm(X) ** 2)
    Rl = np.linalg.qr(X, mode="r")
    np.testing.assert_allclose(np.abs(np.diag(R)), np.abs(np.diag(Rl)), rtol=1e-9)


def test_jacobi_against_lapack(orc):
    rng = np.random.default_rng(2)
    X = rng.standard_normal((120, 50)) @ np.diag(10.0 ** np.linspace(0, -8, 50))
    R = orc.qr_r(X)
    W, sweeps = orc.jacobi_rt(R)
    assert 0 < sweeps < 30
    nrm = np.linalg.norm(W, axis=1)
    C = (W @ W.T) / np.outer(nrm, nrm)
    assert np.abs(C - np.eye(50)).max() < 1e-13          # relative orthogonality
    np.testing.assert_allclose(W.T @ W, R.T @ R, atol=1e-13 * np.linalg.norm(R) ** 2)
    sv = np.linalg.svd(X, compute_uv=False)
    np.testing.assert_allclose(np.sort(nrm)[::-1], sv, rtol=1e-10)


def test_precond_rank_deficient(orc):
    """rank(X) = 30 of 50: r = 30, X N orthonormal, range(N) = range(X^T)."""
    P = workloads.dense_problem(400, 50, rank=30, smin=1e-4, seed=3)
    M = orc.Matrix.dense(P.A)
    X = orc.sketch(M, 100, 17)
    r, sigma, N, _ = orc.precond(X)
    assert r == 30
    Q = X @ N
    assert np.abs(Q.T @ Q - np.eye(r)).max() < 1e-9
    Vx = np.linalg.svd(X)[2][:30].T                       # basis of range(X^T)
    assert np.linalg.norm(N - Vx @ (Vx.T @ N)) / np.linalg.norm(N) < 1e-10
    np.testing.assert_allclose(sigma[:r], np.linalg.svd(X, compute_uv=False)[:r], rtol=1e-8)


def test_lemma2_spectrum_of_AN(orc):
    """Lemma 2: the singular values of A N are those of (G U)^+, independent of A."""
    for kappa in (1e2, 1e6):
        P = workloads.dense_problem(500, 40, smin=1 / kappa, seed=4)
        M = orc.Matrix.dense(P.A)
        s = 80
        X = orc.sketch(M, s, 21)
        r, _, N, _ = orc.precond(X)
        assert r == 40
        sv_an = np.linalg.svd(P.A @ N, compute_uv=False)
        G = orc.gauss_fill(21, 0, s, 0, 500)
        sv_gu = np.sort(1.0 / np.linalg.svd(G @ P.U, compute_uv=False))[::-1]
        np.testing.assert_allclose(sv_an, sv_gu, rtol=1e-9 if kappa < 1e3 else 1e-6)


def test_fat_precond_is_left_preconditioner(orc):
    """Alg. 2: range(M) = range(A) and M^T A has the same spectrum bound."""
    P = workloads.dense_problem(600, 30, rank=25, smin=1e-5, seed=6)
    Afat = P.A.T.copy()                                   # 30 x 600, rank 25
    M = orc.Matrix.dense(Afat)
    X = orc.sketch(M, 60, 8)                              # = (A G)^T, 60 x 30
    r, _, Mp, _ = orc.precond(X)
    assert r == 25
    Ua = np.linalg.svd(Afat)[0][:, :25]
    assert np.linalg.norm(Mp - Ua @ (Ua.T @ Mp)) / np.linalg.norm(Mp) < 1e-9
    sv = np.linalg.svd(Mp.T @ Afat, compute_uv=False)
    assert sv[0] / sv[-1] < 8.0
