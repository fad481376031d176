"""Sparse (CSR) path and the QR-inverse preconditioner on the GPU, through
the C ABI, against the CPU oracle on seeded synthetic inputs, and at the
full 2,000,000 x 20,000 size against properties that hold at any size."""
import math

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1109_5981_amd import lsrn
    lsrn.lib()  # raises if the library is missing: there is no CPU fallback
    return lsrn


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def gcsr(L, S):
    return L.Csr.from_host(S.m, S.n, S.rowptr, S.colind, S.val)


def ocsr(orc, S, lam=0.0):
    return orc.Matrix.csr(S.m, S.n, S.rowptr, S.colind, S.val, lam=lam)


# ------------------------------------------------------------ sparse sketch

@pytest.mark.parametrize("m,n,per_row,lam,s", [
    (3000, 200, 20, 0.0, 57),        # tall, one column block, ragged sketch rows
    (20000, 5000, 6, 1e-3, 41),      # tall, two column blocks (4096 + 904), Tikhonov rows
    (1500, 30000, 4, 0.0, 18),       # fat: T = A^T (transposed structure), 30000 rows of T
    (257, 9, 3, 0.0, 19),            # tiny, rows of T not a multiple of the batch
    (20000, 5000, 1, 0.0, 41),       # ~1.6 nonzeros per row: 4 sketch rows per tile, rows split
    (20000, 1024, 20, 0.0, 4096),    # 8 sketch rows per tile, 512 tiles (rows of T not split)
])
def test_sketch_csr_matches_oracle(L, orc, m, n, per_row, lam, s):
    S = workloads.sparse_problem(m, n, per_row=per_row, n_dense=2, fill=0.3, seed=m + n)
    seed = 77
    Xo = orc.sketch(ocsr(orc, S, lam), s, seed)
    Xg = host(L.sketch_csr(gcsr(L, S), s, seed=seed, lam=lam)).T
    assert Xg.shape == Xo.shape
    # both sides round every product and sum: |dX| <= 2 K u |G| |T|
    T = S.to_dense() if m >= n else S.to_dense().T
    if lam > 0:
        T = np.vstack([T, lam * np.eye(T.shape[1])])
    G = orc.gauss_fill(seed, 0, s, 0, T.shape[0])
    bound = (2 * T.shape[0] * np.finfo(float).eps + 1e-14) * (np.abs(G) @ np.abs(T)) + 1e-300
    assert np.all(np.abs(Xg - Xo) <= bound)


def test_sketch_csr_is_deterministic(L):
    S = workloads.sparse_problem(20000, 5000, per_row=6, n_dense=2, fill=0.3, seed=5)
    A = gcsr(L, S)
    x1 = host(L.sketch_csr(A, 33, seed=4))
    x2 = host(L.sketch_csr(A, 33, seed=4))
    np.testing.assert_array_equal(x1, x2)


# ----------------------------------------------------- QR-inverse precond

@pytest.mark.parametrize("s,d,spread", [(200, 100, 1e-3), (263, 131, 1e-2), (300, 150, 1e-3), (700, 333, 1e-6)])
def test_precond_qr_matches_oracle(L, orc, s, d, spread):
    rng = np.random.default_rng(s + d)
    X = rng.standard_normal((s, d)) @ np.diag(10.0 ** np.linspace(0, np.log10(spread), d))
    dg_o, P_o = orc.precond_qr(X)
    dg_g, P_g = L.precond_qr(dev(X.T.copy()))
    dg_g, P_g = host(dg_g), host(P_g)
    eps = np.finfo(float).eps
    kappa = np.linalg.cond(X)
    # the library takes R from the Cholesky factor of X^T X while its
    # estimate of kappa keeps d eps kappa^2 <= 1e-5, else from Householder
    # QR: backward errors of order d eps kappa^2 and d eps kappa
    # respectively (these cases lie far on either side of the threshold)
    cholesky = kappa ** 2 * d * eps <= 1e-5
    err = 10 * d * eps * kappa ** 2 if cholesky else 100 * d * eps * kappa
    assert (spread >= 1e-3) == cholesky
    np.testing.assert_allclose(dg_g, dg_o, rtol=err, atol=0)
    # P = R^-1 is unique up to the signs of R's rows; P P^T = (X^T X)^-1 is
    # unique, and X P has orthonormal columns
    assert np.abs(np.tril(P_g, -1)).max() == 0.0
    PPo, PPg = P_o @ P_o.T, P_g @ P_g.T
    assert np.linalg.norm(PPg - PPo) / np.linalg.norm(PPo) < err
    Q = X @ P_g
    assert np.linalg.norm(Q.T @ Q - np.eye(d), 2) < err


def test_precond_qr_unit_diagonal_ill_conditioned(L):
    """A sketch whose R has a unit diagonal (ratio 1) but kappa 2.8e6: the
    diagonal ratio alone would keep Cholesky QR (orthogonality lost to
    about 8e-6 here); the kappa estimate sends it to Householder QR, whose
    X R^-1 is orthonormal to the order of d eps kappa."""
    d, s = 40, 100
    R0 = np.eye(d) - 0.4 * np.triu(np.ones((d, d)), 1)
    Q0, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((s, d)))
    X = Q0 @ R0
    kappa = np.linalg.cond(X)
    assert 1e6 < kappa < 1e7
    _, P_g = L.precond_qr(dev(X.T.copy()))
    Q = X @ host(P_g)
    assert np.linalg.norm(Q.T @ Q - np.eye(d), 2) < 100 * d * np.finfo(float).eps * kappa


def test_precond_qr_rejects_rank_deficient(L):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((100, 40))
    X[:, 7] = X[:, 3]
    with pytest.raises(L.LSRNError) as e:
        L.precond_qr(dev(X.T.copy()))
    assert e.value.status == 5


# --------------------------------------------------------- iterations

@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("shape", ["tall", "fat", "tikhonov"])
def test_iterate_csr_matches_oracle_with_same_preconditioner(L, orc, method, shape):
    if shape == "fat":
        S = workloads.sparse_problem(90, 4000, per_row=12, n_dense=3, fill=0.2, seed=41)
        lam = 0.0
    else:
        S = workloads.sparse_problem(4000, 90, per_row=8, n_dense=3, fill=0.2, seed=42)
        lam = 1e-2 if shape == "tikhonov" else 0.0
    b = workloads.rhs_gauss(S.m, 43)
    res = orc.lsrn_solve(ocsr(orc, S, lam), b, seed=3, method=method)
    xg, info = L.iterate_csr(gcsr(L, S), dev(b), dev(res.P), res.s, method=method, lam=lam)
    assert rel(host(xg), res.x) < 1e-11
    if method == 1:
        assert info["iters"] == res.iters
    else:
        assert abs(info["iters"] - res.iters) <= 1


# --------------------------------------------------------- end to end

@pytest.fixture(scope="module")
def sparse_replica(orc):
    """The sparse Tikhonov workload's structure at 1/100 of its rows and
    columns: 20 uniform columns per row plus 10 columns with 10% fill,
    N(0,1) values, lambda = 1e-3, b ~ N(0,1)."""
    S = workloads.sparse_problem(20000, 200, per_row=20, n_dense=10, fill=0.1, seed=13)
    b = workloads.rhs_gauss(S.m, 13)
    ref = orc.lsrn_solve(ocsr(orc, S, 1e-3), b, seed=1, tol=1e-12, refine=3)
    return S, b, ref


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precond", ["svd", "qr"])
def test_solve_csr_replica_refined_1e10(L, sparse_replica, method, precond):
    S, b, ref = sparse_replica
    x, info = L.solve_csr(gcsr(L, S), dev(b), lam=1e-3, tol=1e-12, seed=7, method=method,
                          refine=2, precond=precond)
    assert info["tall"] == 1 and info["rank"] == 200 and info["s"] == 400
    assert rel(host(x), ref.x) <= 1e-10


def test_solve_csr_fat_rank_deficient(L, orc):
    # under-determined, with a scaled and a repeated row: rank 58 of 60
    S = workloads.sparse_problem(60, 3000, per_row=30, n_dense=2, fill=0.3, seed=17)
    rowptr, colind, val = S.rowptr.copy(), S.colind.copy(), S.val.copy()
    dense = S.to_dense()
    dense[5] = dense[9] * 2.0
    dense[11] = dense[12]
    keep = np.nonzero(dense)
    rowptr = np.zeros(61, np.int64)
    np.add.at(rowptr, keep[0] + 1, 1)
    rowptr = np.cumsum(rowptr)
    S2 = workloads.Sparse(60, 3000, rowptr, keep[1].astype(np.int32), dense[keep])
    b = workloads.rhs_gauss(60, 17)
    ref = orc.lsrn_solve(ocsr(orc, S2), b, seed=2, refine=3)
    x, info = L.solve_csr(gcsr(L, S2), dev(b), seed=9, refine=2)
    assert info["tall"] == 0 and info["rank"] == ref.rank == 58
    assert rel(host(x), ref.x) < 1e-9


def test_solve_csr_edge_cases(L, orc):
    # rows and columns without entries; all-zero A gives x = 0
    S = workloads.sparse_problem(500, 40, per_row=5, n_dense=0, fill=0.0, seed=3)
    d = S.to_dense()
    d[17] = 0.0
    d[:, 6] = 0.0
    keep = np.nonzero(d)
    rowptr = np.zeros(501, np.int64)
    np.add.at(rowptr, keep[0] + 1, 1)
    rowptr = np.cumsum(rowptr)
    S2 = workloads.Sparse(500, 40, rowptr, keep[1].astype(np.int32), d[keep])
    b = workloads.rhs_gauss(500, 3)
    ref = orc.lsrn_solve(ocsr(orc, S2), b, seed=1, refine=3)
    x, info = L.solve_csr(gcsr(L, S2), dev(b), seed=1, refine=2)
    assert info["rank"] == 39
    assert rel(host(x), ref.x) < 1e-10
    Z = L.Csr.from_host(30, 5, np.zeros(31, np.int64), np.zeros(0, np.int32), np.zeros(0))
    x, info = L.solve_csr(Z, dev(np.ones(30)))
    assert info["rank"] == 0 and np.all(host(x) == 0.0)
    # malformed structure is rejected before any kernel reads it
    bad = L.Csr.from_host(3, 4, np.array([0, 1, 2, 3]), np.array([0, 4, 1], np.int32), np.ones(3))
    with pytest.raises(L.LSRNError) as e:
        L.solve_csr(bad, dev(np.ones(3)))
    assert e.value.status == 1
    bad = L.Csr.from_host(3, 4, np.array([0, 2, 1, 3]), np.array([0, 1, 2], np.int32), np.ones(3))
    with pytest.raises(L.LSRNError) as e:
        L.solve_csr(bad, dev(np.ones(3)))
    assert e.value.status == 1
    # Tikhonov on an under-determined A: Sec. 5's form [A, lambda I_m]
    Sf = workloads.sparse_problem(10, 50, per_row=5, n_dense=0, fill=0.0, seed=2)
    Af = Sf.to_dense()
    x, info = L.solve_csr(gcsr(L, Sf), dev(np.ones(10)), lam=0.1, refine=2)
    x_cf = Af.T @ np.linalg.solve(Af @ Af.T + 0.01 * np.eye(10), np.ones(10))
    assert info["tall"] == 0 and rel(host(x), x_cf) < 1e-10


# ------------------------------------------------ full size, 2e6 x 2e4

@pytest.fixture(scope="module")
def sparse_full():
    print("[sparse_full] generating m=2000000 n=20000 lambda=1e-3", flush=True)
    S = workloads.sparse_problem(2_000_000, 20_000, per_row=20, n_dense=10, fill=0.1, seed=13)
    b = workloads.rhs_gauss(S.m, 13)
    return S, b


def _cg_normal_equations(A, At, b, lam, tol=1e-14, maxiter=2000):
    """Reference by CG on (A^T A + lam^2 I) x = A^T b with torch's sparse
    products (independent of the library)."""
    rhs = At @ b
    x = torch.zeros_like(rhs)
    r = rhs.clone()
    p = r.clone()
    rs = torch.dot(r, r)
    stop = (tol * torch.linalg.norm(rhs)) ** 2
    for _ in range(maxiter):
        q = At @ (A @ p) + lam * lam * p
        a = rs / torch.dot(p, q)
        x += a * p
        r -= a * q
        rs_new = torch.dot(r, r)
        if rs_new <= stop:
            break
        p = r + (rs_new / rs) * p
        rs = rs_new
    return x


def test_solve_csr_full_size_tikhonov(L, orc, sparse_full):
    S, b = sparse_full
    lam = 1e-3
    A = gcsr(L, S)
    bd = dev(b)
    print("[sparse_full] solve", flush=True)
    x, info = L.solve_csr(A, bd, lam=lam, tol=1e-12, seed=5, refine=1, profile=1)
    print(f"[sparse_full] info {info}", flush=True)
    # d = 20000 selects the QR-inverse preconditioner (lambda > 0: full rank)
    assert info["tall"] == 1 and info["s"] == 40000 and info["rank"] == 20000
    assert info["converged"] == 1
    # LSQR's count stays below the Chebyshev count of the same bounds
    sl, su = orc.cs_bounds(40000, 20000, 1.0)
    assert info["iters"] <= orc.cs_iterations(sl, su, 1e-12)
    Ad = torch.sparse_csr_tensor(A.rowptr, A.colind.long(), A.val, size=(S.m, S.n))
    At = Ad.t().to_sparse_csr()
    xr = _cg_normal_equations(Ad, At, bd, lam)
    e = (torch.linalg.norm(x - xr) / torch.linalg.norm(xr)).item()
    print(f"[sparse_full] rel err vs CG on the normal equations {e:.3e}", flush=True)
    assert e <= 1e-10
    # normal-equation residual of the augmented problem, relative
    r = bd - Ad @ x
    h = At @ r - lam * lam * x
    fro = torch.linalg.norm(A.val).item()
    ne = (torch.linalg.norm(h) / (fro * torch.linalg.norm(r))).item()
    assert ne <= 1e-12


def test_sketch_csr_full_size_sampled(L, orc, sparse_full):
    """Entries of the 40000 x 20000 sketch recomputed one by one by the oracle."""
    import scipy.sparse as sp
    S, _ = sparse_full
    lam, s, seed = 1e-3, 40000, 11
    X = L.sketch_csr(gcsr(L, S), s, seed=seed, lam=lam)   # (d, s) = X column-major
    Acsc = sp.csr_matrix((S.val, S.colind, S.rowptr), shape=(S.m, S.n)).tocsc()
    dense_col = int(np.argmax(np.diff(Acsc.indptr)))
    eps = np.finfo(float).eps
    for i, c in [(0, 0), (39999, 19999), (12345, dense_col), (777, 4095), (20001, 4096)]:
        rows = Acsc.indices[Acsc.indptr[c]:Acsc.indptr[c + 1]]
        vals = Acsc.data[Acsc.indptr[c]:Acsc.indptr[c + 1]]
        g = np.array([orc.gauss(seed, i, int(k)) for k in rows])
        ref = math.fsum(g * vals) + lam * orc.gauss(seed, i, S.m + c)
        got = X[c, i].item()
        bound = 2 * (S.m + S.n) * eps * (np.abs(g) @ np.abs(vals) + lam) + 1e-300
        assert abs(got - ref) <= bound, (i, c, got, ref)


@pytest.mark.parametrize("method", [0, 1])
def test_tnimg_replica_vs_oracle(L, orc, method):
    """The tnimg stand-in (Sec. 6.5's matrices: 1024 DCT rows, 20 or 21
    nonzeros per column) at 1024 x 30000: the under-determined CSR path
    (Alg. 2 on the transposed structure) against the oracle's reference mode
    with a preconditioner from LAPACK's SVD of a numpy Gaussian sketch (an
    input taken from neither side)."""
    S = workloads.tnimg_like(30000, seed=16)
    T = S.to_dense().T.copy()                          # tall view, 30000 x m
    d = S.m
    s = 2 * d
    rng = np.random.default_rng(3)
    X = np.zeros((s, d))
    for k0 in range(0, T.shape[0], 4096):
        X += rng.standard_normal((s, min(4096, T.shape[0] - k0))) @ T[k0:k0 + 4096]
    _, sv, Vt = np.linalg.svd(np.linalg.qr(X, mode="r"))
    r = int((sv > max(s, d) * 2.0 ** -52 * sv[0]).sum())
    Pn = np.ascontiguousarray(Vt[:r].T / sv[:r])
    b = workloads.rhs_gauss(d, 17)
    ref, _, _, _ = orc.lsrn_iterate(ocsr(orc, S), b, Pn, s, refine=3)
    x, info = L.solve_csr(gcsr(L, S), dev(b), method=method, seed=5, refine=1)
    e = rel(host(x), ref)
    print(f"tnimg replica {S.m}x{S.n} nnz={S.nnz} method={method}: rank={info['rank']} "
          f"iters={info['iters']} rel_err_vs_oracle={e:.2e}")
    assert info["tall"] == 0 and info["rank"] == r
    assert e <= 1e-10
