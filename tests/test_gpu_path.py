"""Parity of the HIP path (through the C ABI) with the CPU oracle, step by
step and end to end, on seeded synthetic inputs."""
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


# ---------------------------------------------------------------- step 2: G

def test_philox_words_bit_exact(L, orc):
    cases = [(0, 0, 5, 0, 7), (5, 7, 3, 9, 4), (2**63 + 11, 2**33 + 1, 4, 2**35 + 3, 3),
             (0xFFFFFFFFFFFFFFFF, 0xFFFFFFF0, 17, 0xFFFFFFF0, 17)]
    for seed, row0, nrows, q0, nq in cases:
        got = host(L.philox_words(seed, row0, nrows, q0, nq)).view(np.uint32)
        for r in range(nrows):
            for j in range(nq):
                np.testing.assert_array_equal(got[r, j], orc.philox_block(seed, row0 + r, q0 + j))


def test_gauss_fill_matches_oracle(L, orc):
    for seed, row0, nrows, col0, ncols in [(3, 0, 64, 0, 301), (9, 1000, 7, 123457, 66)]:
        g = host(L.gauss_fill(seed, row0, nrows, col0, ncols))
        ref = orc.gauss_fill(seed, row0, nrows, col0, ncols)
        # device sincospi / log vs libm: a few ulps
        assert np.abs(g - ref).max() <= 1e-14 * (1 + np.abs(ref).max())


# ---------------------------------------------------------------- step 3: sketch

def _sketch_bound(orc, M, s, seed):
    """Entrywise bound |X_gpu - X_orc| <= 2 K u (|G| |T|) + normal-transform difference."""
    T = M.to_dense()
    if orc.is_tall(M):
        T = np.vstack([T, M.lam * np.eye(M.n)]) if M.lam > 0 else T
    else:
        T = T.T
    K = T.shape[0]
    G = orc.gauss_fill(seed, 0, s, 0, K)
    return (2 * K * np.finfo(float).eps + 1e-14) * (np.abs(G) @ np.abs(T)) + 1e-300


@pytest.mark.parametrize("m,n,layout,lam,s", [
    (2000, 100, 0, 0.0, 200),      # the dense workload's shape
    (1037, 131, 0, 0.0, 263),      # ragged tiles in every dimension
    (300, 40, 0, 0.5, 81),         # Tikhonov rows
    (100, 2000, 1, 0.0, 200),      # fat, column-major (no copy)
    (77, 900, 0, 0.0, 155),        # fat, row-major (transposed copy)
    (900, 77, 1, 0.0, 155),        # tall, column-major (transposed copy)
    (5, 3, 0, 0.0, 7),             # tiny
])
def test_sketch_matches_oracle(L, orc, m, n, layout, lam, s):
    rng = np.random.default_rng(m * 7 + n)
    A = rng.standard_normal((m, n))
    seed = 1234
    M = orc.Matrix.dense(A, lam=lam)
    Xo = orc.sketch(M, s, seed)
    At = A if layout == 0 else A.T.copy()
    Xg = host(L.sketch_dense(dev(At), s, seed=seed, lam=lam, layout=layout)).T
    assert Xg.shape == Xo.shape
    bound = _sketch_bound(orc, M, s, seed)
    assert np.all(np.abs(Xg - Xo) <= bound)


@pytest.mark.parametrize("K,d,s,pad", [
    (3000, 2048, 4096, 0),    # 64 x 512 tiles (1 x 8 wavefronts), 256 of them
    (3000, 1990, 3990, 0),    # 64 x 512 tiles, ragged in both dimensions
    (3000, 2048, 4096, 1),    # 64 x 512 tiles, odd leading dimension (single loads)
    (3000, 768, 11008, 0),    # 128 x 256 tiles (2 x 4): 512-column tiles would pad
])
def test_sketch_wide_tiles_sampled(L, orc, K, d, s, pad):
    """Sizes whose tile grid fills the chip take the wide tiles; entries
    recomputed one by one by the oracle's G and exact sums."""
    import math
    seed = 77
    rng = np.random.default_rng(5)
    Tbuf = rng.standard_normal((K, d + pad))
    T = Tbuf[:, :d]
    X = host(L.sketch_dense(dev(Tbuf)[:, :d], s, seed=seed)).T        # s x d
    eps = np.finfo(float).eps
    picks = [(0, 0), (s - 1, d - 1), (63, 511), (64, 512), (127, 255), (128, 256),
             (s - 1, 0), (0, d - 1), (s // 2, d // 2)]
    picks += [(int(i), int(c)) for i, c in zip(rng.integers(0, s, 60), rng.integers(0, d, 60))]
    for i, c in picks:
        g = orc.gauss_fill(seed, i, 1, 0, K)[0]
        ref = math.fsum(g * T[:, c])
        bound = 2 * K * eps * (np.abs(g) @ np.abs(T[:, c])) + 1e-14
        assert abs(X[i, c] - ref) <= bound, (i, c, X[i, c], ref)


# ---------------------------------------------------------------- steps 4-5

@pytest.mark.parametrize("s,d,rank", [(200, 100, 100), (263, 131, 131), (500, 240, 200),
                                      (900, 420, 420), (30, 12, 5)])
def test_precond_matches_oracle(L, orc, s, d, rank):
    P = workloads.dense_problem(4 * s, d, rank=rank, smin=1e-6, seed=s + d)
    X = orc.sketch(orc.Matrix.dense(P.A), s, 5)
    r_o, sig_o, N_o, _ = orc.precond(X)
    r_g, sig_g, N_g, sweeps = L.precond(dev(X.T.copy()))
    sig_g, N_g = host(sig_g), host(N_g)
    assert r_g == r_o == rank
    assert 0 < sweeps < 40
    # QR + Jacobi are backward stable with ||dX|| ~ d eps ||X||; by Weyl the
    # singular values then move by at most that much
    eps = np.finfo(float).eps
    np.testing.assert_allclose(sig_g[:rank], sig_o[:rank], rtol=0, atol=4 * d * eps * sig_o[0])
    # X N is orthonormal to what the preconditioner needs: ||C - I||_2 <= 1e-6
    # moves every singular value of A N (Lemma 2, Theorem 3) by at most that
    # relative amount.  With N = W Sigma^-2 the rotations' normwise backward
    # error leaves ~5e-8 at kappa = 1e6 (the oracle's own N measures the same).
    Xl = X.astype(np.longdouble)
    Q = Xl @ N_g.astype(np.longdouble)
    C = (Q.T @ Q).astype(float)
    assert np.linalg.norm(C - np.eye(rank), 2) <= 1e-6
    # same range as the oracle's N (N itself is unique only up to signs)
    Qo, _ = np.linalg.qr(N_o)
    assert np.linalg.norm(N_g - Qo @ (Qo.T @ N_g)) / np.linalg.norm(N_g) < 1e-9


@pytest.mark.parametrize("d,rank", [(600, 560), (1100, 1100)])
def test_precond_wide_variants_against_lapack(L, d, rank):
    """Widths that select the other Jacobi round kernels; the sketch comes
    from the GPU and LAPACK's SVD of the same X is the reference."""
    s = 2 * d
    P = workloads.dense_problem(3 * s, d, rank=rank, smin=1e-6, seed=d)
    Xcm = L.sketch_dense(dev(P.A), s, seed=9)
    X = host(Xcm).T
    r, sig, N, sweeps = L.precond(Xcm)
    sig, N = host(sig), host(N)
    ref = np.linalg.svd(X, compute_uv=False)
    assert r == rank
    eps = np.finfo(float).eps
    np.testing.assert_allclose(sig[:rank], ref[:rank], rtol=0, atol=4 * d * eps * ref[0])
    Q = X.astype(np.longdouble) @ N.astype(np.longdouble)
    C = (Q.T @ Q).astype(float)
    assert np.linalg.norm(C - np.eye(rank), 2) <= 1e-6


@pytest.mark.parametrize("d,rank", [(2500, 2400), (4500, 4500)])
def test_precond_large_variants_against_lapack(L, d, rank):
    """The two widest Jacobi round kernels (4 and 2 columns per block);
    LAPACK's singular values of the same sketch are the reference.  With
    kappa = 1e3 the FP64 product X N is accurate to ~d eps kappa, far below
    the 1e-6 bound, so no extended precision is needed."""
    s = 2 * d
    A, _, _, _ = workloads.dense_problem_device(3 * s, d, rank=rank, smin=1e-3, seed=d)
    Xcm = L.sketch_dense(A, s, seed=3)
    del A
    X = host(Xcm).T
    r, sig, N, sweeps = L.precond(Xcm)
    sig, N = host(sig), host(N)
    ref = np.linalg.svd(X, compute_uv=False)
    assert r == rank and 0 < sweeps < 40
    eps = np.finfo(float).eps
    np.testing.assert_allclose(sig[:rank], ref[:rank], rtol=0, atol=4 * d * eps * ref[0])
    Q = X @ N
    assert np.linalg.norm(Q.T @ Q - np.eye(rank), 2) <= 1e-6
    # N = V Sigma^-1: the rescaled columns are orthonormal up to the stopping
    # rule, which leaves every off-diagonal cosine below d eps, so the d x d
    # deviation has norm at most d * d eps
    V = N * sig[:rank]
    assert np.linalg.norm(V.T @ V - np.eye(rank), 2) <= d * d * eps


# ---------------------------------------------------------------- steps 6-7

@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("shape", ["tall", "fat", "tikhonov"])
def test_iterations_match_oracle_with_same_preconditioner(L, orc, method, shape):
    """Given the oracle's N (or M), the GPU LSQR / Chebyshev iterates agree
    with the oracle's to rounding, and the iteration counts agree."""
    if shape == "fat":
        Pd = workloads.dense_problem(1500, 60, smin=1e-4, seed=21)
        A = Pd.A.T.copy()                        # 60 x 1500
        M = orc.Matrix.dense(A)
        At, layout, lam = Pd.A, 1, 0.0           # column-major storage
    else:
        lam = 1e-2 if shape == "tikhonov" else 0.0
        Pd = workloads.dense_problem(1500, 60, smin=1e-4, seed=22)
        A = Pd.A
        M = orc.Matrix.dense(A, lam=lam)
        At, layout = A, 0
    b = workloads.rhs_gauss(A.shape[0], 23)
    res = orc.lsrn_solve(M, b, seed=3, method=method)
    Pm = res.P
    xg, info = L.iterate_dense(dev(At), dev(b), dev(Pm), res.s, layout=layout, method=method,
                               lam=lam)
    xg = host(xg)
    assert rel(xg, res.x) < 1e-11
    if method == 1:
        assert info["iters"] == res.iters
    else:
        assert abs(info["iters"] - res.iters) <= 1


# ---------------------------------------------------------------- end to end

@pytest.fixture(scope="module")
def dense_workload(orc):
    P = workloads.dense_problem(2000, 100, smin=1e-6, seed=11)
    b, _ = workloads.rhs_model(P.A, 1e-3, 11)
    ref = orc.lsrn_solve(orc.Matrix.dense(P.A), b, seed=1, refine=3)
    return P, b, ref


@pytest.mark.parametrize("method", [0, 1])
def test_solve_dense_workload_refined_1e10(L, orc, dense_workload, method):
    P, b, ref = dense_workload
    x, info = L.solve_dense(dev(P.A), dev(b), seed=99, method=method, refine=2)
    x = host(x)
    assert info["rank"] == 100 and info["s"] == 200 and info["tall"] == 1
    assert rel(x, ref.x) <= 1e-10
    if method == 1:
        assert info["iters"] == 133
    else:
        assert info["iters"] <= 95


def test_solve_dense_unrefined_close(L, dense_workload):
    P, b, ref = dense_workload
    x, info = L.solve_dense(dev(P.A), dev(b), seed=4)
    # unrefined FP64 LSRN sits at the perturbation floor of this problem
    assert rel(host(x), ref.x) < 1e-7


def test_solve_is_bitwise_deterministic(L, dense_workload):
    P, b, _ = dense_workload
    A_d, b_d = dev(P.A), dev(b)
    x1, _ = L.solve_dense(A_d, b_d, seed=8, refine=1)
    x2, _ = L.solve_dense(A_d, b_d, seed=8, refine=1)
    np.testing.assert_array_equal(host(x1), host(x2))


@pytest.mark.parametrize("view", ["odd_lda", "misaligned"])
def test_padded_and_misaligned_views(L, dense_workload, view):
    """Rows with an odd leading dimension, or a base that is not 16-byte
    aligned, are read element by element by the sketch and the sweeps (the
    paired loads need aligned rows).  The solve reaches the oracle's
    solution and equals the contiguous solve bit for bit: the summation
    orders do not depend on how the rows are loaded."""
    P, b, ref = dense_workload
    m, n = P.A.shape
    A_c, b_d = dev(P.A), dev(b)
    if view == "odd_lda":
        big = torch.zeros((m, n + 1), dtype=torch.float64, device="cuda")
        big[:, :n] = A_c
        A_v = big[:, :n]                     # lda = n + 1 = 101
    else:
        big = torch.zeros((m, n + 2), dtype=torch.float64, device="cuda")
        big[:, 1:n + 1] = A_c
        A_v = big[:, 1:n + 1]                # base 8 bytes past a 16-byte boundary
    assert A_v.stride(0) % 2 == 1 or A_v.data_ptr() % 16 == 8
    x_v, info_v = L.solve_dense(A_v, b_d, seed=5, refine=2)
    x_c, info_c = L.solve_dense(A_c, b_d, seed=5, refine=2)
    assert info_v["iters"] == info_c["iters"]
    np.testing.assert_array_equal(host(x_v), host(x_c))
    assert rel(host(x_v), ref.x) <= 1e-10


@pytest.mark.parametrize("method", [0, 1])
def test_solve_fat_rank_deficient(L, orc, method):
    Pd = workloads.dense_problem(2500, 60, rank=50, smin=1e-6, seed=13)
    A = Pd.A.T.copy()                             # 60 x 2500, rank 50
    b = workloads.rhs_gauss(60, 13)
    ref = orc.lsrn_solve(orc.Matrix.dense_colmajor(Pd.A), b, seed=6, method=method, refine=3)
    x, info = L.solve_dense(dev(Pd.A), dev(b), layout=1, seed=2, method=method, refine=2)
    x = host(x)
    assert info["tall"] == 0 and info["rank"] == 50
    # the row space of a numerically rank-deficient stored matrix is itself
    # defined only to about eps * sigma_1 / sigma_r = 1e-10
    assert rel(x, ref.x) < 1e-9


def test_solve_tikhonov(L, orc):
    Pd = workloads.dense_problem(3000, 80, smin=1e-6, seed=31)
    b = workloads.rhs_gauss(3000, 31)
    lam = 1e-3
    ref = orc.lsrn_solve(orc.Matrix.dense(Pd.A, lam=lam), b, seed=2, refine=3)
    x, info = L.solve_dense(dev(Pd.A), dev(b), lam=lam, seed=5, refine=2)
    assert rel(host(x), ref.x) <= 1e-10


def test_solve_exactly_rank_deficient_vs_pinv(L, orc):
    rng = np.random.default_rng(3)
    B = rng.standard_normal((400, 12)) @ np.diag(10.0 ** np.linspace(0, -3, 12))
    A = np.column_stack([B, B[:, :4] * 0.5, B[:, 4:8] * 0.25])      # rank 12 of 20
    b = rng.standard_normal(400)
    xp, r = orc.pinv_solve(orc.Matrix.dense(A), b)
    x, info = L.solve_dense(dev(A), dev(b), seed=3, refine=2)
    assert info["rank"] == r == 12
    assert rel(host(x), xp) < 1e-11


def test_edge_cases(L, orc):
    # b = 0 -> x = 0
    A = np.random.default_rng(0).standard_normal((50, 5))
    x, info = L.solve_dense(dev(A), dev(np.zeros(50)))
    assert not host(x).any()
    # n = 1
    a = np.random.default_rng(1).standard_normal((40, 1))
    b = np.random.default_rng(2).standard_normal(40)
    x, _ = L.solve_dense(dev(a), dev(b), refine=1)
    np.testing.assert_allclose(host(x), np.linalg.lstsq(a, b, rcond=None)[0], rtol=1e-13)
    # square-ish: m = n + 1 (s = 2n >= m)
    A = np.random.default_rng(4).standard_normal((9, 8))
    b = np.random.default_rng(5).standard_normal(9)
    x, _ = L.solve_dense(dev(A), dev(b), refine=2)
    np.testing.assert_allclose(host(x), np.linalg.lstsq(A, b, rcond=None)[0], rtol=1e-10)
    # invalid arguments are rejected, not run
    with pytest.raises(L.LSRNError) as e:
        L.solve_dense(dev(A), dev(b), gamma=1.0)
    assert e.value.status == 1
    # Tikhonov on an under-determined A (8 x 9): Sec. 5's form [A, lambda I_m]
    Af = A.T.copy()
    x, info = L.solve_dense(dev(Af), dev(np.ones(8)), lam=0.1, refine=2)
    x_cf = Af.T @ np.linalg.solve(Af @ Af.T + 0.01 * np.eye(8), np.ones(8))
    assert info["tall"] == 0
    np.testing.assert_allclose(host(x), x_cf, rtol=1e-10, atol=1e-12)
    with pytest.raises(L.LSRNError) as e:
        L.solve_dense(dev(A), dev(b), t_margin=float("nan"))
    assert e.value.status == 1


@pytest.mark.parametrize("method", [0, 1])
def test_graph_replays_match_eager_launches(L, dense_workload, method):
    """The iteration chunks replayed as HIP graphs (profile off) give the
    same bits as the eager launches (profile on), on the null stream and on
    a stream of the caller's, over repeated solves with eager work between."""
    P, b, _ = dense_workload
    A_d, b_d = dev(P.A), dev(b)
    ref, _ = L.solve_dense(A_d, b_d, seed=8, refine=2, method=method, profile=1)
    ref = host(ref)
    s = torch.cuda.Stream()
    for rep in range(3):
        x0, _ = L.solve_dense(A_d, b_d, seed=8, refine=2, method=method)
        np.testing.assert_array_equal(host(x0), ref)
        with torch.cuda.stream(s):
            x1, _ = L.solve_dense(A_d, b_d, seed=8, refine=2, method=method)
        s.synchronize()
        np.testing.assert_array_equal(host(x1), ref)
        _ = A_d.sum().item()  # eager work between replays


@pytest.mark.parametrize("fat", [False, True])
def test_chebyshev_check_restarts_lsqr(L, orc, fat):
    """A Chebyshev run outside its bounds (margin t = -4 squeezes [sigma_L,
    sigma_U] inside the spectrum of A N) fails the check after the run and
    LSQR continues, on the GPU as in the oracle; the answer is the
    oracle's.  With the default margin no run falls back."""
    Pd = workloads.dense_problem(1200, 60, smin=1e-3, seed=41)
    if fat:
        M = orc.Matrix.dense_colmajor(Pd.A)
        b = workloads.rhs_gauss(60, 41)
        At, layout = Pd.A, 1
    else:
        M = orc.Matrix.dense(Pd.A)
        b = workloads.rhs_gauss(1200, 41)
        At, layout = Pd.A, 0
    ref = orc.lsrn_solve(M, b, seed=2, refine=3)
    A_d, b_d = dev(At), dev(b)
    x0, i0 = L.solve_dense(A_d, b_d, layout=layout, method=1, seed=3)
    assert i0["cs_fallbacks"] == 0 and i0["converged"] == 1
    x1, i1 = L.solve_dense(A_d, b_d, layout=layout, method=1, seed=3, t_margin=-4.0)
    orc_bad = orc.lsrn_solve(M, b, seed=3, method=orc.CS, t_margin=-4.0)
    assert i1["cs_fallbacks"] == 1 == orc_bad.cs_fallbacks
    assert i1["converged"] == 1
    assert rel(host(x1), ref.x) <= 1e-10
    assert rel(host(x0), ref.x) <= 1e-10
