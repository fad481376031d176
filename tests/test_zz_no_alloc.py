"""lsrn_sketch_dense_noalloc (through the C ABI) against lsrn_sketch_dense:
the same bits on two calls in a row (the second smaller, so it reuses the
scratch the first left behind), within Higham's bound of the oracle, and
clear errors for shapes it does not take."""
import numpy as np
import pytest

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


def oracle_bound_ok(orc, A, lam, s, seed, X, fat=False):
    M = orc.Matrix.dense_colmajor(A) if fat else orc.Matrix.dense(A, lam=lam)
    Xo = orc.sketch(M, s, seed)
    T = A if fat else (np.vstack([A, lam * np.eye(A.shape[1])]) if lam > 0 else A)
    G = orc.gauss_fill(seed, 0, s, 0, T.shape[0])
    bound = (2 * T.shape[0] * np.finfo(float).eps + 1e-14) * (np.abs(G) @ np.abs(T))
    return np.all(np.abs(X - Xo) <= bound + 1e-300)


@pytest.mark.parametrize("lam", [0.0, 0.25])
def test_noalloc_sketch_equals_allocating_sketch(L, orc, lam):
    rng = np.random.default_rng(71)
    # two calls in a row on one stream: a split-K grid (partial sums in the
    # scratch), then a smaller one that reuses what the first left there
    for m, n, s, seed in [(3000, 300, 600, 5), (1000, 100, 200, 6)]:
        A = rng.standard_normal((m, n))
        A_d = dev(A)
        Xn = L.sketch_dense_noalloc(A_d, s, seed=seed, lam=lam)
        Xa = L.sketch_dense(A_d, s, seed=seed, lam=lam)
        np.testing.assert_array_equal(host(Xn), host(Xa))
        assert oracle_bound_ok(orc, A, lam, s, seed, host(Xn).T)


def test_noalloc_sketch_fat_and_repeated(L, orc):
    rng = np.random.default_rng(72)
    A = rng.standard_normal((120, 1500))          # fat: stored column-major as A^T
    At_d = dev(A.T.copy())
    X1 = host(L.sketch_dense_noalloc(At_d, 240, seed=9, layout=L.COL_MAJOR))
    X2 = host(L.sketch_dense_noalloc(At_d, 240, seed=9, layout=L.COL_MAJOR))
    Xa = host(L.sketch_dense(At_d, 240, seed=9, layout=L.COL_MAJOR))
    np.testing.assert_array_equal(X1, Xa)
    np.testing.assert_array_equal(X2, Xa)
    assert oracle_bound_ok(orc, A.T.copy(), 0.0, 240, 9, X1.T, fat=True)


def test_noalloc_sketch_rejects_what_it_does_not_take(L):
    A_d = dev(np.random.default_rng(73).standard_normal((400, 30)))
    # column-major storage of a tall matrix would need a transposed copy
    with pytest.raises(L.LSRNError) as e:
        L.sketch_dense_noalloc(A_d.T.contiguous(), 60, layout=L.COL_MAJOR)
    assert e.value.status == 5
    # a sketch whose split-K partial sums exceed the static scratch: s = 2200,
    # d = 1100 takes 162 tiles of 128 x 128 and 4 slices of K, 77 MB of
    # partial sums against 64 MiB
    big = torch.zeros((4096, 1100), dtype=torch.float64, device="cuda")
    with pytest.raises(L.LSRNError) as e:
        L.sketch_dense_noalloc(big, 2200, seed=1)
    assert e.value.status == 2
    assert "static scratch" in str(e.value)
