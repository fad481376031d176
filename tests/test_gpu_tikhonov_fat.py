"""The under-determined Tikhonov form of Sec. 5 on the GPU (through the C
ABI): for m < n and lambda > 0, Alg. 2 on [A, lambda I_m], whose min-length
solution's head is the minimiser of ||A x - b||^2 + lambda^2 ||x||^2.
Checked against the oracle's solve of the same form and, on small inputs,
against the closed form A^T (A A^T + lambda^2 I)^-1 b."""
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


def fat_problem(m, n, rank, smin, seed):
    """A (m x n, m < n) = the transpose of a tall generator matrix."""
    P = workloads.dense_problem(n, m, rank=rank, smin=smin, seed=seed)
    return P.A.T.copy()


@pytest.mark.parametrize("layout", [0, 1], ids=["rowmajor_copy", "colmajor_in_place"])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("lam", [1e-3, 0.3])
def test_fat_tikhonov_dense_vs_closed_form_and_oracle(L, orc, layout, method, lam):
    A = fat_problem(60, 1500, 50, 1e-6, seed=90)          # rank-deficient, kappa 1e6
    b = workloads.rhs_gauss(60, 91)
    x_cf = A.T @ np.linalg.solve(A @ A.T + lam * lam * np.eye(60), b)
    ref = orc.lsrn_solve(orc.Matrix.dense(A, lam=lam), b, seed=1, method=method, refine=3)
    stored = A if layout == 0 else A.T.copy()
    x, info = L.solve_dense(dev(stored), dev(b), layout=layout, lam=lam, method=method, seed=4,
                            refine=2)
    x = host(x)
    assert info["tall"] == 0 and info["s"] == 120 and info["rank"] == 60
    assert rel(x, ref.x) <= 1e-10
    assert rel(x, x_cf) <= 1e-9


@pytest.mark.parametrize("method", [0, 1])
def test_fat_tikhonov_wide_rows(L, orc, method):
    """m = 1100 selects the 4-columns-per-thread sweep; its Tikhonov rows run
    the fat row-local updates."""
    A = fat_problem(1100, 4000, 1100, 1e-5, seed=92)
    b = workloads.rhs_gauss(1100, 93)
    lam = 1e-3
    ref = orc.lsrn_solve(orc.Matrix.dense_colmajor(A.T.copy(), lam=lam), b, seed=2,
                         method=method, refine=3)
    x, info = L.solve_dense(dev(A.T.copy()), dev(b), layout=1, lam=lam, method=method, seed=5,
                            refine=2)
    e = rel(host(x), ref.x)
    print(f"fat tikhonov 1100 x 4000 method={method}: iters={info['iters']} rel_err={e:.2e}")
    assert e <= 1e-10


def test_fat_tikhonov_sketch_matches_oracle(L, orc):
    """Step 3 of the form: X = G [A^T; lambda I_m] (the identity rows take G's
    columns n .. n+m-1)."""
    rng = np.random.default_rng(94)
    A = rng.standard_normal((70, 900))
    lam, s, seed = 0.7, 151, 11
    Xo = orc.sketch(orc.Matrix.dense(A, lam=lam), s, seed)
    Xg = host(L.sketch_dense(dev(A.T.copy()), s, seed=seed, lam=lam, layout=1)).T
    T = np.vstack([A.T, lam * np.eye(70)])
    G = orc.gauss_fill(seed, 0, s, 0, T.shape[0])
    bound = (2 * T.shape[0] * np.finfo(float).eps + 1e-14) * (np.abs(G) @ np.abs(T))
    assert Xg.shape == Xo.shape == (s, 70)
    assert np.all(np.abs(Xg - Xo) <= bound + 1e-300)


@pytest.mark.parametrize("method", [0, 1])
def test_fat_tikhonov_csr_vs_oracle(L, orc, method):
    S = workloads.sparse_problem(4000, 300, per_row=6, n_dense=3, fill=0.2, seed=95)
    # the fat matrix is the transpose: 300 x 4000
    D = S.to_dense().T.copy()
    rows, cols = np.nonzero(D)
    rowptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=300))])
    colind = cols.astype(np.int32)
    val = D[rows, cols]
    b = workloads.rhs_gauss(300, 96)
    lam = 1e-2
    ref = orc.lsrn_solve(orc.Matrix.csr(300, 4000, rowptr, colind, val, lam=lam), b, seed=3,
                         method=method, refine=3)
    A = L.Csr.from_host(300, 4000, rowptr, colind, val)
    x, info = L.solve_csr(A, dev(b), lam=lam, method=method, seed=6, refine=2)
    assert info["tall"] == 0 and info["rank"] == 300
    assert rel(host(x), ref.x) <= 1e-10


def test_fat_tikhonov_operator_vs_oracle(L, orc):
    A = fat_problem(80, 2000, 80, 1e-4, seed=97)
    b = workloads.rhs_gauss(80, 98)
    lam = 1e-2
    Ad = dev(A)
    m, n = A.shape

    def apply(trans, k, pin, ldin, pout, ldout, stream):
        X = L.device_view(pin, m if trans else n, k, ldin)
        Y = L.device_view(pout, n if trans else m, k, ldout)
        M = Ad.T if trans else Ad
        with torch.cuda.stream(torch.cuda.ExternalStream(stream) if stream else
                               torch.cuda.default_stream()):
            Y.copy_(M @ X.contiguous())
        return 0

    x, info = L.solve_op(m, n, apply, dev(b), seed=7, lam=lam, tol=1e-14)
    ref = orc.lsrn_solve(orc.Matrix.dense(A, lam=lam), b, seed=1, refine=3)
    assert info["tall"] == 0
    assert rel(host(x), ref.x) <= 1e-10
