"""FP32 storage of A (lsrn_solve_dense_f32): the least-squares problem of
the stored FP32 values is solved to the FP64 bar; the oracle solves the same
values held in FP64."""
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("shape,layout,method", [
    ("tall", 0, "lsqr"), ("tall", 1, "lsqr"), ("tall", 0, "chebyshev"),
    ("fat", 1, "lsqr"), ("fat", 0, "lsqr"), ("tikhonov", 0, "lsqr")])
def test_f32_storage_matches_oracle(L, orc, shape, layout, method):
    P = workloads.dense_problem(2500, 90, smin=1e-5, seed=101)
    A64 = P.A.astype(np.float32).astype(np.float64)   # the stored values
    if shape == "fat":
        A64 = A64.T.copy()                             # 90 x 2500
    m, n = A64.shape
    lam = 1e-2 if shape == "tikhonov" else 0.0
    b = workloads.rhs_gauss(m, 102)
    ref = orc.lsrn_solve(orc.Matrix.dense(A64, lam=lam), b, seed=1, refine=3).x
    stored = A64 if layout == 0 else A64.T             # column-major: the array holds A^T
    A32 = torch.from_numpy(np.ascontiguousarray(stored.astype(np.float32))).cuda()
    x, info = L.solve_dense_f32(A32, torch.from_numpy(b).cuda(), layout=layout, lam=lam,
                                method=method, seed=4, refine=1)
    e = np.linalg.norm(host(x) - ref) / np.linalg.norm(ref)
    print(f"[f32 {shape} layout={layout} {method}] rel err {e:.2e} iters {info['iters']}")
    assert info["converged"] == 1 and e <= 1e-10


def test_f32_storage_equals_fp64_storage_of_same_values(L):
    P = workloads.dense_problem(4000, 150, smin=1e-4, seed=103)
    A32 = torch.from_numpy(P.A.astype(np.float32)).cuda()
    b = torch.from_numpy(workloads.rhs_gauss(4000, 104)).cuda()
    x1, i1 = L.solve_dense_f32(A32, b, seed=7, refine=1)
    x2, i2 = L.solve_dense(A32.double(), b, seed=7, refine=1)
    assert i1["rank"] == i2["rank"] == 150
    assert np.linalg.norm(host(x1) - host(x2)) / np.linalg.norm(host(x2)) < 1e-11


def test_f32_odd_leading_dimension_equals_contiguous(L):
    """FP32 rows with an odd leading dimension take the element-by-element
    loads; the solve equals the contiguous one bit for bit."""
    P = workloads.dense_problem(3000, 70, smin=1e-4, seed=107)
    A32 = torch.from_numpy(P.A.astype(np.float32)).cuda()
    m, n = A32.shape
    big = torch.zeros((m, n + 1), dtype=torch.float32, device="cuda")
    big[:, :n] = A32
    A_v = big[:, :n]
    b = torch.from_numpy(workloads.rhs_gauss(m, 108)).cuda()
    x_v, _ = L.solve_dense_f32(A_v, b, seed=3, refine=1)
    x_c, _ = L.solve_dense_f32(A32, b, seed=3, refine=1)
    np.testing.assert_array_equal(host(x_v), host(x_c))


def test_f32_rejections(L):
    A32 = torch.ones(100, 5, dtype=torch.float32, device="cuda")
    b = torch.ones(100, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LSRNError) as e:
        L.solve_dense_f32(A32, b, precision="mixed")
    assert e.value.status == 5
