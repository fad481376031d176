"""Plans (lsrn_plan_*): one sketch and preconditioner, many right-hand
sides; each solve returns what a whole solve returns for the same A, b and
options (Thm. 2: N does not depend on b)."""
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


@pytest.mark.parametrize("shape,method,precision", [
    ("tall", "lsqr", "fp64"), ("tall", "chebyshev", "fp64"), ("fat", "lsqr", "fp64"),
    ("tikhonov", "lsqr", "fp64"), ("tall", "lsqr", "mixed")])
def test_plan_solves_equal_whole_solves(L, orc, shape, method, precision):
    P = workloads.dense_problem(3000, 120, rank=110 if shape == "fat" else 120, smin=1e-5, seed=71)
    layout = 1 if shape == "fat" else 0       # fat: the array read as A^T (120 x 3000)
    lam = 1e-2 if shape == "tikhonov" else 0.0
    A = dev(P.A)
    m = 120 if shape == "fat" else 3000
    opts = dict(seed=9, lam=lam, method=method, precision=precision, refine=1)
    plan = L.Plan.dense(A, layout=layout, **opts)
    assert plan.info["rank"] == (110 if shape == "fat" else 120)
    rng = np.random.default_rng(3)
    for k in range(3):
        b = dev(rng.standard_normal(m))
        x1, i1 = plan.solve(b)
        x2, i2 = L.solve_dense(A, b, layout=layout, **opts)
        # same sketch, preconditioner and kernels: bit for bit
        assert np.array_equal(host(x1), host(x2))
        assert i1["iters"] == i2["iters"] and i1["rank"] == i2["rank"]
    # per-solve settings may change; the sketch settings may not
    x3, i3 = plan.solve(b, tol=1e-8, refine=0)
    assert i3["iters"] <= i2["iters"]
    with pytest.raises(L.LSRNError) as e:
        plan.solve(b, seed=10)
    assert e.value.status == 1
    plan.close()


def test_plan_csr_matches_solve_csr(L):
    S = workloads.sparse_problem(6000, 150, per_row=6, n_dense=3, fill=0.2, seed=72)
    A = L.Csr.from_host(S.m, S.n, S.rowptr, S.colind, S.val)
    opts = dict(seed=4, lam=1e-3, refine=1)
    plan = L.Plan.csr(A, **opts)
    rng = np.random.default_rng(8)
    for k in range(2):
        b = dev(rng.standard_normal(S.m))
        x1, _ = plan.solve(b)
        x2, _ = L.solve_csr(A, b, **opts)
        assert np.array_equal(host(x1), host(x2))
    plan.close()


def test_plan_reaches_oracle_solution(L, orc):
    P = workloads.dense_problem(2500, 90, smin=1e-6, seed=73)
    plan = L.Plan.dense(dev(P.A), seed=2, refine=1)
    for k in range(2):
        b = workloads.rhs_gauss(2500, 730 + k)
        ref = orc.lsrn_solve(orc.Matrix.dense(P.A), b, seed=1, refine=3)
        x, info = plan.solve(dev(b))
        e = np.linalg.norm(host(x) - ref.x) / np.linalg.norm(ref.x)
        assert info["converged"] == 1 and e <= 1e-10
    plan.close()
