"""The certified N = R^-1 preconditioner (full-rank sketch, no Jacobi
sweeps) at orders where the triangular inverse's halving tree needs a
larger product buffer below its top split (129 .. 159: 128 + r splits into
64 + 64), and around them; solutions against the oracle's."""
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


@pytest.mark.parametrize("d", [64, 65, 128, 129, 130, 143, 159, 160, 191, 257])
def test_certified_inverse_solve_vs_oracle(L, orc, d):
    m = 12 * d
    P = workloads.dense_problem(m, d, smin=1e-3, seed=300 + d)
    b = workloads.rhs_gauss(m, 300 + d)
    ref = orc.lsrn_solve(orc.Matrix.dense(P.A), b, seed=1, refine=3).x
    x, info = L.solve_dense(dev(P.A), dev(b), seed=9, refine=2)
    assert info["precond_used"] == L.PRECOND["qr"] and info["sweeps"] == 0 and info["rank"] == d
    e = np.linalg.norm(host(x) - ref) / np.linalg.norm(ref)
    assert e <= 1e-10, e
