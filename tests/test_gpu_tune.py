"""Launch-shape autotuning of the dense sweep: a tuned solve records its
shape, later solves reuse it, an imported table reproduces the tuned
result bit for bit, and every shape gives the same solution to rounding."""
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


def test_autotune_records_and_reproduces(L):
    A, _, _, _ = workloads.dense_problem_device(60000, 300, smin=1e-5, seed=91)
    b = workloads.rhs_gauss_device(60000, 92)
    opts = dict(seed=3, refine=1)
    L.tune_clear()
    x0, i0 = L.solve_dense(A, b, **opts)                  # built-in shape
    assert L.tune_export() == ""
    x1, i1 = L.solve_dense(A, b, autotune=1, **opts)      # tunes, records, uses
    text = L.tune_export()
    lines = text.strip().splitlines()
    assert len(lines) == 1 and lines[0].startswith("sweep f64 16 300 ")
    per_cu = int(lines[0].split()[-1])
    assert 1 <= per_cu <= 4
    x2, _ = L.solve_dense(A, b, **opts)                   # reuses the record
    assert np.array_equal(host(x1), host(x2))
    L.tune_clear()
    L.tune_import(text)
    x3, _ = L.solve_dense(A, b, **opts)                   # imported table
    assert np.array_equal(host(x1), host(x3))
    # shapes only reorder the partial sums
    e = np.linalg.norm(host(x1) - host(x0)) / np.linalg.norm(host(x0))
    assert e < 1e-11 and abs(i1["iters"] - i0["iters"]) <= 1
    for c in (1, 4):
        L.tune_clear()
        L.tune_import(f"sweep f64 16 300 {c}")
        xc, _ = L.solve_dense(A, b, **opts)
        assert np.linalg.norm(host(xc) - host(x0)) / np.linalg.norm(host(x0)) < 1e-11
    L.tune_clear()
