"""The precision form (BF16 sketch, FP32-stored sweeps, FP64 refinement) on
the GPU through the C ABI, against the CPU oracle."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24  # FP32 unit roundoff


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


@pytest.mark.parametrize("m,n,layout,lam,s", [
    (2000, 100, 0, 0.0, 200),       # 63 stages of 32 k: several FP64 flushes
    (9001, 131, 0, 0.5, 263),       # ragged tiles and stages, Tikhonov rows
    (100, 3000, 1, 0.0, 200),       # fat, column-major
    (5, 3, 0, 0.0, 7),              # tiny
])
def test_sketch_bf16_matches_oracle(L, orc, m, n, layout, lam, s):
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)) * np.exp(rng.standard_normal((m, n)))
    seed = 31
    M = orc.Matrix.dense(A, lam=lam)
    Xo = orc.sketch_bf16(M, s, seed)
    At = A if layout == 0 else A.T.copy()
    Xg = host(L.sketch_dense_bf16(dev(At), s, seed=seed, lam=lam, layout=layout)).T
    # the three BF16 terms reproduce fl32(A) exactly and their products with
    # bf16(G) are exact in FP32; the error is the FP32 accumulation inside one
    # flush window (8 stages x 32 k x 3 terms) plus FP64 sums
    T = A if (m >= n or lam > 0) else A.T
    K = T.shape[0]
    G = orc.gauss_fill(seed, 0, s, 0, K)
    Gb = np.array([[orc.bf16_round(float(v)) for v in row] for row in G.astype(np.float32)])
    mag = np.abs(Gb) @ np.abs(T.astype(np.float32).astype(np.float64))
    bound = (3 * 256 + 16) * U32 * mag + 2 * K * np.finfo(float).eps * (mag + lam) + 1e-300
    assert np.all(np.abs(Xg - Xo) <= bound)


@pytest.mark.parametrize("m,n,layout,lam,s", [
    (2000, 100, 0, 0.0, 200),
    (9001, 131, 0, 0.5, 263),
    (100, 3000, 1, 0.0, 200),
])
def test_sketch_bf16_operand_paths_agree(L, orc, monkeypatch, m, n, layout, lam, s):
    """The three ways the kernel takes its operands -- bf16(G) and the split
    terms of T pre-formed in device memory, only bf16(G) pre-formed, both
    formed per stage -- give the same bits (same values, same order of
    products and sums), and match the oracle.  LSRN_PREGEN_MAX_BYTES caps
    the pre-formed operands: 8e6 bytes holds bf16(G) of these shapes
    (at most 64 s ceil(K / 32) bytes) but not the split terms (at least
    3 x 64 x 128 ceil(K / 32) bytes)."""
    rng = np.random.default_rng(7 * m + n)
    A = rng.standard_normal((m, n)) * np.exp(rng.standard_normal((m, n)))
    seed = 17
    At = dev(A if layout == 0 else A.T.copy())
    out = {}
    for name, cap in (("both", None), ("g_only", "8000000"), ("none", "0")):
        if cap is None:
            monkeypatch.delenv("LSRN_PREGEN_MAX_BYTES", raising=False)
        else:
            monkeypatch.setenv("LSRN_PREGEN_MAX_BYTES", cap)
        out[name] = host(L.sketch_dense_bf16(At, s, seed=seed, lam=lam, layout=layout))
    monkeypatch.delenv("LSRN_PREGEN_MAX_BYTES", raising=False)
    np.testing.assert_array_equal(out["g_only"], out["both"])
    np.testing.assert_array_equal(out["none"], out["both"])
    Xo = orc.sketch_bf16(orc.Matrix.dense(A, lam=lam), s, seed)
    e = np.abs(out["both"].T - Xo).max() / np.abs(Xo).max()
    assert e <= 1e-5, e


@pytest.fixture(scope="module")
def kappa6(orc):
    P = workloads.dense_problem(20000, 200, smin=1e-6, seed=61)
    b, _ = workloads.rhs_model(P.A, 1e-6, 61)
    ref = orc.lsrn_solve(orc.Matrix.dense(P.A), b, seed=1, refine=3)
    return P, b, ref


def test_mixed_solve_reaches_fp64_accuracy_at_kappa_1e6(L, kappa6):
    P, b, ref = kappa6
    x, info = L.solve_dense(dev(P.A), dev(b), seed=5, precision="mixed", refine=20)
    e = rel(host(x), ref.x)
    print(f"[mixed kappa=1e6] rel err {e:.2e} iters {info['iters']} refine_steps "
          f"{info['refine_steps']} refine_iters {info['refine_iters']}")
    assert info["rank"] == 200 and info["converged"] == 1
    assert e <= 1e-10


def test_mixed_solve_at_kappa_1e8_falls_back_to_fp64_sweeps(L, orc):
    """At kappa = 1e8, kappa u32 > 1: the FP32 sweeps cannot carry the
    refinement to FP64 accuracy.  Once their corrections stop shrinking the
    refinement continues with sweeps over the FP64 A and reaches the FP64
    path's accuracy; the info reports those steps."""
    P = workloads.dense_problem(20000, 200, smin=1e-8, seed=63)
    b, _ = workloads.rhs_model(P.A, 1e-6, 63)
    ref = orc.lsrn_solve(orc.Matrix.dense(P.A), b, seed=1, refine=6)
    A, bd = dev(P.A), dev(b)
    x64, i64 = L.solve_dense(A, bd, seed=5, refine=6)
    e64 = rel(host(x64), ref.x)
    print(f"[fp64 kappa=1e8] rel err {e64:.2e} refine_steps {i64['refine_steps']}")
    assert e64 <= 1e-10 and i64["fp64_refine_steps"] == 0
    xm, info = L.solve_dense(A, bd, seed=5, precision="mixed", refine=20)
    e = rel(host(xm), ref.x)
    print(f"[mixed kappa=1e8] rel err {e:.2e} refine_steps {info['refine_steps']} "
          f"fp64 steps {info['fp64_refine_steps']}")
    assert info["converged"] == 1 and info["fp64_refine_steps"] >= 1
    assert e <= 1e-10


def test_mixed_rejections(L):
    P = workloads.dense_problem(500, 20, smin=1e-3, seed=64)
    b = workloads.rhs_gauss(500, 64)
    with pytest.raises(L.LSRNError) as e:
        L.solve_dense(dev(P.A), dev(b), precision="mixed", method="chebyshev")
    assert e.value.status == 5
    # under-determined A (stored column-major as its transpose)
    with pytest.raises(L.LSRNError) as e:
        L.solve_dense(dev(P.A), dev(b[:20]), layout=1, precision="mixed")
    assert e.value.status == 5
    S = workloads.sparse_problem(500, 20, per_row=4, n_dense=0, fill=0.0, seed=64)
    with pytest.raises(L.LSRNError) as e:
        L.solve_csr(L.Csr.from_host(S.m, S.n, S.rowptr, S.colind, S.val), dev(b),
                    precision="mixed")
    assert e.value.status == 5
