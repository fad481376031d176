"""Pins of the oracle's precision-form sketch: BF16 rounding against torch's
bfloat16 conversion, and the sketch against a product formed with torch's
rounding (not with the oracle's)."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")


def test_bf16_round_matches_torch(orc):
    rng = np.random.default_rng(0)
    vals = np.concatenate([rng.standard_normal(2000).astype(np.float32),
                           (rng.standard_normal(500) * 1e-30).astype(np.float32),
                           (rng.standard_normal(500) * 1e30).astype(np.float32),
                           np.float32([0.0, -0.0, 1.0, -1.0, 3.0e-38])])
    # exact halfway cases: 1 + 2^-8 (tie, rounds to 1: even) and 1 + 3 * 2^-8
    vals = np.concatenate([vals, np.float32([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8)])])
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([orc.bf16_round(float(v)) for v in vals], dtype=np.float32)
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert orc.bf16_round(1 + 2.0 ** -8) == 1.0
    assert orc.bf16_round(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6


@pytest.mark.parametrize("m,n,lam", [(300, 40, 0.0), (90, 700, 0.0), (200, 30, 0.25)])
def test_sketch_bf16_is_rounded_g_times_fp32_a(orc, m, n, lam):
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)) * np.exp(rng.standard_normal((m, n)))
    s, seed = 37, 5
    M = orc.Matrix.dense(A, lam=lam)
    X = orc.sketch_bf16(M, s, seed)
    T = A if m >= n or lam > 0 else A.T
    K = T.shape[0]
    G = orc.gauss_fill(seed, 0, s, 0, K)
    Gb = torch.from_numpy(G).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    T32 = T.astype(np.float32).astype(np.float64)
    ref = Gb @ T32
    if lam > 0:
        ref += lam * orc.gauss_fill(seed, 0, s, K, n)
    bound = 2 * K * np.finfo(float).eps * (np.abs(Gb) @ np.abs(T32) + lam) + 1e-300
    assert np.all(np.abs(X - ref) <= bound)
