"""Pins for the oracle's random normal matrix G (Alg. 1/2, step 2).

The Philox words are checked against an independent implementation: the
header-only philox4x32_10 engine of rocRAND, compiled for the host.  The
normals are checked against closed-form special values of the Box-Muller
map and against N(0,1) by moments and a Kolmogorov-Smirnov test.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

ROCRAND_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int a = 1; a + 2 < argc; a += 3) {
    unsigned long long seed = strtoull(argv[a], 0, 0), row = strtoull(argv[a+1], 0, 0),
                       q = strtoull(argv[a+2], 0, 0);
    /* key = seed; counter = (offset/4, subsequence) = (q, row) */
    rocrand_device::philox4x32_10_engine e(seed, row, 4ull * q);
    uint4 v = e.next4();
    printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
"""


def _hipcc():
    for c in ("hipcc", "/opt/rocm/bin/hipcc"):
        p = shutil.which(c)
        if p:
            return p
    return None


def test_philox_matches_rocrand_engine(orc):
    hipcc = _hipcc()
    if hipcc is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND header / hipcc not available")
    cases = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (5, 7, 9),
             (0xFFFFFFFFFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF), (2**32 + 3, 2**32 + 5, 2**33 + 1),
             (123456789, 199999, 49999), (42, 3999, 12345678901)]
    rng = np.random.default_rng(3)
    for _ in range(40):
        cases.append((int(rng.integers(0, 2**63)), int(rng.integers(0, 2**40)),
                      int(rng.integers(0, 2**40))))
    with tempfile.TemporaryDirectory() as td:
        src, exe = os.path.join(td, "p.cpp"), os.path.join(td, "p")
        with open(src, "w") as f:
            f.write(ROCRAND_PROG)
        subprocess.run([hipcc, "-O1", src, "-o", exe], check=True, capture_output=True)
        args = [str(v) for c in cases for v in c]
        out = subprocess.run([exe] + args, check=True, capture_output=True, text=True).stdout
    ref = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()],
                   dtype=np.uint64)
    got = np.array([orc.philox_block(*c) for c in cases], dtype=np.uint64)
    np.testing.assert_array_equal(got, ref)


def test_philox_counter_and_key_layout(orc):
    """philox_block(seed, row, q) = Philox(ctr=(q_lo,q_hi,row_lo,row_hi), key=(seed_lo,seed_hi))."""
    seed, row, q = 0x0123456789ABCDEF, 0x1122334455, 0x66778899AA
    ctr = [q & 0xFFFFFFFF, q >> 32, row & 0xFFFFFFFF, row >> 32]
    key = [seed & 0xFFFFFFFF, seed >> 32]
    np.testing.assert_array_equal(orc.philox4x32_10(ctr, key), orc.philox_block(seed, row, q))


def test_box_muller_special_values(orc):
    # u1 = 1/4 turn: cos = 0, sin = 1 (up to the half-ulp offset of u)
    half = (1 << 31)
    rad_half = np.sqrt(2.0 * np.log(2.0))           # -2 ln(1/2)
    g0, g1 = orc.box_muller(half, 0)                  # u0 ~ 1/2, u1 ~ 0
    assert abs(g0 - rad_half) < 1e-8 and abs(g1) < 1e-8
    g0, g1 = orc.box_muller(half, 1 << 30)            # u1 ~ 1/4
    assert abs(g0) < 1e-8 and abs(g1 - rad_half) < 1e-8
    g0, g1 = orc.box_muller(half, 1 << 31)            # u1 ~ 1/2
    assert abs(g0 + rad_half) < 1e-8 and abs(g1) < 1e-8
    # smallest u0 = 2^-33 gives the largest radius sqrt(66 ln 2)
    g0, _ = orc.box_muller(0, 0)
    assert abs(g0 - np.sqrt(66 * np.log(2.0))) < 1e-8


def test_gauss_is_standard_normal(orc):
    G = orc.gauss_fill(2024, 0, 500, 0, 2000)
    z = G.ravel()
    assert abs(z.mean()) < 5 * 1 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / z.size)
    assert abs(stats.skew(z)) < 0.02
    assert abs(stats.kurtosis(z)) < 0.04
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # no correlation between neighbouring rows / columns / block words
    for a, b in ((G[:-1], G[1:]), (G[:, :-1], G[:, 1:]), (G[:, 0::4], G[:, 1::4]),
                 (G[:, 1::4], G[:, 2::4])):
        c = np.corrcoef(a.ravel(), b.ravel())[0, 1]
        assert abs(c) < 5 / np.sqrt(a.size)


def test_gauss_is_a_pure_function_of_seed_row_col(orc):
    A = orc.gauss_fill(7, 100, 20, 37, 50)
    B = orc.gauss_fill(7, 0, 200, 0, 100)[100:120, 37:87]
    np.testing.assert_array_equal(A, B)
    assert orc.gauss(7, 105, 40) == A[5, 3]
    C = orc.gauss_fill(8, 100, 20, 37, 50)
    assert np.abs(A - C).max() > 1.0
