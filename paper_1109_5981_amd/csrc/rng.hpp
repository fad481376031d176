// rng.hpp -- the counter-based Gaussian stream behind the sketch matrix G.
//
// G (Alg. 1/2 step 2) is never stored: entry (i, k) is a pure function of
// (seed, i, k).  Block q = k / 4 of row i is one Philox4x32-10 evaluation
// (Salmon, Moraes, Dror, Shaw, SC'11) with counter (q_lo, q_hi, i_lo, i_hi)
// and key (seed_lo, seed_hi); its four 32-bit words become four normals by
// two Box-Muller transforms (Box & Muller 1958) on u = (w + 1/2) 2^-32,
// which never reaches 0 or 1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lsrn {

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

// Ten rounds of the Philox4x32 bijection: each round takes the 64-bit
// products of words 0 and 2 with the two round multipliers, xors their
// high halves into words 1 and 3 with the round key, and the key advances
// by the two Weyl increments between rounds.
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo_a = kMulA * c0, hi_a = __umulhi(kMulA, c0);
        const uint32_t lo_b = kMulB * c2, hi_b = __umulhi(kMulB, c2);
        const uint32_t n0 = hi_b ^ c1 ^ k0;
        const uint32_t n2 = hi_a ^ c3 ^ k1;
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ Words4 philox_block(uint64_t seed, uint64_t row, uint64_t q) {
    return philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), (uint32_t)row, (uint32_t)(row >> 32),
                         (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Two standard normals from two words; sincospi avoids rounding 2 pi u.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double &g0, double &g1) {
    const double u0 = ((double)a + 0.5) * 0x1p-32;
    const double u1 = ((double)b + 0.5) * 0x1p-32;
    const double rad = sqrt(-2.0 * log(u0));
    double sn, cs;
    sincospi(2.0 * u1, &sn, &cs);
    g0 = rad * cs;
    g1 = rad * sn;
}

// G(row, 4q .. 4q+3).
__device__ __forceinline__ void gauss4(uint64_t seed, uint64_t row, uint64_t q, double g[4]) {
    const Words4 w = philox_block(seed, row, q);
    box_muller(w.w0, w.w1, g[0], g[1]);
    box_muller(w.w2, w.w3, g[2], g[3]);
}

}  // namespace lsrn
