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
        const uint64_t pa = (uint64_t)kMulA * c0, pb = (uint64_t)kMulB * c2;  // 32 x 32 -> 64
        const uint32_t lo_a = (uint32_t)pa, hi_a = (uint32_t)(pa >> 32);
        const uint32_t lo_b = (uint32_t)pb, hi_b = (uint32_t)(pb >> 32);
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

// -2 ln(u) for u = (a + 1/2) 2^-32.  With a + 1/2 = m 2^e, m in
// [sqrt(1/2), sqrt(2)), ln m = 2 atanh(f), f = (m - 1)/(m + 1), |f| <= 0.1716,
// summed as the Taylor series of atanh through f^21 (the next term is below
// 1e-18 |f|); ln 2 enters split so that (e - 32) ln2_hi is exact.  A few ulp.
__device__ __forceinline__ double neg2_log_u(uint32_t a) {
    constexpr double kLn2Hi = 0x1.62e42fefa2000p-1, kLn2Lo = 0x1.9ef35793c7673p-41;
    const double x = (double)a + 0.5;  // exact
    int e;
    double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
    const bool low = m < 0x1.6a09e667f3bcdp-1;
    m = low ? 2.0 * m : m;
    e = low ? e - 1 : e;
    const double num = m - 1.0;  // exact
    const double den = m + 1.0;
    double y = __builtin_amdgcn_rcp(den);
    y = y * fma(-den, y, 2.0);
    y = y * fma(-den, y, 2.0);
    double f = num * y;
    f = fma(y, fma(-f, den, num), f);  // one correction from the exact residual
    const double z = f * f;
    double p = 0x1.8618618618618p-5;  // 1/21
    p = fma(p, z, 0x1.af286bca1af28p-5);  // 1/19
    p = fma(p, z, 0x1.e1e1e1e1e1e1ep-5);  // 1/17
    p = fma(p, z, 0x1.1111111111111p-4);  // 1/15
    p = fma(p, z, 0x1.3b13b13b13b14p-4);  // 1/13
    p = fma(p, z, 0x1.745d1745d1746p-4);  // 1/11
    p = fma(p, z, 0x1.c71c71c71c71cp-4);  // 1/9
    p = fma(p, z, 0x1.2492492492492p-3);  // 1/7
    p = fma(p, z, 0x1.999999999999ap-3);  // 1/5
    p = fma(p, z, 0x1.5555555555555p-2);  // 1/3
    const double s = fma(f * z, p, f);      // atanh f
    const double k = (double)(e - 32);
    const double lnu = fma(k, kLn2Hi, fma(k, kLn2Lo, 2.0 * s));
    return -2.0 * lnu;
}

// sin and cos of 2 pi (b + 1/2) 2^-32.  The octant is the top three bits of
// b; the rest gives r = (c + 1/2) 2^-32 in (0, 1/8) exactly (reflected to
// 1/8 - r, also exact, in odd octants), t = 2 pi r in (0, pi/4), and the
// Taylor series of sin t through t^17 and of cos t through t^16 (next
// terms below 1e-19 and 3e-18); the octant's symmetry then swaps and
// negates.
__device__ __forceinline__ void sincos_2pi_u(uint32_t b, double &sn, double &cs) {
    constexpr double kTwoPiHi = 0x1.921fb54442d18p+2, kTwoPiLo = 0x1.1a62633145c07p-52;
    const uint32_t oct = b >> 29;
    uint32_t c = b & 0x1fffffffu;
    c = (oct & 1u) ? 0x1fffffffu - c : c;
    const double r = ((double)c + 0.5) * 0x1p-32;
    const double t = fma(r, kTwoPiHi, r * kTwoPiLo);
    const double z = t * t;
    double ps = 0x1.952c77030ad4ap-49;        // 1/17!
    ps = fma(ps, z, -0x1.ae7f3e733b81fp-41);   // -1/15!
    ps = fma(ps, z, 0x1.6124613a86d09p-33);    // 1/13!
    ps = fma(ps, z, -0x1.ae64567f544e4p-26);   // -1/11!
    ps = fma(ps, z, 0x1.71de3a556c734p-19);    // 1/9!
    ps = fma(ps, z, -0x1.a01a01a01a01ap-13);   // -1/7!
    ps = fma(ps, z, 0x1.1111111111111p-7);     // 1/5!
    ps = fma(ps, z, -0x1.5555555555555p-3);    // -1/3!
    const double st = fma(t * z, ps, t);
    double pc = 0x1.ae7f3e733b81fp-45;        // 1/16!
    pc = fma(pc, z, -0x1.93974a8c07c9dp-37);   // -1/14!
    pc = fma(pc, z, 0x1.1eed8eff8d898p-29);    // 1/12!
    pc = fma(pc, z, -0x1.27e4fb7789f5cp-22);   // -1/10!
    pc = fma(pc, z, 0x1.a01a01a01a01ap-16);    // 1/8!
    pc = fma(pc, z, -0x1.6c16c16c16c17p-10);   // -1/6!
    pc = fma(pc, z, 0x1.5555555555555p-5);     // 1/4!
    pc = fma(pc, z, -0.5);                     // -1/2!
    const double ct = fma(z, pc, 1.0);
    const bool swap = (((oct + 1u) >> 1) & 1u) != 0;
    const double s0 = swap ? ct : st, c0 = swap ? st : ct;
    sn = oct >= 4u ? -s0 : s0;
    cs = ((oct + 2u) & 7u) >= 4u ? -c0 : c0;
}

// Two standard normals from two words.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double &g0, double &g1) {
    const double rad = sqrt(neg2_log_u(a));
    double sn, cs;
    sincos_2pi_u(b, sn, cs);
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
