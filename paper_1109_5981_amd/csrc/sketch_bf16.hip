// sketch_bf16.hip -- the sketch of the precision form on the BF16 matrix
// cores (v_mfma_f32_16x16x32_bf16).
//
// X = bf16(G) fl32(T): G(i, k) is the same Philox/Box-Muller normal as in
// the FP64 sketch, rounded to BF16 (round to nearest even through FP32); each
// entry of T is rounded to FP32 and split exactly into three BF16 terms
// t1 + t2 + t3 (8 + 8 + 8 significant bits), so the three BF16 products
// reproduce the product with the FP32 copy of A.  Products are exact in
// FP32; the matrix core accumulates in FP32 for FLUSH stages (FLUSH * 32
// values of k), then the partial sums are added into FP64 registers.
//
// Workgroup: 512 threads (two wavefronts per SIMD; the FP32 and FP64
// accumulators of a wavefront's 64 x 32 block, 96 registers a lane, leave
// room for the operands in flight), a 128 x 128 tile of X (2 x 4
// wavefronts, each 4 x 2 blocks of 16 x 16), 32 values of k per stage; the
// operands of the next two stages are loaded into registers while the
// current one is multiplied.
#include <cstdlib>

#include "internal.hpp"
#include "rng.hpp"

namespace lsrn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // 16 bytes of operands in flight

constexpr int HBM_ = 128;  // sketch rows per workgroup
constexpr int HBN = 128;   // columns per workgroup
constexpr int HKT = 32;    // k per stage
constexpr int HP = 32;     // LDS row (bf16): the 32 k of a stage, 64 bytes, chunks swizzled (swz)
constexpr int HNT = 512;
constexpr int FLUSH = 8;   // stages accumulated in FP32 before the FP64 flush
constexpr size_t kPreGenMaxBytes = (size_t)32 << 30;  // default cap of the pre-generated operands

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rn(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Position of 16-byte chunk c (k = 8 c .. 8 c + 7) within LDS row r: rows
// are 64 bytes, unpadded, and the chunk index is XORed with a function of
// the row so that neither the 16-byte stores (four lanes a row, or one lane
// a row) nor the MFMA operand reads (sixteen rows, one chunk each) put two
// lanes of one LDS cycle on the same bank, for 128- and 256-byte cycles.
__device__ __forceinline__ int swz(int r, int c) { return c ^ (((r >> 1) ^ (r >> 2)) & 3); }

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

// G for the 128 rows x 32 k of a stage: 128 rows x 8 Philox blocks, two
// per thread; Gs[row] holds the row's 32 k in chunks of 8 placed by swz,
// each block's four values stored as one 8-byte vector.
__device__ __forceinline__ void gen_g(uint16_t (*Gs)[HP], uint64_t seed, int64_t m0, int64_t k0) {
    const int t = threadIdx.x;
    const int row = t & (HBM_ - 1);
    const int qb = t >> 7;  // 0..3
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = qb + 4 * h;  // 0..7
        double g[4];
        gauss4(seed, (uint64_t)(m0 + row), (uint64_t)((k0 >> 2) + q), g);
        uint2 v;
        v.x = (uint32_t)bf16_rn((float)g[0]) | ((uint32_t)bf16_rn((float)g[1]) << 16);
        v.y = (uint32_t)bf16_rn((float)g[2]) | ((uint32_t)bf16_rn((float)g[3]) << 16);
        *reinterpret_cast<uint2 *>(&Gs[row][8 * swz(row, q >> 1) + 4 * (q & 1)]) = v;
    }
}

// The three BF16 terms of fl32(v): t1 = bf16(f), t2 = bf16(f - t1),
// t3 = bf16(f - t1 - t2), each difference exact in FP32.
__device__ __forceinline__ void split3(double v, uint32_t (&t)[3]) {
    const float f = (float)v;
    const uint16_t t1 = bf16_rn(f);
    const float r1 = f - bf16_to_f32(t1);
    const uint16_t t2 = bf16_rn(r1);
    const float r2 = r1 - bf16_to_f32(t2);
    t[0] = t1;
    t[1] = t2;
    t[2] = bf16_rn(r2);
}

// T tile (32 k x 128 columns, FP64 row-major) into registers: thread t
// takes column t & 127 of rows 8 (t >> 7) + j, j = 0..7 (each load of a
// wavefront reads 64 consecutive columns of one row).  Rows at or past K
// (K >= 1) and columns past d load the last row / column; bit j of the
// returned mask is set where the value is T's (store_t zeroes the others).
__device__ __forceinline__ uint32_t load_t(const double *__restrict__ T, int64_t ldt, int64_t k0,
                                           int64_t K, int64_t n0, int64_t d, double (&reg)[8]) {
    const int t = threadIdx.x;
    const int64_t col = n0 + (t & (HBN - 1));
    const int64_t kb = k0 + 8 * (t >> 7);
    const double *__restrict__ Tc = T + min(col, d - 1);
    uint32_t mask = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int64_t k = kb + j;
        reg[j] = Tc[min(k, K - 1) * ldt];
        mask |= (k < K && col < d) ? (1u << j) : 0u;
    }
    return mask;
}

// Split and store: As[term][col] holds column col's 32 k in chunks of 8
// placed by swz; the 8 values of k of a thread go as one 16-byte vector per
// term.  The empty asm ties each loaded value to this
// point, so the compiler cannot convert it (and wait for its load) where the
// load was issued, a stage earlier.
__device__ __forceinline__ void store_t(uint16_t (*As)[HBN][HP], const double (&reg)[8], uint32_t mask) {
    const int t = threadIdx.x;
    const int c = t & (HBN - 1);
    const int kb = 8 * (t >> 7);
    uint32_t w[3][4];
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
        uint32_t lo[3], hi[3];
        double v0 = reg[j], v1 = reg[j + 1];
        asm volatile("" : "+v"(v0), "+v"(v1));
        split3((mask >> j) & 1u ? v0 : 0.0, lo);
        split3((mask >> (j + 1)) & 1u ? v1 : 0.0, hi);
#pragma unroll
        for (int term = 0; term < 3; ++term) w[term][j / 2] = lo[term] | (hi[term] << 16);
    }
#pragma unroll
    for (int term = 0; term < 3; ++term)
        *reinterpret_cast<uint4 *>(&As[term][c][8 * swz(c, kb >> 3)]) =
            make_uint4(w[term][0], w[term][1], w[term][2], w[term][3]);
}

// bf16(G) for the whole sketch, generated once: panel p (k = 32 p ..
// 32 p + 31) holds rows 0 .. s - 1, each as 32 consecutive values of k, so
// the 128 x 32 tile of a stage is one contiguous 8 KB block.  One thread per
// Philox block (row, four values of k); the values are those gen_g forms.
__global__ void __launch_bounds__(256)
gauss_bf16_panels_kernel(uint64_t seed, int64_t s, int64_t npanel, uint16_t *__restrict__ Gb) {
    const int64_t total = npanel * s * 8;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = t / (s * 8), rem = t % (s * 8);
        const int64_t row = rem >> 3;
        const int qq = (int)(rem & 7);
        double g[4];
        gauss4(seed, (uint64_t)row, (uint64_t)(8 * p + qq), g);
        uint2 v;
        v.x = (uint32_t)bf16_rn((float)g[0]) | ((uint32_t)bf16_rn((float)g[1]) << 16);
        v.y = (uint32_t)bf16_rn((float)g[2]) | ((uint32_t)bf16_rn((float)g[3]) << 16);
        *reinterpret_cast<uint2 *>(Gb + ((p * s + row) * 32 + 4 * qq)) = v;
    }
}

// The stage's 128 x 32 tile of a pre-generated G into registers: thread t
// takes 8 values of k (quarter t & 3) of row t >> 2 (rows past s repeat row
// s - 1: their sketch rows are not written).
__device__ __forceinline__ u32x4 load_g(const uint16_t *__restrict__ Gb, int64_t s, int64_t m0, int64_t k0) {
    const int t = threadIdx.x;
    const int64_t row = min(m0 + (t >> 2), s - 1);
    return *reinterpret_cast<const u32x4 *>(Gb + (((k0 >> 5) * s + row) * 32 + 8 * (t & 3)));
}

__device__ __forceinline__ void store_g(uint16_t (*Gs)[HP], u32x4 v) {
    const int t = threadIdx.x;
    *reinterpret_cast<u32x4 *>(&Gs[t >> 2][8 * swz(t >> 2, t & 3)]) = v;
}

// fl32(T) split into its three BF16 terms once, in the layout of the
// kernel's LDS tile: plane `term`, panel p (k = 32 p .. 32 p + 31), column
// c holds the 32 values of k contiguously (zero past K and past d, padded
// to dp columns).  Workgroup b splits 32 k (panel b / (dp / 64)) x 64
// columns (block b % (dp / 64)): thread t loads 8
// rows of column t & 63 (each load of a wavefront reads 64 consecutive
// columns of one row), and writes each term as one 16-byte vector.
__global__ void __launch_bounds__(256)
split_t_planes_kernel(const double *__restrict__ T, int64_t ldt, int64_t K, int64_t d, int64_t npanel,
                      int64_t dp, uint16_t *__restrict__ Tp) {
    const int t = threadIdx.x;
    const int64_t cblocks = dp / 64;
    const int64_t col = ((int64_t)blockIdx.x % cblocks) * 64 + (t & 63);
    const int64_t p = (int64_t)blockIdx.x / cblocks;
    const int kq = t >> 6;  // 0..3: k = 32 p + 8 kq + j
    uint32_t w[3][4];
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
        uint32_t lo[3], hi[3];
        const int64_t k = 32 * p + 8 * kq + j;
        split3((k < K && col < d) ? T[k * ldt + col] : 0.0, lo);
        split3((k + 1 < K && col < d) ? T[(k + 1) * ldt + col] : 0.0, hi);
#pragma unroll
        for (int term = 0; term < 3; ++term) w[term][j / 2] = lo[term] | (hi[term] << 16);
    }
    if (col < dp) {
#pragma unroll
        for (int term = 0; term < 3; ++term) {
            uint4 *dst = reinterpret_cast<uint4 *>(Tp + (((int64_t)term * npanel + p) * dp + col) * 32 + 8 * kq);
            *dst = make_uint4(w[term][0], w[term][1], w[term][2], w[term][3]);
        }
    }
}

// The stage's three 128-column x 32-k tiles of the split planes (each an
// 8 KB block of 512 16-byte vectors): thread t takes vector t of every
// term, column t >> 2, k 8 (t & 3) .. 8 (t & 3) + 7.
__device__ __forceinline__ void load_tp(const uint16_t *__restrict__ Tp, int64_t npanel, int64_t dp,
                                        int64_t k0, int64_t n0, u32x4 (&reg)[3]) {
    const int t = threadIdx.x;
    const int64_t p = k0 >> 5;
#pragma unroll
    for (int term = 0; term < 3; ++term)
        reg[term] = reinterpret_cast<const u32x4 *>(Tp + (((int64_t)term * npanel + p) * dp + n0) * 32)[t];
}

__device__ __forceinline__ void store_tp(uint16_t (*As)[HBN][HP], const u32x4 (&reg)[3]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int term = 0; term < 3; ++term)
        *reinterpret_cast<u32x4 *>(&As[term][t >> 2][8 * swz(t >> 2, t & 3)]) = reg[term];
}

// One stage's operands on their way from HBM to LDS: the T terms (PRET),
// else the FP64 tile of T; the G tile when PRE (else G is generated at the
// store).
template <bool PRE, bool PRET, int NH>
struct StageRegs {
    u32x4 tp[NH][PRET ? 3 : 1];
    double t[PRET ? 1 : 8];
    uint32_t tmask;
    u32x4 g[NH];
};

// PRE: G comes from the pre-generated panels Gb, else each stage generates
// its tile (gen_g).  PRET (with PRE): the three terms of T come from the
// split planes Tp, else each stage splits its tile of T (store_t).  A stage
// covers NH panels of 32 k (NH = 2 with the pre-formed operands: half the
// barriers and stores per product), each with its own LDS tiles; the
// products run in the same k order either way.
template <bool PRE, bool PRET, int NH>
__global__ void __launch_bounds__(HNT, 1)
sketch_bf16_kernel(const double *__restrict__ T, int64_t ldt, int64_t K, int64_t d, int64_t s,
                   uint64_t seed, const uint16_t *__restrict__ Gb, const uint16_t *__restrict__ Tp,
                   int64_t npanel, int64_t dp, int64_t k_per_split, int tiles_m, double *__restrict__ Xp) {
    static_assert(PRE || !PRET, "the split planes come with the pre-generated G");
    static_assert(NH == 1 || PRET, "stages of several panels read the pre-formed operands");
    static_assert(FLUSH % NH == 0, "flushes fall on stage boundaries");
    constexpr int KS = HKT * NH;  // k per stage
    __shared__ uint16_t Gs[NH][HBM_][HP];
    __shared__ uint16_t As[NH][3][HBN][HP];
    const int tile = blockIdx.x;
    const int64_t m0 = (int64_t)(tile % tiles_m) * HBM_;
    const int64_t n0 = (int64_t)(tile / tiles_m) * HBN;
    const int64_t kbeg = (int64_t)blockIdx.y * k_per_split;
    const int64_t kend = min(K, kbeg + k_per_split);
    double *__restrict__ Xout = Xp + (int64_t)blockIdx.y * s * d;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 2, wn = wave & 3;  // 2 x 4 wavefronts of 64 rows x 32 columns
    const int lr = lane & 15, lk = lane >> 4;

    f32x4 acc[4][2];
    double acc64[4][2][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[i][j][v] = 0.0;
        }
    const int64_t nstage = kend > kbeg ? ceil_div(kend - kbeg, KS) : 0;
    using Regs = StageRegs<PRE, PRET, NH>;
    // (with NH = 2 the stage's second panel always exists: the host pads the
    // panels to a multiple of NH, zero past K in the planes)
    auto load = [&](Regs &r, int64_t k0) {
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            if constexpr (PRET) load_tp(Tp, npanel, dp, k0 + HKT * h, n0, r.tp[h]);
            if constexpr (PRE) r.g[h] = load_g(Gb, s, m0, k0 + HKT * h);
        }
        if constexpr (!PRET) r.tmask = load_t(T, ldt, k0, kend, n0, d, r.t);
    };
    auto store = [&](const Regs &r, int64_t k0) {
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            if constexpr (PRET) store_tp(As[h], r.tp[h]);
            if constexpr (PRE) store_g(Gs[h], r.g[h]);
        }
        if constexpr (!PRET) store_t(As[0], r.t, r.tmask);
        if constexpr (!PRE) gen_g(Gs[0], seed, m0, k0);
    };
    // one stage: 24 MFMA per wavefront and panel on the operands in LDS
    // (rows of T past the end of the slice were loaded as zero and the G
    // values there are finite, so their products vanish), then the FP64
    // flush every FLUSH panels
    auto mma = [&](int64_t st) {
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            bf16x8 a[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = wm * 64 + i * 16 + lr;
                a[i] = load8(&Gs[h][r][8 * swz(r, lk)]);
            }
#pragma unroll
            for (int term = 0; term < 3; ++term) {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int c = wn * 32 + j * 16 + lr;
                    const bf16x8 b = load8(&As[h][term][c][8 * swz(c, lk)]);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[i][j], 0, 0, 0);
                }
            }
        }
        if ((st + 1) % (FLUSH / NH) == 0 || st + 1 == nstage) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc64[i][j][v] += (double)acc[i][j][v];
                    acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
        }
    };
    // the operands of the next two stages are in flight (two register
    // sets; the stage's parity picks the set).  Loads are unconditional,
    // those past the last stage repeat it (unused), so that every path
    // through the loop leaves the same loads in flight and the waits before
    // the LDS stores cover one set only.
    if (nstage > 0) {
        const int64_t klast = kbeg + (nstage - 1) * KS;
        auto kst = [&](int64_t st) { return min(kbeg + st * KS, klast); };
        auto stage = [&](Regs &r, int64_t st) {
            __syncthreads();  // the previous stage's operands are consumed
            store(r, kst(st));
            __syncthreads();
            load(r, kst(st + 2));
            mma(st);
        };
        Regs r0, r1;
        load(r0, kst(0));
        load(r1, kst(1));
        // pairs of stages (a fixed trip count: every iteration runs both
        // halves), then the odd last stage from r0
        const int64_t npair = nstage / 2;
        for (int64_t pr = 0; pr < npair; ++pr) {
            stage(r0, 2 * pr);
            stage(r1, 2 * pr + 1);
        }
        if (nstage & 1) stage(r0, nstage - 1);
    }
    // accumulator element v of lane (lr, lk) is row 4 lk + v, column lr of its
    // 16 x 16 block; X is column-major
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t col = n0 + wn * 32 + j * 16 + lr;
            if (col < d) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = m0 + wm * 64 + i * 16 + 4 * lk + v;
                    if (row < s) Xout[col * s + row] = acc64[i][j][v];
                }
            }
        }
}

__global__ void __launch_bounds__(256)
sum_slices_bf16_kernel(const double *__restrict__ Xp, int nslice, int64_t count, double *__restrict__ X) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int sl = 0; sl < nslice; ++sl) acc += Xp[(int64_t)sl * count + t];
        X[t] = acc;
    }
}

// Rows of T rounded to FP32 (the storage of the precision form's sweeps).
__global__ void __launch_bounds__(256)
to_f32_kernel(int64_t rows, int64_t cols, const double *__restrict__ T, int64_t ldt,
              float *__restrict__ T32) {
    const int64_t total = rows * cols;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / cols, c = t % cols;
        T32[r * ldt + c] = (float)T[r * ldt + c];
    }
}

}  // namespace

// The largest pre-generated bf16(G), and the largest set of split T
// planes: LSRN_PREGEN_MAX_BYTES when set (read at every call; 0 turns both
// off), else 32 GiB.
static size_t pregen_max_bytes() {
    const char *e = std::getenv("LSRN_PREGEN_MAX_BYTES");
    if (e && *e) {
        char *end = nullptr;
        const unsigned long long v = std::strtoull(e, &end, 10);
        if (end && *end == '\0') return (size_t)v;
    }
    return kPreGenMaxBytes;
}

size_t sketch_bf16_g_bytes(int64_t K, int64_t d, int64_t s) {
    const size_t cap = pregen_max_bytes();
    const size_t np = (size_t)round_up(ceil_div(K, HKT), 2);
    const size_t b = np * (size_t)s * 32 * sizeof(uint16_t);
    if (b > cap) return 0;
    const size_t t = (size_t)3 * np * (size_t)(ceil_div(d, HBN) * HBN) * 32 * sizeof(uint16_t);
    return b + (t <= cap ? t : 0);
}

void sketch_rows_bf16(int64_t K, int64_t d, const double *T, int64_t ldt, double lambda, int64_t s,
                      uint64_t seed, double *X, hipStream_t st, double *kernel_ms) {
    const int tiles_m = (int)ceil_div(s, HBM_), tiles_n = (int)ceil_div(d, HBN);
    const int64_t tiles = (int64_t)tiles_m * tiles_n;
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (kernel_ms) {
        LSRN_HIP(hipEventCreate(&ev[0]));
        LSRN_HIP(hipEventCreate(&ev[1]));
        LSRN_HIP(hipEventRecord(ev[0], st));
    }
    // bf16(G) generated once into panels (s x K x 2 bytes) when that fits:
    // each tile of G is then read instead of generated once per column tile.
    // The panels are padded to an even count (the kernel's stages of two
    // panels), and so are the split planes below.
    DevBuf gpan;
    const size_t pre_cap = pregen_max_bytes();
    const int64_t npanel = round_up(ceil_div(K, HKT), 2);
    const size_t gbytes = (size_t)npanel * (size_t)s * 32 * sizeof(uint16_t);
    if (gbytes <= pre_cap) {
        try {
            gpan.alloc(gbytes);
        } catch (const Error &) {
            gpan.release();  // not enough device memory: generate in the kernel
        }
    }
    // with the panels, fl32(T) split once into its three BF16 terms (6 bytes
    // per entry) when that fits too: each stage then loads the terms
    // instead of splitting its tile of T (s / 128 times over)
    DevBuf tpl;
    const int64_t dp = (int64_t)tiles_n * HBN;
    const size_t tbytes = (size_t)3 * (size_t)npanel * (size_t)dp * 32 * sizeof(uint16_t);
    if (gpan.bytes() && tbytes <= pre_cap) {
        try {
            tpl.alloc(tbytes);
        } catch (const Error &) {
            tpl.release();  // split in the kernel
        }
    }
    // k split into slices when the tiles alone do not fill the chip; each
    // slice a whole number of two-panel stages on every path, so that the
    // paths share their slices and flush windows (and give the same bits)
    const int64_t kstage = 2 * HKT;
    const int64_t want = 2 * (int64_t)device_cus();
    int64_t nsplit = tiles >= want ? 1 : ceil_div(want, tiles);
    nsplit = std::min<int64_t>(nsplit, std::max<int64_t>(1, K / (16 * HKT)));
    const int64_t cap = std::max<int64_t>(1, (int64_t(1) << 31) / (8 * s * d));
    nsplit = std::max<int64_t>(1, std::min(nsplit, cap));
    const int64_t kps = round_up(ceil_div(K, nsplit), kstage);
    nsplit = std::max<int64_t>(1, ceil_div(K, kps));
    DevBuf part;
    double *Xp = X;
    if (nsplit > 1) {
        part.alloc((size_t)nsplit * (size_t)s * (size_t)d * sizeof(double));
        Xp = part.as<double>();
    }
    dim3 grid((unsigned)tiles, (unsigned)nsplit);
    if (gpan.bytes()) {
        const int64_t total = npanel * s * 8;
        gauss_bf16_panels_kernel<<<(unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 20), 256, 0, st>>>(
            seed, s, npanel, gpan.as<uint16_t>());
        if (tpl.bytes()) {
            // npanel x dp / 64 workgroups: at most 2^22 within the 32 GiB bound
            split_t_planes_kernel<<<(unsigned)(npanel * (dp / 64)), 256, 0, st>>>(
                T, ldt, K, d, npanel, dp, tpl.as<uint16_t>());
            sketch_bf16_kernel<true, true, 2><<<grid, HNT, 0, st>>>(T, ldt, K, d, s, seed, gpan.as<uint16_t>(),
                                                                 tpl.as<uint16_t>(), npanel, dp, kps, tiles_m, Xp);
        } else {
            sketch_bf16_kernel<true, false, 1><<<grid, HNT, 0, st>>>(T, ldt, K, d, s, seed, gpan.as<uint16_t>(),
                                                                  nullptr, npanel, dp, kps, tiles_m, Xp);
        }
    } else {
        sketch_bf16_kernel<false, false, 1><<<grid, HNT, 0, st>>>(T, ldt, K, d, s, seed, nullptr, nullptr, npanel,
                                                               dp, kps, tiles_m, Xp);
    }
    LSRN_HIP(hipGetLastError());
    if (kernel_ms) {
        LSRN_HIP(hipEventRecord(ev[1], st));
        LSRN_HIP(hipEventSynchronize(ev[1]));
        float ms = 0.f;
        LSRN_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        *kernel_ms = ms;
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
    }
    const int64_t count = s * d;
    if (nsplit > 1) {
        sum_slices_bf16_kernel<<<(unsigned)std::min<int64_t>(ceil_div(count, 256), 8192), 256, 0, st>>>(
            Xp, (int)nsplit, count, X);
        LSRN_HIP(hipGetLastError());
    }
    add_identity_rows(K, d, s, lambda, seed, X, st);
    LSRN_HIP(hipStreamSynchronize(st));  // before `part` is freed
}

void to_f32(int64_t rows, int64_t cols, const double *T, int64_t ldt, float *T32, hipStream_t st) {
    to_f32_kernel<<<(unsigned)std::min<int64_t>(ceil_div(rows * cols, 256), 65535), 256, 0, st>>>(
        rows, cols, T, ldt, T32);
    LSRN_HIP(hipGetLastError());
}

}  // namespace lsrn
