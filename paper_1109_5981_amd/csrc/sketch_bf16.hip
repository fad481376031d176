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
// Workgroup: 256 threads (one wavefront per SIMD, so the FP32 and FP64
// accumulators fit in registers), a 128 x 128 tile of X (2 x 2 wavefronts of
// 64 x 64, each 4 x 4 blocks of 16 x 16), 32 values of k per stage; the next
// stage's T tile is loaded into registers while the current one is
// multiplied.
#include "internal.hpp"
#include "rng.hpp"

namespace lsrn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int HBM_ = 128;  // sketch rows per workgroup
constexpr int HBN = 128;   // columns per workgroup
constexpr int HKT = 32;    // k per stage
constexpr int HP = 40;     // LDS pitch (bf16) of a row of 32 k: 80 bytes
constexpr int HNT = 256;
constexpr int FLUSH = 8;   // stages accumulated in FP32 before the FP64 flush
constexpr size_t kPreGenMaxBytes = (size_t)32 << 30;  // largest pre-generated bf16(G)

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rn(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

// G for the 128 rows x 32 k of a stage: 128 rows x 8 Philox blocks, four
// per thread; Gs[row][k] (k contiguous), each block's four values stored
// as one 8-byte vector.
__device__ __forceinline__ void gen_g(uint16_t (*Gs)[HP], uint64_t seed, int64_t m0, int64_t k0) {
    const int t = threadIdx.x;
    const int row = t & (HBM_ - 1);
    const int qb = t >> 7;  // 0..1
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        const int q = qb + 2 * h;  // 0..7
        double g[4];
        gauss4(seed, (uint64_t)(m0 + row), (uint64_t)((k0 >> 2) + q), g);
        uint2 v;
        v.x = (uint32_t)bf16_rn((float)g[0]) | ((uint32_t)bf16_rn((float)g[1]) << 16);
        v.y = (uint32_t)bf16_rn((float)g[2]) | ((uint32_t)bf16_rn((float)g[3]) << 16);
        *reinterpret_cast<uint2 *>(&Gs[row][4 * q]) = v;
    }
}

// T tile (32 k x 128 columns, FP64 row-major) into registers: thread t
// takes column t & 127 of rows 16 (t >> 7) + j, j = 0..15 (each load of a
// wavefront reads 64 consecutive columns of one row).
__device__ __forceinline__ void load_t(const double *__restrict__ T, int64_t ldt, int64_t k0,
                                       int64_t K, int64_t n0, int64_t d, double (&reg)[16]) {
    const int t = threadIdx.x;
    const int64_t col = n0 + (t & (HBN - 1));
    const int64_t kb = k0 + 16 * (t >> 7);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int64_t k = kb + j;
        reg[j] = (k < K && col < d) ? T[k * ldt + col] : 0.0;
    }
}

// Split and store: As[term][col][k], the 16 values of k of a thread as two
// 16-byte vectors per term.
__device__ __forceinline__ void store_t(uint16_t (*As)[HBN][HP], const double (&reg)[16]) {
    const int t = threadIdx.x;
    const int c = t & (HBN - 1);
    const int kb = 16 * (t >> 7);
    uint32_t w[3][8];
#pragma unroll
    for (int j = 0; j < 16; j += 2) {
        uint32_t lo[3], hi[3];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float f = (float)reg[j + h];
            const uint16_t t1 = bf16_rn(f);
            const float r1 = f - bf16_to_f32(t1);
            const uint16_t t2 = bf16_rn(r1);
            const float r2 = r1 - bf16_to_f32(t2);
            const uint16_t t3 = bf16_rn(r2);
            (h ? hi : lo)[0] = t1;
            (h ? hi : lo)[1] = t2;
            (h ? hi : lo)[2] = t3;
        }
#pragma unroll
        for (int term = 0; term < 3; ++term) w[term][j / 2] = lo[term] | (hi[term] << 16);
    }
#pragma unroll
    for (int term = 0; term < 3; ++term) {
        uint4 *dst = reinterpret_cast<uint4 *>(&As[term][c][kb]);
        dst[0] = make_uint4(w[term][0], w[term][1], w[term][2], w[term][3]);
        dst[1] = make_uint4(w[term][4], w[term][5], w[term][6], w[term][7]);
    }
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
// takes 16 values of k (half t & 1) of row t >> 1 (rows past s repeat row
// s - 1: their sketch rows are not written).
__device__ __forceinline__ void load_g(const uint16_t *__restrict__ Gb, int64_t s, int64_t m0, int64_t k0,
                                       uint4 (&reg)[2]) {
    const int t = threadIdx.x;
    const int64_t row = min(m0 + (t >> 1), s - 1);
    const uint4 *src = reinterpret_cast<const uint4 *>(Gb + (((k0 >> 5) * s + row) * 32 + 16 * (t & 1)));
    reg[0] = src[0];
    reg[1] = src[1];
}

__device__ __forceinline__ void store_g(uint16_t (*Gs)[HP], const uint4 (&reg)[2]) {
    const int t = threadIdx.x;
    uint4 *dst = reinterpret_cast<uint4 *>(&Gs[t >> 1][16 * (t & 1)]);
    dst[0] = reg[0];
    dst[1] = reg[1];
}

// PRE: G comes from the pre-generated panels Gb, else each stage generates
// its tile (gen_g).
template <bool PRE>
__global__ void __launch_bounds__(HNT, 1)
sketch_bf16_kernel(const double *__restrict__ T, int64_t ldt, int64_t K, int64_t d, int64_t s,
                   uint64_t seed, const uint16_t *__restrict__ Gb, int64_t k_per_split, int tiles_m,
                   double *__restrict__ Xp) {
    __shared__ uint16_t Gs[HBM_][HP];
    __shared__ uint16_t As[3][HBN][HP];
    const int tile = blockIdx.x;
    const int64_t m0 = (int64_t)(tile % tiles_m) * HBM_;
    const int64_t n0 = (int64_t)(tile / tiles_m) * HBN;
    const int64_t kbeg = (int64_t)blockIdx.y * k_per_split;
    const int64_t kend = min(K, kbeg + k_per_split);
    double *__restrict__ Xout = Xp + (int64_t)blockIdx.y * s * d;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;  // 2 x 2 wavefronts
    const int lr = lane & 15, lk = lane >> 4;

    f32x4 acc[4][4];
    double acc64[4][4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[i][j][v] = 0.0;
        }
    const int64_t nstage = kend > kbeg ? ceil_div(kend - kbeg, HKT) : 0;
    double treg[16];
    uint4 greg[2];
    if (nstage > 0) {
        load_t(T, ldt, kbeg, kend, n0, d, treg);
        if (PRE) load_g(Gb, s, m0, kbeg, greg);
    }
    for (int64_t st = 0; st < nstage; ++st) {
        const int64_t k0 = kbeg + st * HKT;
        __syncthreads();  // the previous stage's operands are consumed
        store_t(As, treg);
        if (PRE) store_g(Gs, greg);
        else gen_g(Gs, seed, m0, k0);
        __syncthreads();
        if (st + 1 < nstage) {
            load_t(T, ldt, k0 + HKT, kend, n0, d, treg);
            if (PRE) load_g(Gb, s, m0, k0 + HKT, greg);
        }
        // rows of T past the end of the slice were loaded as zero and the
        // G values there are finite, so their products vanish
        bf16x8 a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = load8(&Gs[wm * 64 + i * 16 + lr][lk * 8]);
#pragma unroll
        for (int term = 0; term < 3; ++term) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bf16x8 b = load8(&As[term][wn * 64 + j * 16 + lr][lk * 8]);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[i][j], 0, 0, 0);
            }
        }
        if ((st + 1) % FLUSH == 0 || st + 1 == nstage) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc64[i][j][v] += (double)acc[i][j][v];
                    acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
        }
    }
    // accumulator element v of lane (lr, lk) is row 4 lk + v, column lr of its
    // 16 x 16 block; X is column-major
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t col = n0 + wn * 64 + j * 16 + lr;
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

size_t sketch_bf16_g_bytes(int64_t K, int64_t s) {
    const size_t b = (size_t)ceil_div(K, HKT) * (size_t)s * 32 * sizeof(uint16_t);
    return b <= kPreGenMaxBytes ? b : 0;
}

void sketch_rows_bf16(int64_t K, int64_t d, const double *T, int64_t ldt, double lambda, int64_t s,
                      uint64_t seed, double *X, hipStream_t st, double *kernel_ms) {
    const int tiles_m = (int)ceil_div(s, HBM_), tiles_n = (int)ceil_div(d, HBN);
    const int64_t tiles = (int64_t)tiles_m * tiles_n;
    const int64_t want = 2 * (int64_t)device_cus();
    int64_t nsplit = tiles >= want ? 1 : ceil_div(want, tiles);
    nsplit = std::min<int64_t>(nsplit, std::max<int64_t>(1, K / (16 * HKT)));
    const int64_t cap = std::max<int64_t>(1, (int64_t(1) << 31) / (8 * s * d));
    nsplit = std::max<int64_t>(1, std::min(nsplit, cap));
    const int64_t kps = round_up(ceil_div(K, nsplit), HKT);
    nsplit = std::max<int64_t>(1, ceil_div(K, kps));
    DevBuf part;
    double *Xp = X;
    if (nsplit > 1) {
        part.alloc((size_t)nsplit * (size_t)s * (size_t)d * sizeof(double));
        Xp = part.as<double>();
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (kernel_ms) {
        LSRN_HIP(hipEventCreate(&ev[0]));
        LSRN_HIP(hipEventCreate(&ev[1]));
        LSRN_HIP(hipEventRecord(ev[0], st));
    }
    // bf16(G) generated once into panels (s x K x 2 bytes) when that fits:
    // each tile of G is then read instead of generated once per column tile
    DevBuf gpan;
    const int64_t npanel = ceil_div(K, HKT);
    const size_t gbytes = (size_t)npanel * (size_t)s * 32 * sizeof(uint16_t);
    if (gbytes <= kPreGenMaxBytes && fast_paths_allowed()) {
        try {
            gpan.alloc(gbytes);
        } catch (const Error &) {
            gpan.release();  // not enough device memory: generate in the kernel
        }
    }
    dim3 grid((unsigned)tiles, (unsigned)nsplit);
    if (gpan.bytes()) {
        const int64_t total = npanel * s * 8;
        gauss_bf16_panels_kernel<<<(unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 20), 256, 0, st>>>(
            seed, s, npanel, gpan.as<uint16_t>());
        sketch_bf16_kernel<true><<<grid, HNT, 0, st>>>(T, ldt, K, d, s, seed, gpan.as<uint16_t>(), kps,
                                                       tiles_m, Xp);
    } else {
        sketch_bf16_kernel<false><<<grid, HNT, 0, st>>>(T, ldt, K, d, s, seed, nullptr, kps, tiles_m, Xp);
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
