// sketch.hip -- the random normal projection of Alg. 1/2 step 3.
//
// X = G T for the tall view T of A (K x d, row-major): X is s x d, written
// column-major.  G (s x K) is generated on the fly from the Philox stream
// (rng.hpp) into LDS, one 16-column slice of the tile's rows at a time, and
// never reaches HBM.  The product runs on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): each workgroup owns a tile of X (64 x 512,
// 128 x 256 or 128 x 128) and one slice of K; the slices are summed in a
// fixed order by a second kernel.
#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "rng.hpp"

// Device memory of the no-allocation sketch (lsrn_sketch_dense_noalloc):
// the split-K partial sketches.  Every device the library runs on holds
// this array until the process ends.  In host code `scratch` is only a
// handle for hipGetSymbolAddress; kernels get the address it returns.
static __device__ __align__(256) unsigned char scratch[LSRN_NOALLOC_SCRATCH_BYTES];

namespace lsrn {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int KT = 16;    // k per LDS stage (four MFMA k-steps)
// A workgroup is WM x WN wavefronts of 64 x 64 each: 64 WM x 64 WN of X, so
// each generated slice of G serves 64 WN columns.  LDS row pitches are
// 32 (mod 64) dwords, so the four 16-lane groups of a wave read two
// disjoint bank halves.
template <int WM> constexpr int BM_ = 64 * WM;                  // rows of X per workgroup
template <int WN> constexpr int BN_ = 64 * WN;                  // cols of X per workgroup
template <int WM, int WN> constexpr int NT_ = 64 * WM * WN;     // threads
template <int WM> constexpr int LDP_ = 64 * WM + 16;            // pitch of the G slice
template <int WN> constexpr int TP_ = 64 * WN + 16;             // pitch of the T tile

// One MFMA 16x16x4 f64 step: lane l supplies A[l%16][l/16] (a 16x4 slice of
// G) and B[l/16][l%16] (a 4x16 slice of T); the 16x16 accumulator holds
// D[l/16 + 4 v][l%16] in element v of lane l.
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// G(i, k) for the BM rows of the tile and the 16 k of one stage: BM rows x
// 4 Philox blocks, block b of the slice (row b % BM, block b / BM of the
// stage) taken by thread b % NT.  With more threads than blocks (WM = 1,
// WN = 8) the first four wavefronts generate, one on each SIMD.
template <int WM, int WN>
__device__ __forceinline__ void gen_g_stage(double (*Gs)[LDP_<WM>], uint64_t seed, int64_t m0,
                                            int64_t kstage) {
    constexpr int NB = 4 * BM_<WM>, NT = NT_<WM, WN>;
#pragma unroll
    for (int h = 0; h < (NB + NT - 1) / NT; ++h) {
        const int b = (int)threadIdx.x + NT * h;
        if (NB % NT != 0 && b >= NB) break;
        const int row = b % BM_<WM>, qloc = b / BM_<WM>;  // qloc 0..3
        double g[4];
        gauss4(seed, (uint64_t)(m0 + row), (uint64_t)((kstage >> 2) + qloc), g);
#pragma unroll
        for (int j = 0; j < 4; ++j) Gs[qloc * 4 + j][row] = g[j];
    }
}

// 16 rows x BN columns of T for one stage into registers (zero outside
// [k0, kend) x [0, d)): 8 / WM double2 per thread.
template <int WM> constexpr int NLD_ = 8 / WM;
template <int WM, int WN, bool VEC2, typename TT>
__device__ __forceinline__ void load_t_stage(const TT *__restrict__ T, int64_t ldt,
                                             int64_t kstage, int64_t kend, int64_t n0, int64_t d,
                                             double2 (&reg)[NLD_<WM>]) {
    constexpr int HALF = BN_<WN> / 2;  // double2 per row of the tile
#pragma unroll
    for (int it = 0; it < NLD_<WM>; ++it) {
        const int idx = it * NT_<WM, WN> + threadIdx.x;
        const int kk = idx / HALF;         // 0..15
        const int c2 = (idx % HALF) * 2;   // 0..BN-2
        const int64_t k = kstage + kk, col = n0 + c2;
        double2 v = make_double2(0.0, 0.0);
        if (k < kend) {
            const TT *p = T + k * ldt + col;
            if (VEC2 && col + 1 < d) {
                if constexpr (sizeof(TT) == 8) {
                    v = *reinterpret_cast<const double2 *>(p);
                } else {
                    const float2 f = *reinterpret_cast<const float2 *>(p);
                    v = make_double2((double)f.x, (double)f.y);
                }
            } else {
                if (col < d) v.x = (double)p[0];
                if (col + 1 < d) v.y = (double)p[1];
            }
        }
        reg[it] = v;
    }
}

template <int WM, int WN>
__device__ __forceinline__ void store_t_stage(double (*Ts)[TP_<WN>], const double2 (&reg)[NLD_<WM>]) {
    constexpr int HALF = BN_<WN> / 2;
#pragma unroll
    for (int it = 0; it < NLD_<WM>; ++it) {
        const int idx = it * NT_<WM, WN> + threadIdx.x;
        const int kk = idx / HALF, c2 = (idx % HALF) * 2;
        Ts[kk][c2] = reg[it].x;
        Ts[kk][c2 + 1] = reg[it].y;
    }
}

// Tile `tile` of X for K-slice `split` (the workgroup's whole work).
template <int WM, int WN, bool VEC2, typename TT>
__device__ __forceinline__ void sketch_tile(const TT *__restrict__ T, int64_t ldt, int64_t K,
                                            int64_t d, int64_t s, uint64_t seed,
                                            int64_t k_per_split, int tiles_m,
                                            double *__restrict__ Xp, int tile, int split) {
    __shared__ double Gs[2][KT][LDP_<WM>];
    __shared__ double Ts[2][KT][TP_<WN>];

    const int64_t m0 = (int64_t)(tile % tiles_m) * BM_<WM>;
    const int64_t n0 = (int64_t)(tile / tiles_m) * BN_<WN>;
    const int64_t kbeg = (int64_t)split * k_per_split;
    const int64_t kend = min(K, kbeg + k_per_split);
    double *__restrict__ Xout = Xp + (int64_t)split * s * d;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int lr = lane & 15, lk = lane >> 4;

    f64x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int64_t nstage = kend > kbeg ? ceil_div(kend - kbeg, KT) : 0;
    double2 treg[NLD_<WM>];
    if (nstage > 0) {
        gen_g_stage<WM, WN>(Gs[0], seed, m0, kbeg);
        load_t_stage<WM, WN, VEC2, TT>(T, ldt, kbeg, kend, n0, d, treg);
        store_t_stage<WM, WN>(Ts[0], treg);
    }
    __syncthreads();

    for (int64_t st = 0; st < nstage; ++st) {
        const int buf = (int)(st & 1);
        const bool more = st + 1 < nstage;
        const int64_t knext = kbeg + (st + 1) * KT;
        if (more) load_t_stage<WM, WN, VEC2, TT>(T, ldt, knext, kend, n0, d, treg);
#pragma unroll
        for (int kk = 0; kk < KT / 4; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = Gs[buf][kk * 4 + lk][wm * 64 + i * 16 + lr];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Ts[buf][kk * 4 + lk][wn * 64 + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
        }
        if (more) {
            gen_g_stage<WM, WN>(Gs[buf ^ 1], seed, m0, knext);
            store_t_stage<WM, WN>(Ts[buf ^ 1], treg);
        }
        __syncthreads();
    }

    // Column-major store: element v of lane group lk is row lk + 4 v of its
    // 16 x 16 block, so for each v the four groups write 4 consecutive rows.
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t col = n0 + wn * 64 + j * 16 + lr;
            const int64_t rbase = m0 + wm * 64 + i * 16 + lk;
            if (col < d) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (rbase + 4 * v < s) Xout[col * s + rbase + 4 * v] = acc[i][j][v];
            }
        }
}

template <int WM, int WN, bool VEC2, typename TT = double>
__global__ void __launch_bounds__((NT_<WM, WN>), 8 / (WM * WN))
sketch_mfma_kernel(const TT *__restrict__ T, int64_t ldt, int64_t K, int64_t d, int64_t s,
                   uint64_t seed, int64_t k_per_split, int tiles_m, double *__restrict__ Xp) {
    sketch_tile<WM, WN, VEC2, TT>(T, ldt, K, d, s, seed, k_per_split, tiles_m, Xp, (int)blockIdx.x,
                              (int)blockIdx.y);
}

// One problem of a batched sketch: tiles_m x tiles_n tiles of X, each over
// nsplit slices of k_per_split rows of T (slice j's partial sums in
// Xp + j s d when nsplit > 1, else in X itself).
struct SkItem {
    const double *T;
    int64_t ldt, K, d, s;
    double *X;
    int tiles_m, tiles, nsplit;
    int64_t k_per_split;
    double *Xp;
    uint64_t seed;  // the problem's Philox key
};

// Every (tile, slice) of every problem in one launch: workgroup g is work
// item g - off[p] of problem p (off: prefix sums of tiles x nsplit).
template <bool VEC2>
__global__ void __launch_bounds__((NT_<2, 2>), 2)
sketch_batch_kernel(const SkItem *__restrict__ items, const int *__restrict__ off, int n) {
    const int g = (int)blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    const SkItem it = items[lo];
    const int w = g - off[lo];
    sketch_tile<2, 2, VEC2, double>(it.T, it.ldt, it.K, it.d, it.s, it.seed, it.k_per_split, it.tiles_m,
                                 it.nsplit > 1 ? it.Xp : it.X, w % it.tiles, w / it.tiles);
}

// X = the sum of a split problem's slices in ascending order, for every
// split problem of a batch: workgroup g covers 256 entries of problem p.
__global__ void __launch_bounds__(256)
sum_slices_batch_kernel(const SkItem *__restrict__ items, const int *__restrict__ off, int n) {
    const int g = (int)blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    const SkItem &it = items[lo];
    const int64_t count = it.s * it.d;
    const int64_t t = (int64_t)(g - off[lo]) * 256 + threadIdx.x;
    if (t >= count) return;
    double acc = 0.0;
    for (int sl = 0; sl < it.nsplit; ++sl) acc += it.Xp[(int64_t)sl * count + t];
    it.X[t] = acc;
}

// X[idx] = sum over slices of Xp[slice][idx], slices in ascending order.
__global__ void __launch_bounds__(256)
sum_slices_kernel(const double *__restrict__ Xp, int nslice, int64_t count, double *__restrict__ X) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int sl = 0; sl < nslice; ++sl) acc += Xp[(int64_t)sl * count + t];
        X[t] = acc;
    }
}

// Rows lambda * I of the augmented matrix (Sec. 5): X(i, c) += lambda G(i, K + c).
__global__ void __launch_bounds__(256)
add_identity_rows_kernel(int64_t K, int64_t d, int64_t s, double lambda, uint64_t seed,
                         double *__restrict__ X) {
    const int64_t total = s * d;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = t / s, i = t % s;
        const uint64_t col = (uint64_t)(K + c);
        double g[4];
        gauss4(seed, (uint64_t)i, col >> 2, g);
        X[t] += lambda * g[col & 3];
    }
}

template <typename E = double>
__global__ void __launch_bounds__(256)
transpose_kernel(int64_t rows, int64_t cols, const E *__restrict__ in, int64_t ldin,
                 E *__restrict__ out) {
    __shared__ E tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int64_t r = r0 + k, c = c0 + tx;
        tile[k][tx] = (r < rows && c < cols) ? in[r * ldin + c] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int64_t c = c0 + k, r = r0 + tx;
        if (c < cols && r < rows) out[c * rows + r] = tile[tx][k];
    }
}

struct SketchPlan {
    int wm, wn, tiles_m, tiles_n, nsplit;
    int64_t k_per_split;
};

// G is generated once per column tile, so wider tiles regenerate it less.
// The 64 x 512 tile (8 wavefronts across, one workgroup per CU) is taken
// when its grid gives all but a sixteenth of the CUs a tile without padding
// more columns than the 128 x 256 tile (4 across, one per CU), which is
// taken when it alone gives every CU a tile; else the 128 x 128 tile (two
// workgroups per CU), with split-K when even that is too few.  The sums
// over k run in the same order in every tile shape.  FP32 entries keep to
// the 128-row tiles (measured: the 64 x 512 tile is slower for them).
SketchPlan plan_sketch(int64_t K, int64_t d, int64_t s, bool f64_entries) {
    SketchPlan p;
    const int64_t cus = device_cus();
    const int64_t tiles8 = ceil_div(s, BM_<1>) * ceil_div(d, BN_<8>);
    const bool pad_ok = ceil_div(d, BN_<8>) * BN_<8> <= ceil_div(d, BN_<4>) * BN_<4>;
    if (f64_entries && pad_ok && tiles8 * 16 >= cus * 15) {
        p.wm = 1;
        p.wn = 8;
    } else {
        p.wm = 2;
        p.wn = ceil_div(s, BM_<2>) * ceil_div(d, BN_<4>) >= cus ? 4 : 2;
    }
    p.tiles_m = (int)ceil_div(s, 64 * p.wm);
    p.tiles_n = (int)ceil_div(d, 64 * p.wn);
    const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n;
    const int64_t want = (p.wm * p.wn == 8 ? 1 : 2) * cus;  // resident workgroups
    int64_t nsplit = (tiles >= want || p.wm == 1) ? 1 : ceil_div(want, tiles);
    // keep at least 8 stages per slice and the partial sums under 2 GiB
    nsplit = std::min<int64_t>(nsplit, std::max<int64_t>(1, K / (8 * KT)));
    const int64_t cap = std::max<int64_t>(1, (int64_t(1) << 31) / (8 * s * d));
    nsplit = std::max<int64_t>(1, std::min(nsplit, cap));
    p.k_per_split = round_up(ceil_div(K, nsplit), KT);
    p.nsplit = (int)ceil_div(K, p.k_per_split);
    if (p.nsplit < 1) p.nsplit = 1;
    return p;
}

}  // namespace

size_t sketch_workspace_bytes(int64_t K, int64_t d, int64_t s) {
    size_t most = 0;
    for (const bool f64 : {true, false}) {
        const SketchPlan p = plan_sketch(K, d, s, f64);
        if (p.nsplit > 1) most = std::max(most, (size_t)p.nsplit * (size_t)s * (size_t)d * sizeof(double));
    }
    return most;
}

namespace {

// With `slices` (device memory of at least nsplit s d doubles) the split-K
// partial sketches go there and nothing is allocated or synchronised.
template <typename TT>
void sketch_rows_t(int64_t K, int64_t d, const TT *T, int64_t ldt, double lambda, int64_t s,
                   uint64_t seed, double *X, hipStream_t st, double *kernel_ms,
                   double *slices = nullptr) {
    SketchPlan p = plan_sketch(K, d, s, sizeof(TT) == sizeof(double));
    DevBuf part;
    double *Xp = X;
    if (p.nsplit > 1) {
        if (slices) {
            Xp = slices;
        } else {
            part.alloc((size_t)p.nsplit * (size_t)s * (size_t)d * sizeof(double));
            Xp = part.as<double>();
        }
    }
    dim3 grid((unsigned)(p.tiles_m * p.tiles_n), (unsigned)p.nsplit);
    const bool vec2 = (ldt % 2 == 0) && ((reinterpret_cast<uintptr_t>(T) & (2 * sizeof(TT) - 1)) == 0);
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (kernel_ms) {
        LSRN_HIP(hipEventCreate(&ev[0]));
        LSRN_HIP(hipEventCreate(&ev[1]));
        LSRN_HIP(hipEventRecord(ev[0], st));
    }
    auto launch = [&](auto wm_c, auto wn_c) {
        constexpr int WM = decltype(wm_c)::value, WN = decltype(wn_c)::value;
        if (vec2)
            sketch_mfma_kernel<WM, WN, true, TT><<<grid, NT_<WM, WN>, 0, st>>>(
                T, ldt, K, d, s, seed, p.k_per_split, p.tiles_m, Xp);
        else
            sketch_mfma_kernel<WM, WN, false, TT><<<grid, NT_<WM, WN>, 0, st>>>(
                T, ldt, K, d, s, seed, p.k_per_split, p.tiles_m, Xp);
    };
    if (p.wm == 1) {  // FP64 entries only
        if constexpr (sizeof(TT) == sizeof(double))
            launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 8>{});
    } else if (p.wn == 4)
        launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 4>{});
    else
        launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{});
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
    const int blocks = (int)std::min<int64_t>(ceil_div(count, 256), 8192);
    if (p.nsplit > 1) {
        sum_slices_kernel<<<blocks, 256, 0, st>>>(Xp, p.nsplit, count, X);
        LSRN_HIP(hipGetLastError());
    }
    if (lambda > 0.0) {
        add_identity_rows_kernel<<<blocks, 256, 0, st>>>(K, d, s, lambda, seed, X);
        LSRN_HIP(hipGetLastError());
    }
    if (p.nsplit > 1 && !slices) LSRN_HIP(hipStreamSynchronize(st));  // before `part` is freed
}

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
double *scratch_on_current_device() {
    int dev = 0;
    LSRN_HIP(hipGetDevice(&dev));
    LSRN_REQUIRE(dev >= 0 && dev < kMaxDevices, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        LSRN_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        LSRN_REQUIRE(ptr != nullptr, "no device address for the static scratch");
        g_scratch_ptr[dev] = ptr;
    }
    return static_cast<double *>(g_scratch_ptr[dev]);
}

}  // namespace

size_t sketch_slices_bytes(int64_t K, int64_t d, int64_t s) {
    const SketchPlan p = plan_sketch(K, d, s, true);
    return p.nsplit > 1 ? (size_t)p.nsplit * (size_t)s * (size_t)d * sizeof(double) : 0;
}

void sketch_rows_noalloc(int64_t K, int64_t d, const double *T, int64_t ldt, double lambda,
                         int64_t s, uint64_t seed, double *X, hipStream_t st) {
    const size_t need = sketch_slices_bytes(K, d, s);
    if (need > (size_t)LSRN_NOALLOC_SCRATCH_BYTES)
        fail(LSRN_E_NOMEM, "the sketch needs " + std::to_string(need) +
                               " bytes of partial sums; the static scratch holds " +
                               std::to_string((size_t)LSRN_NOALLOC_SCRATCH_BYTES));
    double *slices = need > 0 ? scratch_on_current_device() : nullptr;
    sketch_rows_t(K, d, T, ldt, lambda, s, seed, X, st, nullptr, slices);
}

void sketch_rows(int64_t K, int64_t d, const double *T, int64_t ldt, double lambda, int64_t s,
                 uint64_t seed, double *X, hipStream_t st, double *kernel_ms) {
    sketch_rows_t(K, d, T, ldt, lambda, s, seed, X, st, kernel_ms);
}

void sketch_rows(int64_t K, int64_t d, const float *T, int64_t ldt, double lambda, int64_t s,
                 uint64_t seed, double *X, hipStream_t st, double *kernel_ms) {
    sketch_rows_t(K, d, T, ldt, lambda, s, seed, X, st, kernel_ms);
}

// Slices of K for one problem of a batch, from its own sizes alone (so its
// bits do not depend on the rest of the batch): slices of at least
// kBatchSliceRows rows, and no more than about 256 work items a problem.
constexpr int64_t kBatchSliceRows = 2048;

void sketch_rows_batch(int count, const int64_t *K, const int64_t *d, const double *const *T,
                       const int64_t *ldt, const int64_t *s, const uint64_t *seeds, double *const *X,
                       hipStream_t st) {
    for (int pass = 0; pass < 2; ++pass) {  // rows aligned for paired loads, then the rest
        std::vector<SkItem> items;
        std::vector<int> off(1, 0);
        size_t slice_elems = 0;
        for (int p = 0; p < count; ++p) {
            const bool vec2 = (ldt[p] % 2 == 0) && ((reinterpret_cast<uintptr_t>(T[p]) & 15) == 0);
            if (vec2 != (pass == 0)) continue;
            const int tm = (int)ceil_div(s[p], BM_<2>), tn = (int)ceil_div(d[p], BN_<2>);
            const int tiles = tm * tn;
            int nsplit = (int)std::min<int64_t>(K[p] / kBatchSliceRows, std::max(1, 256 / tiles));
            nsplit = std::max(nsplit, 1);
            int64_t kps = round_up(ceil_div(K[p], (int64_t)nsplit), (int64_t)KT);
            nsplit = (int)ceil_div(K[p], kps);  // no empty slice
            items.push_back(SkItem{T[p], ldt[p], K[p], d[p], s[p], X[p], tm, tiles, nsplit, kps, nullptr,
                                   seeds[p]});
            if (nsplit > 1) slice_elems += (size_t)nsplit * (size_t)s[p] * (size_t)d[p];
            off.push_back(off.back() + tiles * nsplit);
        }
        if (items.empty()) continue;
        const int n = (int)items.size();
        DevBuf slices(slice_elems * sizeof(double));
        std::vector<SkItem> split_items;
        std::vector<int> off_sum(1, 0);
        size_t at = 0;
        for (SkItem &it : items) {
            if (it.nsplit <= 1) continue;
            it.Xp = slices.as<double>() + at;
            at += (size_t)it.nsplit * (size_t)it.s * (size_t)it.d;
            split_items.push_back(it);
            off_sum.push_back(off_sum.back() + (int)ceil_div(it.s * it.d, (int64_t)256));
        }
        const int ns = (int)split_items.size();
        DevBuf ditems((size_t)(n + ns) * sizeof(SkItem)), doff((off.size() + off_sum.size()) * sizeof(int));
        LSRN_HIP(hipMemcpyAsync(ditems.as<SkItem>(), items.data(), (size_t)n * sizeof(SkItem),
                                hipMemcpyHostToDevice, st));
        LSRN_HIP(hipMemcpyAsync(doff.as<int>(), off.data(), off.size() * sizeof(int),
                                hipMemcpyHostToDevice, st));
        if (ns > 0) {
            LSRN_HIP(hipMemcpyAsync(ditems.as<SkItem>() + n, split_items.data(), (size_t)ns * sizeof(SkItem),
                                    hipMemcpyHostToDevice, st));
            LSRN_HIP(hipMemcpyAsync(doff.as<int>() + off.size(), off_sum.data(), off_sum.size() * sizeof(int),
                                    hipMemcpyHostToDevice, st));
        }
        if (pass == 0)
            sketch_batch_kernel<true><<<(unsigned)off.back(), NT_<2, 2>, 0, st>>>(ditems.as<SkItem>(),
                                                                               doff.as<int>(), n);
        else
            sketch_batch_kernel<false><<<(unsigned)off.back(), NT_<2, 2>, 0, st>>>(ditems.as<SkItem>(),
                                                                                doff.as<int>(), n);
        LSRN_HIP(hipGetLastError());
        if (ns > 0) {
            sum_slices_batch_kernel<<<(unsigned)off_sum.back(), 256, 0, st>>>(
                ditems.as<SkItem>() + n, doff.as<int>() + off.size(), ns);
            LSRN_HIP(hipGetLastError());
        }
        LSRN_HIP(hipStreamSynchronize(st));  // before the tables and slices are freed
    }
}

void add_identity_rows(int64_t K, int64_t d, int64_t s, double lambda, uint64_t seed, double *X,
                       hipStream_t st) {
    if (!(lambda > 0.0)) return;
    const int blocks = (int)std::min<int64_t>(ceil_div(s * d, 256), 8192);
    add_identity_rows_kernel<<<blocks, 256, 0, st>>>(K, d, s, lambda, seed, X);
    LSRN_HIP(hipGetLastError());
}

void transpose(int64_t rows, int64_t cols, const float *in, int64_t ldin, float *out,
               hipStream_t st) {
    dim3 grid((unsigned)ceil_div(cols, 32), (unsigned)ceil_div(rows, 32));
    transpose_kernel<float><<<grid, 256, 0, st>>>(rows, cols, in, ldin, out);
    LSRN_HIP(hipGetLastError());
}

void transpose(int64_t rows, int64_t cols, const double *in, int64_t ldin, double *out,
               hipStream_t st) {
    dim3 grid((unsigned)ceil_div(cols, 32), (unsigned)ceil_div(rows, 32));
    transpose_kernel<double><<<grid, 256, 0, st>>>(rows, cols, in, ldin, out);
    LSRN_HIP(hipGetLastError());
}

}  // namespace lsrn
