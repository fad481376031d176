// csr.hip -- sparse A in CSR: validation, the transposed structure, and the
// sketch X = G T of the tall view T (Alg. 1/2 steps 2-3 for sparse A;
// Sec. 5 for the Tikhonov rows).
//
// The sketch keeps an S x C tile of X in LDS per workgroup (S sketch rows,
// C columns of T) and walks the nonzeros of T that fall in those C columns
// in order of their row k.  G(i, 4q .. 4q+3) is one Philox block, so the
// workgroup generates, batch by batch, the S x 4QB slice of G for the rows
// kb .. kb + 4QB of T once into LDS; every nonzero (k, c, v) of the batch
// then adds v G(i, k) to a slot of the tile for the S rows.  Each slot has
// one writer thread (slot mod NT) and its nonzeros come in row order, so
// the summation order is fixed and the result deterministic.  A column of
// T with many nonzeros per batch (the dense columns of a sparse matrix, the
// low DCT frequencies of an image matrix) would make its one writer walk
// all of them while the workgroup waits at the next batch: such a column
// gets P slots past the C column slots (a power of two chosen so that each
// receives about 4 nonzeros per batch), nonzero k goes to slot k mod P, and
// the column is the sum of its slots in slot order at the end.  Each slice
// of G is generated once per column block.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "rng.hpp"

namespace lsrn {

namespace {

constexpr int SK_PF = 8;    // entries per thread loaded one batch ahead
constexpr int SK_LDS = 160 * 1024 / (int)sizeof(double);  // doubles of LDS per workgroup

// Rows of T per batch for S sketch rows per workgroup of NT threads: every
// thread generates one Philox block (4 entries of G) per batch, so the
// slice of G is S x KB = 4 NT entries.
constexpr int sk_kb(int S, int NT) { return 4 * (NT / S); }

struct SkEntry {
    int32_t k;  // row of T
    int32_t c;  // column of T minus the block's first column
    double v;
};

// Structure checks, parallel over rows (the offsets) and over entries (the
// column indices), so that long rows do not serialise a thread.
__global__ void check_ptr_kernel(int64_t m, int64_t nnz, const int64_t *__restrict__ ptr,
                                 int *__restrict__ bad) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = ptr[r], b = ptr[r + 1];
        if (a < 0 || b < a || b > nnz) atomicOr(bad, 1);
    }
}

__global__ void check_idx_kernel(int64_t nnz, int64_t n, const int32_t *__restrict__ idx,
                                 int *__restrict__ bad) {
    bool out = false;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = idx[e];
        out = out || c < 0 || (int64_t)c >= n;
    }
    if (__any(out) && (threadIdx.x & 63) == 0) atomicOr(bad, 2);
}

// One wavefront per row (grid-stride over rows), its lanes over the row's
// entries, so that a long row (a fat matrix has rows of ~nnz / m entries)
// does not serialise one thread.
__global__ void expand_rows_kernel(int64_t nrows, const int64_t *__restrict__ ptr,
                                   int32_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = wave; r < nrows; r += nwaves)
        for (int64_t e = ptr[r] + lane; e < ptr[r + 1]; e += 64) out[e] = (int32_t)r;
}

__global__ void iota_kernel(int64_t n, int32_t *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)i;
}

// ptr[g] = first position of key >= g in the sorted keys, g = 0 .. ngroups.
__global__ void bounds_kernel(int64_t nkeys, const uint32_t *__restrict__ keys, int64_t ngroups,
                              int64_t *__restrict__ ptr) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= ngroups;
         g += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = nkeys;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)keys[mid] < g) lo = mid + 1;
            else hi = mid;
        }
        ptr[g] = lo;
    }
}

__global__ void gather_transpose_kernel(int64_t nnz, const int32_t *__restrict__ perm,
                                        const int32_t *__restrict__ rowof,
                                        const double *__restrict__ val, int32_t *__restrict__ tidx,
                                        double *__restrict__ tval) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = perm[j];
        tidx[j] = rowof[e];
        tval[j] = val[e];
    }
}

// Tile slot of a nonzero in column c, row k of T: the column's own slot
// c mod C, or for a column split into nslot[c] > 1 slots, slot
// C + sbase[c] + (k mod nslot[c]).
__device__ __forceinline__ int sketch_slot(int32_t c, int32_t k, int C,
                                           const int32_t *__restrict__ sbase,
                                           const int32_t *__restrict__ nslot) {
    const int p = nslot[c];
    return p > 1 ? C + sbase[c] + (k & (p - 1)) : c % C;
}

// key of entry e for the sketch order: (column block, batch of rows of T,
// writer thread of its slot); the stable sort keeps the rows in order
// within a key.
__global__ void sketch_keys_kernel(int64_t nnz, const int32_t *__restrict__ idx,
                                   const int32_t *__restrict__ rowof, int C, int KB, int NT, int64_t nbatch,
                                   const int32_t *__restrict__ sbase,
                                   const int32_t *__restrict__ nslot, uint32_t *__restrict__ keys) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = idx[e], k = rowof[e];
        const int64_t batch = k / KB;
        const int slot = sketch_slot(c, k, C, sbase, nslot);
        keys[e] = (uint32_t)(((int64_t)(c / C) * nbatch + batch) * NT + (slot % NT));
    }
}

__global__ void gather_sketch_kernel(int64_t nnz, const int32_t *__restrict__ perm,
                                     const int32_t *__restrict__ rowof,
                                     const int32_t *__restrict__ idx,
                                     const double *__restrict__ val, int C,
                                     const int32_t *__restrict__ sbase,
                                     const int32_t *__restrict__ nslot,
                                     SkEntry *__restrict__ out) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = perm[j];
        const int32_t c = idx[e], k = rowof[e];
        out[j] = SkEntry{k, sketch_slot(c, k, C, sbase, nslot), val[e]};
    }
}

// LDS position (in 16-byte vectors) of vector h of slot c in a tile of H
// vectors per slot.  The lanes of a wavefront touch unrelated slots; with a
// plain c H + h, H = 2 / 4 / 8 would put every lane's vector h on the same
// 1/8 .. 1/2 of the 16 bank groups of a 256-byte LDS row.  Rotating h by
// the slot's position within the row period spreads them over all 16.
template <int H>
__device__ __forceinline__ int tix(int c, int h) {
    static_assert(H == 2 || H == 4, "2 or 4 vectors per slot");
    constexpr int SPAN = 16 / H;  // slots per 256-byte row
    return c * H + (h ^ ((c / SPAN) & (H - 1)));
}

template <int S, int NT>
__global__ void __launch_bounds__(NT)
csr_sketch_kernel(const SkEntry *__restrict__ ent, const int64_t *__restrict__ optr, int64_t K,
                  int64_t d, int C, int W, int64_t nbatch, int64_t bpz, int64_t s, uint64_t seed,
                  const int32_t *__restrict__ sbase, const int32_t *__restrict__ nslot,
                  double *__restrict__ out, int64_t zstride) {
    static_assert(S % 2 == 0 && NT % S == 0, "the tiles hold the S rows of a column as 16-byte vectors");
    constexpr int H = S / 2;    // 16-byte vectors per column of a tile
    constexpr int QB = NT / S;  // Philox blocks (quads of rows of T) per batch per sketch row
    constexpr int KB = 4 * QB;  // rows of T per batch
    extern __shared__ double lds[];
    // Xs: slot w holds X(i0 .. i0 + S - 1, :) of its column (slot c < C:
    // column c0 + c), Gs: row kl of the slice holds G(i0 .. i0 + S - 1,
    // kb + kl), each as H 16-byte vectors placed by tix.  W = C + the split
    // columns' slots (for every block).
    double2 *Xs = reinterpret_cast<double2 *>(lds);                      // [W][H]
    double2 *Gs = reinterpret_cast<double2 *>(lds + (size_t)S * W);      // [KB][H]
    double *Gd = lds + (size_t)S * W;
    const int tid = threadIdx.x;
    const int b = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * S;
    const int64_t c0 = (int64_t)b * C;
    const int cw = (int)min<int64_t>((int64_t)C, d - c0);
    // this workgroup's batches: [j0, j1) (the split over rows of T)
    const int64_t j0 = (int64_t)blockIdx.z * bpz, j1 = min<int64_t>(nbatch, j0 + bpz);
    for (int j = tid; j < S * W; j += NT) lds[j] = 0.0;
    const int gi = tid / QB, gq = tid % QB;
    const uint64_t grow = (uint64_t)min<int64_t>(i0 + gi, s - 1);
    // this thread's entries of batch j: [optr[g], optr[g + 1]), g = (b nbatch + j) NT + tid
    const int64_t *op = optr + ((int64_t)b * nbatch + j0) * NT + tid;
    int64_t lo = 0, hi = 0;
    if (j0 < j1) {
        lo = op[0];
        hi = op[1];
    }
    SkEntry pf[SK_PF] = {};
#pragma unroll
    for (int u = 0; u < SK_PF; ++u)
        if (lo + u < hi) pf[u] = ent[lo + u];
    auto apply = [&](const SkEntry &t, int64_t kb) {
        const int kl = (int)((int64_t)t.k - kb);
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const double2 g = Gs[tix<H>(kl, h)];
            const int xi = tix<H>(t.c, h);
            double2 x = Xs[xi];
            x.x += t.v * g.x;
            x.y += t.v * g.y;
            Xs[xi] = x;
        }
    };
    for (int64_t j = j0; j < j1; ++j) {
        const int64_t kb = j * KB;
        // next batch's range and first entries are loaded while this batch
        // generates its slice of G and applies its entries
        int64_t nlo = 0, nhi = 0;
        if (j + 1 < j1) {
            nlo = op[(j + 1 - j0) * NT];
            nhi = op[(j + 1 - j0) * NT + 1];
        }
        SkEntry cur[SK_PF];
#pragma unroll
        for (int u = 0; u < SK_PF; ++u) cur[u] = pf[u];
        double g[4];
        gauss4(seed, grow, (uint64_t)(kb / 4 + gq), g);
        __syncthreads();  // previous batch done with Gs
#pragma unroll
        for (int w = 0; w < 4; ++w) Gd[2 * tix<H>(4 * gq + w, gi >> 1) + (gi & 1)] = g[w];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SK_PF; ++u)
            if (nlo + u < nhi) pf[u] = ent[nlo + u];
#pragma unroll
        for (int u = 0; u < SK_PF; ++u)
            if (lo + u < hi) apply(cur[u], kb);
        for (int64_t e = lo + SK_PF; e < hi; ++e) apply(ent[e], kb);
        lo = nlo;
        hi = nhi;
    }
    __syncthreads();
    double *X = out + (int64_t)blockIdx.z * zstride;
    for (int j = tid; j < S * cw; j += NT) {
        const int c = j / S, i = j % S;
        const int p = nslot[c0 + c];
        double v = lds[2 * tix<H>(c, i >> 1) + (i & 1)];
        if (p > 1) {  // a split column: its slots in order
            const int w0 = C + sbase[c0 + c];
            for (int q = 0; q < p; ++q) v += lds[2 * tix<H>(w0 + q, i >> 1) + (i & 1)];
        }
        if (i0 + i < s) X[(c0 + c) * s + i0 + i] = v;
    }
}

// X = the sum of the nz partial sketches (one per range of rows of T), in
// range order.
__global__ void sum_partials_kernel(const double *__restrict__ part, int nz, int64_t n,
                                    double *__restrict__ X) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        double v = part[e];
        for (int z = 1; z < nz; ++z) v += part[(int64_t)z * n + e];
        X[e] = v;
    }
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 65535)); }

// blocks of 256 threads (4 wavefronts) for one wavefront per row
int grid_rows(int64_t rows) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(rows, 4), 65535)); }

void launch_expand_rows(int64_t nrows, const int64_t *ptr, int32_t *out, hipStream_t st) {
    expand_rows_kernel<<<grid_rows(nrows), 256, 0, st>>>(nrows, ptr, out);
    LSRN_HIP(hipGetLastError());
}

// Stable sort of (keys, values) by the low `bits` bits of the keys.
void sort_pairs(const uint32_t *kin, uint32_t *kout, const int32_t *vin, int32_t *vout, int64_t n,
                int bits, hipStream_t st) {
    size_t tb = 0;
    LSRN_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, kin, kout, vin, vout, (int)n, 0, bits, st));
    DevBuf tmp(std::max<size_t>(tb, 16));
    LSRN_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.as<void>(), tb, kin, kout, vin, vout, (int)n, 0,
                                                bits, st));
    LSRN_HIP(hipStreamSynchronize(st));  // before tmp is freed
}

int bits_for(int64_t maxkey) {
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) <= maxkey) ++b;
    return b;
}

}  // namespace

void make_sparse_view(SparseView &v, int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                      const int32_t *colind, const double *val, hipStream_t st) {
    LSRN_REQUIRE(m > 0 && n > 0 && nnz >= 0, "sizes must be positive");
    LSRN_REQUIRE(rowptr && (nnz == 0 || (colind && val)), "NULL pointer");
    LSRN_REQUIRE(nnz < ((int64_t)1 << 31) && m < ((int64_t)1 << 31) && n < ((int64_t)1 << 31),
                 "CSR input needs nnz, m, n < 2^31");
    // structure check before any kernel indexes with it
    int64_t ends[2] = {0, 0};
    LSRN_HIP(hipMemcpyAsync(&ends[0], rowptr, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    LSRN_HIP(hipMemcpyAsync(&ends[1], rowptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    LSRN_HIP(hipStreamSynchronize(st));
    LSRN_REQUIRE(ends[0] == 0 && ends[1] == nnz, "rowptr[0] must be 0 and rowptr[m] must be nnz");
    {
        DevBuf flag(sizeof(int));
        LSRN_HIP(hipMemsetAsync(flag.as<int>(), 0, sizeof(int), st));
        check_ptr_kernel<<<grid_for(m), 256, 0, st>>>(m, nnz, rowptr, flag.as<int>());
        if (nnz > 0) check_idx_kernel<<<grid_for(nnz), 256, 0, st>>>(nnz, n, colind, flag.as<int>());
        LSRN_HIP(hipGetLastError());
        int bad = 0;
        LSRN_HIP(hipMemcpyAsync(&bad, flag.as<int>(), sizeof(int), hipMemcpyDeviceToHost, st));
        LSRN_HIP(hipStreamSynchronize(st));
        LSRN_REQUIRE(!(bad & 1), "rowptr must be nondecreasing within [0, nnz]");
        LSRN_REQUIRE(!(bad & 2), "column index out of range");
    }
    v.tall = m >= n;
    v.K = v.tall ? m : n;
    v.d = v.tall ? n : m;
    v.nnz = nnz;
    const CsrMat a{m, n, nnz, rowptr, colind, val};
    // A^T, row-compressed: stable sort of the entries by column
    v.tptr.alloc((size_t)(n + 1) * sizeof(int64_t));
    v.tidx.alloc((size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t));
    v.tval.alloc((size_t)std::max<int64_t>(nnz, 1) * sizeof(double));
    const CsrMat at{n, m, nnz, v.tptr.as<int64_t>(), v.tidx.as<int32_t>(), v.tval.as<double>()};
    if (nnz > 0) {
        DevBuf rowof((size_t)nnz * 4), iota((size_t)nnz * 4), perm((size_t)nnz * 4), ksort((size_t)nnz * 4);
        launch_expand_rows(m, rowptr, rowof.as<int32_t>(), st);
        iota_kernel<<<grid_for(nnz), 256, 0, st>>>(nnz, iota.as<int32_t>());
        LSRN_HIP(hipGetLastError());
        sort_pairs(reinterpret_cast<const uint32_t *>(colind), ksort.as<uint32_t>(), iota.as<int32_t>(),
                   perm.as<int32_t>(), nnz, bits_for(n), st);
        bounds_kernel<<<grid_for(n + 1), 256, 0, st>>>(nnz, ksort.as<uint32_t>(), n, v.tptr.as<int64_t>());
        gather_transpose_kernel<<<grid_for(nnz), 256, 0, st>>>(nnz, perm.as<int32_t>(), rowof.as<int32_t>(),
                                                               val, v.tidx.as<int32_t>(), v.tval.as<double>());
        LSRN_HIP(hipGetLastError());
        LSRN_HIP(hipStreamSynchronize(st));  // before the temporaries are freed
    } else {
        LSRN_HIP(hipMemsetAsync(v.tptr.as<int64_t>(), 0, (size_t)(n + 1) * sizeof(int64_t), st));
    }
    v.rows = v.tall ? a : at;
    v.cols = v.tall ? at : a;
    // segments of the column pass (host table from the d + 1 offsets)
    {
        const int64_t d = v.cols.nrows;
        std::vector<int64_t> ptr((size_t)d + 1);
        LSRN_HIP(hipMemcpyAsync(ptr.data(), v.cols.ptr, (size_t)(d + 1) * sizeof(int64_t),
                                hipMemcpyDeviceToHost, st));
        LSRN_HIP(hipStreamSynchronize(st));
        std::vector<int32_t> rseg((size_t)d + 1), srow;
        srow.reserve((size_t)d + (size_t)(nnz / SparseView::kColSeg) + 1);
        for (int64_t j = 0; j < d; ++j) {
            rseg[(size_t)j] = (int32_t)srow.size();
            const int64_t len = ptr[(size_t)j + 1] - ptr[(size_t)j];
            const int64_t ns = std::max<int64_t>(1, ceil_div(len, SparseView::kColSeg));
            for (int64_t g = 0; g < ns; ++g) srow.push_back((int32_t)j);
        }
        rseg[(size_t)d] = (int32_t)srow.size();
        v.nseg = (int64_t)srow.size();
        v.seg_row.alloc(srow.size() * sizeof(int32_t));
        v.row_seg.alloc(rseg.size() * sizeof(int32_t));
        LSRN_HIP(hipMemcpyAsync(v.seg_row.as<int32_t>(), srow.data(), srow.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, st));
        LSRN_HIP(hipMemcpyAsync(v.row_seg.as<int32_t>(), rseg.data(), rseg.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, st));
        LSRN_HIP(hipStreamSynchronize(st));  // before the host tables go out of scope
    }
}

size_t sparse_view_bytes(int64_t m, int64_t n, int64_t nnz) {
    const int64_t d = std::min(m, n);
    const size_t seg = (size_t)(d + 1 + nnz / SparseView::kColSeg + d) * 4;
    return (size_t)(n + 1) * 8 + (size_t)nnz * 12 + (size_t)nnz * 16 + (size_t)nnz * 8 + seg;
}

// Split columns: column c of T with about e nonzeros per batch (of KB
// rows) gets P = the power of two >= e / 4 slots (P = 1: not split), as
// long as every block's extra slots fit in `room`; the largest columns are
// split first.  sbase[c] = first extra slot of c within its block.
int plan_split_columns(const SparseView &v, int C, int KB, int room, std::vector<int32_t> &sbase,
                       std::vector<int32_t> &nslot, hipStream_t st) {
    const int64_t d = v.d, K = v.K;
    std::vector<int64_t> ptr((size_t)d + 1);
    LSRN_HIP(hipMemcpyAsync(ptr.data(), v.cols.ptr, ((size_t)d + 1) * sizeof(int64_t),
                            hipMemcpyDeviceToHost, st));
    LSRN_HIP(hipStreamSynchronize(st));
    sbase.assign((size_t)d, 0);
    nslot.assign((size_t)d, 1);
    const int64_t nb = ceil_div(d, C);
    int most = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t c0 = b * C, c1 = std::min<int64_t>(d, c0 + C);
        std::vector<std::pair<double, int64_t>> heavy;
        for (int64_t c = c0; c < c1; ++c) {
            const double per_batch = (double)(ptr[(size_t)c + 1] - ptr[(size_t)c]) * KB / (double)K;
            if (per_batch > 8.0) heavy.emplace_back(per_batch, c);
        }
        std::sort(heavy.begin(), heavy.end(), [](const auto &x, const auto &y) {
            return x.first > y.first || (x.first == y.first && x.second < y.second);
        });
        int used = 0;
        for (const auto &h : heavy) {
            int p = 1;
            while (p < 256 && p * 4.0 < h.first) p *= 2;
            if (used + p > room) break;
            sbase[(size_t)h.second] = used;
            nslot[(size_t)h.second] = p;
            used += p;
        }
        most = std::max(most, used);
    }
    return most;
}

// Tile of the sparse sketch: S sketch rows x C columns of T per workgroup
// (plus the split columns' slots), nz ranges of batches of rows of T.
struct SkTile {
    int S = 4, NT = 1024, KB = sk_kb(4, 1024), C = 0, room = 0;
    int64_t nb = 1, nbatch = 1, nz = 1, bpz = 1;
};

// The workgroup reads all entries of its column block once per S sketch
// rows and generates its S rows of G over all K rows of T once per column
// block.  S = 8 (C = 2048, 512 threads) halves the entry reads of S = 4 at
// the same generation of G when T has at most 2048 columns; a wider T keeps
// S = 4, since narrower blocks would generate G once more per block, with
// 1024 threads (C = 3584), whose extra wavefronts hide the latency of the
// uneven per-thread work.  (Measured, one sketch: 4e6 x 1024 with 8.4e7
// nonzeros 327 / 228 / 472 ms for S = 4 / 8 / 16 at 512 threads, 266 ms for
// S = 8 at 1024; 2e6 x 2e4 with 4.2e7 nonzeros 3.41 / 5.21 / 10.6 s at 512
// threads, 2.93 s for S = 4 at 1024.)
SkTile choose_tile(int64_t K, int64_t d, int64_t nnz, int64_t s) {
    (void)nnz;
    SkTile t;
    t.S = d <= 2048 ? 8 : 4;
    t.NT = t.S == 8 ? 512 : 1024;
    t.KB = sk_kb(t.S, t.NT);
    const int wmax = SK_LDS / t.S - t.KB;               // tile slots within the LDS
    const int cmax = t.S == 8 ? 2048 : 3584;            // the rest: split columns' slots
    t.C = (int)std::min<int64_t>((int64_t)cmax, d);
    t.room = wmax - t.C;
    t.nb = ceil_div(d, t.C);
    t.nbatch = std::max<int64_t>(1, ceil_div(K, t.KB));
    // fill the chip: split the rows of T into ranges when there are fewer
    // tiles than CUs (one workgroup per CU fits in the LDS)
    const int64_t tiles = ceil_div(s, t.S) * t.nb;
    const int64_t cus = device_cus();
    t.nz = tiles >= cus ? 1 : std::min<int64_t>(t.nbatch, ceil_div(cus, tiles));
    t.bpz = ceil_div(t.nbatch, t.nz);
    t.nz = ceil_div(t.nbatch, t.bpz);
    return t;
}

// Device bytes of the sparse sketch's per-group offsets and partial sketches.
size_t sketch_csr_tile_bytes(int64_t K, int64_t d, int64_t nnz, int64_t s) {
    const SkTile t = choose_tile(K, d, nnz, s);
    size_t bytes = (size_t)(t.nb * t.nbatch * t.NT + 1) * sizeof(int64_t);
    if (t.nz > 1) bytes += (size_t)t.nz * (size_t)s * (size_t)d * sizeof(double);
    return bytes;
}

template <int S, int NT>
void launch_sketch(const SkTile &t, const SkEntry *ent, const int64_t *optr, int64_t K, int64_t d, int W,
                   int64_t s, uint64_t seed, const int32_t *sbase, const int32_t *nslot, double *out,
                   int64_t zstride, hipStream_t st) {
    // the dynamic-LDS limit (the most any call takes) is raised once per
    // process: solves on several host threads (the serving runtime's
    // workers) would otherwise set the attribute of the same kernel
    // concurrently
    static std::once_flag lds_once;
    std::call_once(lds_once, [] {
        LSRN_HIP(hipFuncSetAttribute((const void *)csr_sketch_kernel<S, NT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    });
    const size_t lds = sizeof(double) * ((size_t)S * W + (size_t)S * t.KB);
    dim3 grid((unsigned)ceil_div(s, S), (unsigned)t.nb, (unsigned)t.nz);
    csr_sketch_kernel<S, NT><<<grid, NT, lds, st>>>(ent, optr, K, d, t.C, W, t.nbatch, t.bpz, s,
                                                          seed, sbase, nslot, out, zstride);
    LSRN_HIP(hipGetLastError());
}

void sketch_csr(const SparseView &v, double lambda, int64_t s, uint64_t seed, double *X,
                hipStream_t st, double *kernel_ms) {
    const int64_t K = v.K, d = v.d, nnz = v.nnz;
    const SkTile tile = choose_tile(K, d, nnz, s);
    const int C = tile.C;
    const int64_t nb = tile.nb, nbatch = tile.nbatch;
    const int64_t ngroups = nb * nbatch * tile.NT;
    LSRN_REQUIRE(ngroups < ((int64_t)1 << 31), "sparse sketch: too many (column block, batch) groups");
    LSRN_REQUIRE(nb <= 65535, "sparse sketch: too many column blocks");
    std::vector<int32_t> sbase_h, nslot_h;
    const int extra = plan_split_columns(v, C, tile.KB, std::max(tile.room, 0), sbase_h, nslot_h, st);
    const int W = C + extra;
    DevBuf sbase((size_t)d * sizeof(int32_t)), nslot((size_t)d * sizeof(int32_t));
    LSRN_HIP(hipMemcpyAsync(sbase.as<int32_t>(), sbase_h.data(), (size_t)d * sizeof(int32_t),
                            hipMemcpyHostToDevice, st));
    LSRN_HIP(hipMemcpyAsync(nslot.as<int32_t>(), nslot_h.data(), (size_t)d * sizeof(int32_t),
                            hipMemcpyHostToDevice, st));
    DevBuf ent((size_t)std::max<int64_t>(nnz, 1) * sizeof(SkEntry));
    DevBuf optr((size_t)(ngroups + 1) * sizeof(int64_t));
    const CsrMat &t = v.rows;  // CSR(T)
    if (nnz > 0) {
        DevBuf rowof((size_t)nnz * 4), keys((size_t)nnz * 4), ksort((size_t)nnz * 4);
        DevBuf iota((size_t)nnz * 4), perm((size_t)nnz * 4);
        launch_expand_rows(t.nrows, t.ptr, rowof.as<int32_t>(), st);
        sketch_keys_kernel<<<grid_for(nnz), 256, 0, st>>>(nnz, t.idx, rowof.as<int32_t>(), C, tile.KB,
                                                          tile.NT, nbatch, sbase.as<int32_t>(), nslot.as<int32_t>(),
                                                          keys.as<uint32_t>());
        iota_kernel<<<grid_for(nnz), 256, 0, st>>>(nnz, iota.as<int32_t>());
        LSRN_HIP(hipGetLastError());
        sort_pairs(keys.as<uint32_t>(), ksort.as<uint32_t>(), iota.as<int32_t>(), perm.as<int32_t>(),
                   nnz, bits_for(ngroups), st);
        bounds_kernel<<<grid_for(ngroups + 1), 256, 0, st>>>(nnz, ksort.as<uint32_t>(), ngroups,
                                                             optr.as<int64_t>());
        gather_sketch_kernel<<<grid_for(nnz), 256, 0, st>>>(nnz, perm.as<int32_t>(), rowof.as<int32_t>(),
                                                            t.idx, t.val, C, sbase.as<int32_t>(),
                                                            nslot.as<int32_t>(), ent.as<SkEntry>());
        LSRN_HIP(hipGetLastError());
        LSRN_HIP(hipStreamSynchronize(st));
    } else {
        LSRN_HIP(hipMemsetAsync(optr.as<int64_t>(), 0, (size_t)(ngroups + 1) * sizeof(int64_t), st));
    }
    // partial sketches of the row ranges (one range: X itself)
    DevBuf part(tile.nz > 1 ? (size_t)tile.nz * (size_t)s * (size_t)d * sizeof(double) : 0);
    double *out = tile.nz > 1 ? part.as<double>() : X;
    const int64_t zstride = tile.nz > 1 ? s * d : 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (kernel_ms) {
        LSRN_HIP(hipEventCreate(&ev[0]));
        LSRN_HIP(hipEventCreate(&ev[1]));
        LSRN_HIP(hipEventRecord(ev[0], st));
    }
    const SkEntry *e = ent.as<SkEntry>();
    const int64_t *o = optr.as<int64_t>();
    if (tile.S == 4)
        launch_sketch<4, 1024>(tile, e, o, K, d, W, s, seed, sbase.as<int32_t>(), nslot.as<int32_t>(), out, zstride,
                               st);
    else
        launch_sketch<8, 512>(tile, e, o, K, d, W, s, seed, sbase.as<int32_t>(), nslot.as<int32_t>(), out, zstride,
                              st);
    if (tile.nz > 1) {
        sum_partials_kernel<<<grid_for(s * d), 256, 0, st>>>(out, (int)tile.nz, s * d, X);
        LSRN_HIP(hipGetLastError());
    }
    if (kernel_ms) {
        LSRN_HIP(hipEventRecord(ev[1], st));
        LSRN_HIP(hipEventSynchronize(ev[1]));
        float ms = 0.f;
        LSRN_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        *kernel_ms = ms;
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
    }
    add_identity_rows(K, d, s, lambda, seed, X, st);
    LSRN_HIP(hipStreamSynchronize(st));  // before ent / optr / part are freed
}

}  // namespace lsrn
