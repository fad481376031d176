// iterate.hip -- the iteration phase of LSRN (Alg. 1/2 step 6-7).
//
// Both shapes are driven through one "row sweep" over a row-major matrix T
// (the tall view): T = A for m >= n (Alg. 1) and T = A^T, i.e. A stored
// column-major, for m < n (Alg. 2).  One sweep reads every row T_j once:
//     q_j = T_j . w                 (w = N v or M u, computed beforehand)
//     c_j = op(q_j, per-row state)  (the LSQR / Chebyshev update of row j)
//     z  += c_j T_j                 (the transposed product)
// so A (x) and A^T (y) of an iteration cost one pass over A in HBM.
// Partial z vectors per workgroup are summed in a fixed order, which makes
// every result bitwise reproducible run to run.
//
// Tall LSQR runs Paige-Saunders LSQR on K = [A; lambda I] N: the long
// vector u lives in row space and is kept unnormalised (u~ = beta u), the
// short vectors v, w, y (length r) and all scalars live in one device
// workgroup.  Fat LSQR runs on K = M^T A: the long vectors v, w, x live in
// row space of T, and the x/w update of iteration i is applied during the
// sweep of iteration i+1, when v_{i+1} is read anyway.  The Chebyshev
// semi-iteration (Alg. 3) has data-independent scalars, computed on the
// host.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <limits>
#include <type_traits>
#include <vector>

#include "internal.hpp"

namespace lsrn {

namespace {

constexpr int NT = 256;

// Device-resident scalar state of an iterative solve.
struct State {
    double alpha, beta, rhobar, phibar, anorm2, bnorm;
    double coef;        // tall LSQR: u~_new = q - coef u~
    double inv_alpha;   // fat LSQR: v = v~ * inv_alpha
    double phi_rho, theta_rho;
    double xnorm2;
    double acc[4];      // reduced sweep accumulators
    double cg_rs, cg_stop;
    int32_t done, iters, converged, pending;
    int32_t maxiter, pad_;
};

enum Op : int {
    OP_ATB = 0,        // c = y[j]                       acc0 += c^2
    OP_LSQR_TALL = 1,  // y[j] = q - coef y[j]; c = y[j]  acc0 += c^2
    OP_CS_TALL = 2,    // y[j] -= alpha q;    c = y[j]    acc0 += c^2
    OP_NORMAL = 3,     // c = q                          acc0 += q^2
    OP_LSQR_FAT = 4,   // see sweep body
    OP_CS_FAT = 5,     // y[j] = beta y[j] + q; x[j] += alpha y[j]; c = y[j]
};

struct SweepArgs {
    const double *T;
    const float *T32;    // FP32 copy of T (precision form), read when F32
    int64_t ldt, rows;
    int L;
    int nblocks;
    int64_t rows_per_block;
    const double *w;     // length L
    double *zpart;       // nblocks x L
    double *spart;       // nblocks x 4
    double *y;           // per-row long vector (length rows, + L Tikhonov rows)
    double *xv, *wv;     // fat LSQR / CS long vectors (length rows)
    State *st;
    double lambda;       // Tikhonov rows (tall only)
    double alpha, beta;  // Chebyshev scalars
};

template <int CPT>
__device__ __forceinline__ int col_of(int tid, int e) {
    return 2 * tid + 512 * (e >> 1) + (e & 1);
}

// Column of element e of a thread when each thread holds groups of W
// consecutive columns (W = 2: double2 loads, W = 4: float4 loads).
template <int W>
__device__ __forceinline__ int col_of_w(int tid, int e) {
    return W * tid + (NT * W) * (e / W) + (e % W);
}

template <int CPT, int R, int OP, bool F32>
__device__ __forceinline__ void sweep_body(const SweepArgs &a, const int block) {
    // FP32 rows load as float4 (16 bytes a lane, like the FP64 double2)
    constexpr int W = (F32 && CPT >= 4) ? 4 : 2;
    if (a.st->done) return;
    __shared__ double red[2][NT / 64][R];
    __shared__ double accred[NT / 64][4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int L = a.L;

    double wr[CPT], zr[CPT];
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int col = col_of_w<W>(tid, e);
        wr[e] = (OP != OP_ATB && col < L) ? a.w[col] : 0.0;
        zr[e] = 0.0;
    }
    // scalars of this sweep
    double coef = 0.0, inv_alpha = 0.0, beta = 0.0, phi_rho = 0.0, theta_rho = 0.0;
    int pending = 0;
    if (OP == OP_LSQR_TALL) coef = a.st->coef;
    if (OP == OP_CS_TALL) coef = a.alpha;
    if (OP == OP_LSQR_FAT) {
        inv_alpha = a.st->inv_alpha;
        beta = a.st->beta;
        phi_rho = a.st->phi_rho;
        theta_rho = a.st->theta_rho;
        pending = a.st->pending;
    }
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;

    const int64_t r0 = (int64_t)block * a.rows_per_block;
    const int64_t r1 = min(a.rows, r0 + a.rows_per_block);
    // rows are loaded W columns a lane at a time when the rows are aligned
    // for it, element by element otherwise
    const bool vec = F32 ? (((a.ldt & (W - 1)) == 0) &&
                            ((reinterpret_cast<uintptr_t>(a.T32) & (4 * W - 1)) == 0))
                         : (((a.ldt & 1) == 0) && ((reinterpret_cast<uintptr_t>(a.T) & 15) == 0));
    // FP32 storage stays FP32 in registers (half the registers per byte in
    // flight) and is widened where it is used
    using E = std::conditional_t<F32, float, double>;
    const E *tbase;
    if constexpr (F32) tbase = a.T32;
    else tbase = a.T;
    // the per-row vector of this block (loads past r1 return 0)
    const __amdgpu_buffer_rsrc_t rsy = __builtin_amdgcn_make_buffer_rsrc(
        a.y + (r0 < r1 ? r0 : 0), (short)0, (int)(r0 < r1 ? (r1 - r0) * 8 : 0), 0x00020000);
    // the fat forms' x (and LSQR's w) of this block's rows, read by thread
    // rr < R for row j0 + rr (the row it owns in the update) before the
    // next rows are requested, so that the owner's update waits for none
    // of the rows in flight
    constexpr bool FATX = OP == OP_LSQR_FAT || OP == OP_CS_FAT, FATW = OP == OP_LSQR_FAT;
    auto row_rsrc = [&](double *v, bool used) {
        const bool ok = used && v != nullptr && r0 < r1;
        return __builtin_amdgcn_make_buffer_rsrc(ok ? v + r0 : a.y, (short)0,
                                                 (int)(ok ? (r1 - r0) * 8 : 0), 0x00020000);
    };
    const __amdgpu_buffer_rsrc_t rsx = row_rsrc(a.xv, FATX), rsw = row_rsrc(a.wv, FATW);
    auto sweep_rows = [&](auto vec_c) {
    constexpr bool VEC = decltype(vec_c)::value;
    // R rows of T (and of the per-row vector) starting at j0 into registers.
    // Each row is read through a raw buffer resource of L elements (none
    // for rows >= r1): the hardware range check, per dword, returns 0 for
    // the columns >= L of a lane's vector and for whole rows past the
    // block, so no load carries a per-lane guard.  (Per-lane guards split
    // every load into a vector and a scalar path writing the same
    // registers, and the compiler then waited for all loads in flight,
    // the prefetched rows included, before each of them.)
    auto load_rows = [&](int64_t j0, E (&av)[R][CPT], double (&yv)[R]) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int64_t row = j0 + rr;
            const bool valid = row < r1;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<E *>(tbase + (valid ? row : 0) * a.ldt), (short)0,
                valid ? L * (int)sizeof(E) : 0, 0x00020000);
            if constexpr (VEC && W * sizeof(E) == 16) {
                typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
                for (int e = 0; e < CPT; e += W) {
                    const int col = col_of_w<W>(tid, e);
                    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, col * (int)sizeof(E), 0, 0);
                    if constexpr (F32) {
                        const float4 f = __builtin_bit_cast(float4, v);
                        av[rr][e] = f.x;
                        av[rr][e + 1] = f.y;
                        av[rr][e + 2] = f.z;
                        av[rr][e + 3] = f.w;
                    } else {
                        const double2 f = __builtin_bit_cast(double2, v);
                        av[rr][e] = f.x;
                        av[rr][e + 1] = f.y;
                    }
                }
            } else if constexpr (VEC) {  // FP32 pairs
#pragma unroll
                for (int e = 0; e < CPT; e += W) {
                    const int col = col_of_w<W>(tid, e);
                    const float2 f = __builtin_bit_cast(
                        float2, __builtin_amdgcn_raw_buffer_load_b64(rs, col * 4, 0, 0));
                    av[rr][e] = f.x;
                    av[rr][e + 1] = f.y;
                }
            } else {
#pragma unroll
                for (int e = 0; e < CPT; ++e) {
                    const int col = col_of_w<W>(tid, e);
                    if constexpr (F32)
                        av[rr][e] = __builtin_bit_cast(
                            float, __builtin_amdgcn_raw_buffer_load_b32(rs, col * 4, 0, 0));
                    else
                        av[rr][e] = __builtin_bit_cast(
                            double, __builtin_amdgcn_raw_buffer_load_b64(rs, col * 8, 0, 0));
                }
            }
            if constexpr (OP != OP_NORMAL)
                yv[rr] = __builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(rsy, (int)(row - r0) * 8, 0, 0));
            else
                yv[rr] = 0.0;
        }
    };
    // software pipeline: the loads of the next DEPTH steps are in flight
    // while step k reduces and updates (two steps ahead where the register
    // budget allows it; FP32 rows take half the registers, so the FP32 form
    // keeps as many bytes in flight as the FP64 one).  Rows past the block
    // load as zeros and are never used.
    constexpr int DEPTH = (F32 ? CPT * R / 2 : CPT * R) <= 16 ? 2 : 1;
    E avn[R][CPT], avm[R][CPT];
    double yvn[R], yvm[R];
    load_rows(r0, avn, yvn);
    if (DEPTH == 2) load_rows(r0 + R, avm, yvm);
    int parity = 0;
    for (int64_t j0 = r0; j0 < r1; j0 += R) {
        E av[R][CPT];
        double yv[R];
        const int own = (int)(j0 - r0) + (tid < R ? tid : 0);
        const double xo_own =
            FATX ? __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rsx, own * 8, 0, 0)) : 0.0;
        const double wo_own =
            FATW ? __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rsw, own * 8, 0, 0)) : 0.0;
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            yv[rr] = yvn[rr];
            if (DEPTH == 2) yvn[rr] = yvm[rr];
#pragma unroll
            for (int e = 0; e < CPT; ++e) {
                av[rr][e] = avn[rr][e];
                if (DEPTH == 2) avn[rr][e] = avm[rr][e];
            }
        }
        if (DEPTH == 2) load_rows(j0 + 2 * R, avm, yvm);
        else load_rows(j0 + R, avn, yvn);
        double q[R];
        if (OP != OP_ATB) {
            double pd[R];
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                double t = 0.0;
#pragma unroll
                for (int e = 0; e < CPT; ++e) t += (double)av[rr][e] * wr[e];
                pd[rr] = wave_sum(t);
            }
            if (lane == 0) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr) red[parity][wid][rr] = pd[rr];
            }
            __syncthreads();
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) t += red[parity][w][rr];
                q[rr] = t;
            }
            parity ^= 1;
        }
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int64_t row = j0 + rr;
            if (row >= r1) continue;
            const bool owner = tid == rr;
            double c;
            if (OP == OP_ATB) {
                c = yv[rr];
                if (owner) acc0 += c * c;
            } else if (OP == OP_LSQR_TALL) {
                c = q[rr] - coef * yv[rr];
                if (owner) { a.y[row] = c; acc0 += c * c; }
            } else if (OP == OP_CS_TALL) {
                c = yv[rr] - coef * q[rr];
                if (owner) { a.y[row] = c; acc0 += c * c; }
            } else if (OP == OP_NORMAL) {
                c = q[rr];
                if (owner) acc0 += c * c;
            } else if (OP == OP_LSQR_FAT) {
                const double v = yv[rr] * inv_alpha;
                c = q[rr] - beta * v;
                if (owner) {
                    if (pending == 1) {
                        a.wv[row] = v;
                        acc3 += v * v;
                    } else if (pending == 2) {
                        const double xo = xo_own + phi_rho * wo_own;
                        const double wn = v - theta_rho * wo_own;
                        a.xv[row] = xo;
                        a.wv[row] = wn;
                        acc1 += xo * xo;
                        acc2 += xo * wn;
                        acc3 += wn * wn;
                    }
                    a.y[row] = c;
                    acc0 += c * c;
                }
            } else {  // OP_CS_FAT
                c = a.beta * yv[rr] + q[rr];
                if (owner) {
                    a.y[row] = c;
                    a.xv[row] = xo_own + a.alpha * c;
                    acc0 += c * c;
                }
            }
#pragma unroll
            for (int e = 0; e < CPT; ++e) zr[e] += c * (double)av[rr][e];
        }
    }

    };
    if (vec) sweep_rows(std::true_type{});
    else sweep_rows(std::false_type{});

    // Tikhonov rows K + k (row vector lambda e_k) of the augmented tall view
    // ([A; lambda I_n], or [A^T; lambda I_m] for the under-determined form
    // [A, lambda I_m]): handled by the thread that owns column k, in block
    // k % nblocks, with the same row-local update as a row of T.
    if (a.lambda > 0.0) {
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int col = col_of_w<W>(tid, e);
            if (col < L && (col % a.nblocks) == block) {
                const int64_t row = a.rows + col;
                const double qv = a.lambda * wr[e];
                double c;
                if (OP == OP_ATB) c = a.y[row];
                else if (OP == OP_LSQR_TALL) { c = qv - coef * a.y[row]; a.y[row] = c; }
                else if (OP == OP_CS_TALL) { c = a.y[row] - coef * qv; a.y[row] = c; }
                else if (OP == OP_NORMAL) c = qv;
                else if (OP == OP_LSQR_FAT) {
                    const double v = a.y[row] * inv_alpha;
                    c = qv - beta * v;
                    if (pending == 1) {
                        a.wv[row] = v;
                        acc3 += v * v;
                    } else if (pending == 2) {
                        const double wo = a.wv[row];
                        const double xo = a.xv[row] + phi_rho * wo;
                        const double wn = v - theta_rho * wo;
                        a.xv[row] = xo;
                        a.wv[row] = wn;
                        acc1 += xo * xo;
                        acc2 += xo * wn;
                        acc3 += wn * wn;
                    }
                    a.y[row] = c;
                } else {  // OP_CS_FAT
                    c = a.beta * a.y[row] + qv;
                    a.y[row] = c;
                    a.xv[row] += a.alpha * c;
                }
                acc0 += c * c;
                zr[e] += a.lambda * c;
            }
        }
    }

#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int col = col_of_w<W>(tid, e);
        if (col < L) a.zpart[(int64_t)block * L + col] = zr[e];
    }
    acc0 = wave_sum(acc0);
    acc1 = wave_sum(acc1);
    acc2 = wave_sum(acc2);
    acc3 = wave_sum(acc3);
    if (lane == 0) {
        accred[wid][0] = acc0; accred[wid][1] = acc1; accred[wid][2] = acc2; accred[wid][3] = acc3;
    }
    __syncthreads();
    if (tid < 4) {
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += accred[w][tid];
        a.spart[(int64_t)block * 4 + tid] = t;
    }
}

template <int CPT, int R, int OP, bool F32>
__global__ void __launch_bounds__(NT, 2) sweep_kernel(SweepArgs a) {
    sweep_body<CPT, R, OP, F32>(a, (int)blockIdx.x);
}

// The sweep for narrow rows (L <= 8 LPR): LPR lanes share a row, each
// holding 8 of its columns (pairs interleaved by LPR), so a wavefront
// works on 64 / LPR rows at a time with no barrier inside the loop; the
// row products reduce over the LPR lanes of a row, the z partials first
// over the lanes of a column slot, then over the wavefronts.  T and the
// per-row vector are read through buffer resources (zeros past the
// problem); the columns >= L are zeroed by a select.  Tall FP64 ops
// without Tikhonov rows.  The problem's rows * ldt doubles must span less
// than 2^31 bytes.  `zred` holds NT / 64 x 64 x 8 doubles.
template <int LPR, int OP>
__device__ __forceinline__ void sweep_narrow_body(const SweepArgs &a, const int block,
                                                  double *__restrict__ zred,
                                                  double *__restrict__ accred) {
    static_assert(OP == OP_ATB || OP == OP_LSQR_TALL || OP == OP_CS_TALL || OP == OP_NORMAL,
                  "tall sweeps");
    constexpr int CPT = 8, RPW = 64 / LPR, NW = NT / 64, STEP = NW * RPW;
    if (a.st->done) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int sl = lane % LPR, rw = lane / LPR;
    const int L = a.L;
    double wr[CPT], zr[CPT];
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int col = 2 * sl + 2 * LPR * (e >> 1) + (e & 1);
        wr[e] = (OP != OP_ATB && col < L) ? a.w[col] : 0.0;
        zr[e] = 0.0;
    }
    const double coef = OP == OP_LSQR_TALL ? a.st->coef : (OP == OP_CS_TALL ? a.alpha : 0.0);
    const int64_t r0 = (int64_t)block * a.rows_per_block;
    const int64_t r1 = min(a.rows, r0 + a.rows_per_block);
    const __amdgpu_buffer_rsrc_t rt = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double *>(a.T), (short)0, (int)(a.rows * a.ldt * (int64_t)sizeof(double)), 0x00020000);
    const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(
        a.y, (short)0, (int)(r1 * (int64_t)sizeof(double)), 0x00020000);
    auto load = [&](int64_t j0, double (&av)[CPT], double &yv) {
        const int64_t row = j0 + wid * RPW + rw;
        const int base = (int)(row * a.ldt) * 8;
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int col = 2 * sl + 2 * LPR * (e >> 1) + (e & 1);
            const double v = __builtin_bit_cast(
                double, __builtin_amdgcn_raw_buffer_load_b64(rt, base + col * 8, 0, 0));
            av[e] = col < L ? v : 0.0;
        }
        yv = OP == OP_NORMAL ? 0.0
                             : __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(ry, (int)row * 8, 0, 0));
    };
    double avn[CPT], yvn;
    load(r0, avn, yvn);
    double acc0 = 0.0;
    for (int64_t j0 = r0; j0 < r1; j0 += STEP) {
        double av[CPT];
#pragma unroll
        for (int e = 0; e < CPT; ++e) av[e] = avn[e];
        const double yv = yvn;
        load(j0 + STEP, avn, yvn);
        const int64_t row = j0 + wid * RPW + rw;
        const bool valid = row < r1;
        double t = 0.0;
#pragma unroll
        for (int e = 0; e < CPT; ++e) t += av[e] * wr[e];
#pragma unroll
        for (int o = 1; o < LPR; o <<= 1) t += __shfl_xor(t, o, 64);
        double c;
        if (OP == OP_ATB) c = yv;
        else if (OP == OP_LSQR_TALL) c = t - coef * yv;
        else if (OP == OP_CS_TALL) c = yv - coef * t;
        else c = t;
        c = valid ? c : 0.0;
        if (sl == 0 && valid) {
            if (OP == OP_LSQR_TALL || OP == OP_CS_TALL) a.y[row] = c;
            acc0 += c * c;
        }
#pragma unroll
        for (int e = 0; e < CPT; ++e) zr[e] += c * av[e];
    }
#pragma unroll
    for (int e = 0; e < CPT; ++e)
#pragma unroll
        for (int o = LPR; o < 64; o <<= 1) zr[e] += __shfl_xor(zr[e], o, 64);
    if (rw == 0) {
#pragma unroll
        for (int e = 0; e < CPT; ++e) zred[(wid * 64 + sl) * CPT + e] = zr[e];
    }
    acc0 = wave_sum(acc0);
    if (lane == 0) accred[wid] = acc0;
    __syncthreads();
    if (wid == 0 && lane < LPR) {
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int col = 2 * lane + 2 * LPR * (e >> 1) + (e & 1);
            if (col < L) {
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) t += zred[(w * 64 + lane) * CPT + e];
                a.zpart[(int64_t)block * L + col] = t;
            }
        }
    }
    if (tid < 4) {
        double t = 0.0;
        if (tid == 0)
#pragma unroll
            for (int w = 0; w < NW; ++w) t += accred[w];
        a.spart[(int64_t)block * 4 + tid] = t;
    }
}

template <int LPR, int OP>
__global__ void __launch_bounds__(NT, 2) sweep_narrow_kernel(SweepArgs a) {
    __shared__ double zred[(NT / 64) * 64 * 8];
    __shared__ double accred[NT / 64];
    sweep_narrow_body<LPR, OP>(a, (int)blockIdx.x, zred, accred);
}


// Stage 1 of the partial-sum reduction: group g of the workgroup partials
// (rows [g*chunk, (g+1)*chunk) of zpart) summed per column.
__global__ void __launch_bounds__(256)
reduce_stage1_kernel(const double *__restrict__ zpart, const double *__restrict__ spart, int nb,
                     int L, int chunk, double *__restrict__ zred, double *__restrict__ sred,
                     const State *st) {
    if (st->done) return;
    const int g = blockIdx.y;
    const int b0 = g * chunk, b1 = min(nb, b0 + chunk);
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col < L) {
        double t = 0.0;
        for (int b = b0; b < b1; ++b) t += zpart[(int64_t)b * L + col];
        zred[(int64_t)g * L + col] = t;
    }
    if (blockIdx.x == 0 && threadIdx.x < 4) {
        double t = 0.0;
        for (int b = b0; b < b1; ++b) t += spart[b * 4 + threadIdx.x];
        sred[g * 4 + threadIdx.x] = t;
    }
}

// Stage 2: z = sum of the group sums; block 0 also reduces the scalar
// accumulators into st->acc.
__global__ void __launch_bounds__(256)
reduce_stage2_kernel(const double *__restrict__ zred, const double *__restrict__ sred, int ng,
                     int L, double *__restrict__ z, State *st) {
    if (st->done) return;
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col < L) {
        double t = 0.0;
        for (int g = 0; g < ng; ++g) t += zred[(int64_t)g * L + col];
        z[col] = t;
    }
    if (blockIdx.x == 0 && threadIdx.x < 4) {
        double t = 0.0;
        for (int g = 0; g < ng; ++g) t += sred[g * 4 + threadIdx.x];
        st->acc[threadIdx.x] = t;
    }
}

// y = M x for row-major M (nrows x ncols, leading dimension ld), one
// wavefront per row.
__global__ void __launch_bounds__(256)
gemv_kernel(const double *__restrict__ M, int64_t ld, int64_t nrows, int64_t ncols,
            const double *__restrict__ x, double *__restrict__ y, const State *st) {
    if (st && st->done) return;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= nrows) return;
    const int lane = threadIdx.x & 63;
    // the row and x through buffer resources of ncols entries: eight loads
    // of each in flight per lane, zeros past the end, and lane l still sums
    // its columns l, l + 64, ... in ascending order
    const int nbytes = (int)(ncols * (int64_t)sizeof(double));
    const __amdgpu_buffer_rsrc_t rm = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double *>(M + row * ld), (short)0, nbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double *>(x), (short)0, nbytes, 0x00020000);
    double t = 0.0;
    for (int64_t c0 = 0; c0 < ncols; c0 += 512) {
        double a[8], b[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int off = (int)(c0 + lane + 64 * k) * 8;
            a[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rm, off, 0, 0));
            b[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rx, off, 0, 0));
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) t += a[k] * b[k];
    }
    t = wave_sum(t);
    if (lane == 0) y[row] = t;
}

// ----------------------------------------------------------- LSQR scalars

constexpr int SNT = 1024;

// Block sum of a length-n vector held in global memory (fixed order).
__device__ double vec_dot(const double *a, const double *b, int64_t n, double *scratch) {
    double t = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += SNT) t += a[i] * b[i];
    return block_sum<SNT>(t, scratch);
}

// Tall LSQR start: t = K^T b^ (unscaled, from the first sweep), acc0 = ||b^||^2.
__device__ __forceinline__ void lsqr_tall_init_body(const double *__restrict__ t, int64_t r,
                                                    double *__restrict__ v, double *__restrict__ wdir,
                                                    double *__restrict__ y, State *st) {
    __shared__ double scratch[SNT / 64];
    const double beta = sqrt(st->acc[0]);
    const double ib = beta > 0.0 ? 1.0 / beta : 0.0;
    double part = 0.0;
    for (int64_t i = threadIdx.x; i < r; i += SNT) {
        const double vi = t[i] * ib;
        part += vi * vi;
    }
    const double alpha = sqrt(block_sum<SNT>(part, scratch));
    const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
    for (int64_t i = threadIdx.x; i < r; i += SNT) {
        const double vi = t[i] * ib * ia;
        v[i] = vi;
        wdir[i] = vi;
        y[i] = 0.0;
    }
    if (threadIdx.x == 0) {
        st->alpha = alpha;
        st->beta = beta;
        st->bnorm = beta;
        st->phibar = beta;
        st->rhobar = alpha;
        st->anorm2 = 0.0;
        st->xnorm2 = 0.0;
        st->coef = beta > 0.0 ? alpha / beta : 0.0;
        st->iters = 0;
        st->converged = (beta == 0.0 || alpha == 0.0) ? 1 : 0;
        st->done = st->converged;
    }
}

__global__ void __launch_bounds__(SNT)
lsqr_tall_init_kernel(const double *__restrict__ t, int64_t r, double *__restrict__ v,
                      double *__restrict__ wdir, double *__restrict__ y, State *st) {
    lsqr_tall_init_body(t, r, v, wdir, y, st);
}

// One LSQR iteration given t = N^T A^T u~ and acc0 = ||u~||^2 from the sweep
// that formed u~ = K v - alpha u.  Stopping rules of Paige-Saunders.
__device__ __forceinline__ void lsqr_tall_step_body(const double *__restrict__ t, int64_t r,
                                                    double *__restrict__ v, double *__restrict__ wdir,
                                                    double *__restrict__ y, double tol, State *st) {
    if (st->done) return;
    __shared__ double scratch[SNT / 64];
    const double alpha_old = st->alpha;
    const double beta = sqrt(st->acc[0]);
    const double anorm2 = st->anorm2 + alpha_old * alpha_old + beta * beta;
    const double ib = beta > 0.0 ? 1.0 / beta : 0.0;
    // alpha v = K^T u - beta v, u = u~ / beta
    double part = 0.0;
    for (int64_t i = threadIdx.x; i < r; i += SNT) {
        const double vi = t[i] * ib - beta * v[i];
        part += vi * vi;
    }
    const double alpha = sqrt(block_sum<SNT>(part, scratch));
    const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
    const double rho = hypot(st->rhobar, beta);
    const double c = st->rhobar / rho, sn = beta / rho;
    const double theta = sn * alpha;
    const double phi = c * st->phibar;
    const double phibar = sn * st->phibar;
    const double f1 = phi / rho, f2 = theta / rho;
    double xpart = 0.0;
    for (int64_t i = threadIdx.x; i < r; i += SNT) {
        const double vi = (t[i] * ib - beta * v[i]) * ia;
        const double yi = y[i] + f1 * wdir[i];
        y[i] = yi;
        wdir[i] = vi - f2 * wdir[i];
        v[i] = vi;
        xpart += yi * yi;
    }
    const double xnorm = sqrt(block_sum<SNT>(xpart, scratch));
    if (threadIdx.x == 0) {
        const double anorm = sqrt(anorm2);
        const double rnorm = phibar;
        const double arnorm = phibar * alpha * fabs(c);
        const double test2 = rnorm > 0.0 ? arnorm / (anorm * rnorm) : 0.0;
        const double test1 = rnorm / st->bnorm;
        const int it = st->iters + 1;
        st->iters = it;
        st->alpha = alpha;
        st->beta = beta;
        st->anorm2 = anorm2;
        st->rhobar = -c * alpha;
        st->phibar = phibar;
        st->coef = beta > 0.0 ? alpha / beta : 0.0;
        const bool conv = test2 <= tol || test1 <= tol + tol * anorm * xnorm / st->bnorm ||
                          beta == 0.0 || alpha == 0.0;
        st->converged = conv ? 1 : 0;
        st->done = (conv || it >= st->maxiter) ? 1 : 0;
    }
}

__global__ void __launch_bounds__(SNT)
lsqr_tall_step_kernel(const double *__restrict__ t, int64_t r, double *__restrict__ v,
                      double *__restrict__ wdir, double *__restrict__ y, double tol, State *st) {
    lsqr_tall_step_body(t, r, v, wdir, y, tol, st);
}

// Fat LSQR start: c = M^T b in t (length r); u = c / beta.
__global__ void __launch_bounds__(SNT)
lsqr_fat_init_kernel(const double *__restrict__ t, int64_t r, double *__restrict__ u, State *st) {
    __shared__ double scratch[SNT / 64];
    const double beta = sqrt(vec_dot(t, t, r, scratch));
    const double ib = beta > 0.0 ? 1.0 / beta : 0.0;
    for (int64_t i = threadIdx.x; i < r; i += SNT) u[i] = t[i] * ib;
    if (threadIdx.x == 0) {
        st->beta = beta;
        st->bnorm = beta;
        st->phibar = beta;
        st->anorm2 = 0.0;
        st->xnorm2 = 0.0;
        st->inv_alpha = 0.0;
        st->pending = 0;
        st->iters = 0;
        st->alpha = 0.0;
        st->converged = beta == 0.0 ? 1 : 0;
        st->done = st->converged;
    }
}

// Fat LSQR after a sweep that produced v~_{i+1} (acc0 = ||v~||^2, acc1..3 =
// ||x_{i-1}||^2, x_{i-1}.w_i, ||w_i||^2) and t = M^T A v~.  first: the sweep
// was the start sweep (v~_1).  Then: Givens step of iteration i and the
// stopping test, followed by the u-step of iteration i+1.
__global__ void __launch_bounds__(SNT)
lsqr_fat_step_kernel(const double *__restrict__ t, int64_t r, double *__restrict__ u, int first,
                     double tol, State *st) {
    if (st->done) return;
    __shared__ double scratch[SNT / 64];
    __shared__ int stop;
    const double alpha = sqrt(st->acc[0]);
    if (threadIdx.x == 0) {
        stop = 0;
        if (first) {
            st->rhobar = alpha;
            st->alpha = alpha;
            st->pending = 1;
            if (alpha == 0.0) { st->converged = 1; st->done = 1; st->pending = 0; stop = 1; }
        } else {
            const double beta = st->beta;  // beta_{i+1}
            const double rho = hypot(st->rhobar, beta);
            const double c = st->rhobar / rho, sn = beta / rho;
            const double theta = sn * alpha;
            const double phi = c * st->phibar;
            const double phibar = sn * st->phibar;
            const double pr = phi / rho;
            st->phi_rho = pr;
            st->theta_rho = theta / rho;
            st->pending = 2;
            const double xnorm2 = st->acc[1] + 2.0 * pr * st->acc[2] + pr * pr * st->acc[3];
            st->xnorm2 = xnorm2;
            st->rhobar = -c * alpha;
            st->phibar = phibar;
            st->alpha = alpha;
            const double anorm = sqrt(st->anorm2);
            const double rnorm = phibar;
            const double arnorm = phibar * alpha * fabs(c);
            const double test2 = rnorm > 0.0 ? arnorm / (anorm * rnorm) : 0.0;
            const double test1 = rnorm / st->bnorm;
            const int it = st->iters + 1;
            st->iters = it;
            const bool conv = test2 <= tol ||
                              test1 <= tol + tol * anorm * sqrt(xnorm2) / st->bnorm ||
                              beta == 0.0 || alpha == 0.0;
            st->converged = conv ? 1 : 0;
            if (conv || it >= st->maxiter) { st->done = 1; stop = 1; }
        }
    }
    __syncthreads();
    if (stop) return;
    // u-step: beta u = K v - alpha u, K v = t / alpha
    const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
    double part = 0.0;
    for (int64_t i = threadIdx.x; i < r; i += SNT) {
        const double ui = t[i] * ia - alpha * u[i];
        part += ui * ui;
    }
    const double beta = sqrt(block_sum<SNT>(part, scratch));
    const double ib = beta > 0.0 ? 1.0 / beta : 0.0;
    for (int64_t i = threadIdx.x; i < r; i += SNT) u[i] = (t[i] * ia - alpha * u[i]) * ib;
    if (threadIdx.x == 0) {
        st->anorm2 += alpha * alpha + beta * beta;
        st->beta = beta;
        st->inv_alpha = ia;
    }
}

// x += phi/rho w after the last fat LSQR iteration.
__global__ void __launch_bounds__(256)
lsqr_fat_finish_kernel(int64_t n, double *__restrict__ x, const double *__restrict__ wdir,
                       const State *st) {
    if (st->pending != 2) return;
    const double pr = st->phi_rho;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] += pr * wdir[i];
}

// ------------------------------------------------------ Chebyshev / misc

// v = beta v + t; y += alpha v (short vectors of the tall Chebyshev solve).
__global__ void __launch_bounds__(256)
cs_short_kernel(int64_t r, double *__restrict__ v, const double *__restrict__ t,
                double *__restrict__ y, double alpha, double beta) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < r;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double vi = beta * v[i] + t[i];
        v[i] = vi;
        y[i] += alpha * vi;
    }
}

// y = a x + b y
__global__ void __launch_bounds__(256)
axpby_kernel(int64_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

__global__ void __launch_bounds__(256)
fill_kernel(int64_t n, double v, double *__restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = v;
}

__global__ void set_state_kernel(State *st, int maxiter) {
    State z = {};
    z.maxiter = maxiter;
    *st = z;
}

// -------------------------------------------------------------- refinement

// Tall: h = T^T (b^ - T x) - lambda^2 x in double-double, one pass over T.
// x (length L) is held per thread like w in the sweep.
template <int CPT, typename TT>
__device__ __forceinline__ void resid_dd_tall_body(const TT *__restrict__ T, int64_t ldt, int64_t rows, int L,
                                                   int nblocks, int64_t rows_per_block,
                                                   const double *__restrict__ b, const double *__restrict__ x,
                                                   double lambda, double *__restrict__ hpart_hi,
                                                   double *__restrict__ hpart_lo, const int block) {
    __shared__ double red_hi[2][NT / 64], red_lo[2][NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double xr[CPT];
    dd zr[CPT];
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int col = col_of<CPT>(tid, e);
        xr[e] = col < L ? x[col] : 0.0;
        zr[e] = {0.0, 0.0};
    }
    const int64_t r0 = (int64_t)block * rows_per_block;
    const int64_t r1 = min(rows, r0 + rows_per_block);
    int parity = 0;
    for (int64_t row = r0; row < r1; ++row) {
        const TT *trow = T + row * ldt;
        double av[CPT];
        dd p = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int col = col_of<CPT>(tid, e);
            av[e] = col < L ? (double)trow[col] : 0.0;
            p = dd_fma(p, av[e], xr[e]);
        }
        p = wave_sum_dd(p);
        if (lane == 0) { red_hi[parity][wid] = p.hi; red_lo[parity][wid] = p.lo; }
        __syncthreads();
        dd tx = {0.0, 0.0};
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) tx = dd_add(tx, dd{red_hi[parity][w], red_lo[parity][w]});
        parity ^= 1;
        // res = b - T x
        const dd res = dd_add(dd{b[row], 0.0}, dd{-tx.hi, -tx.lo});
#pragma unroll
        for (int e = 0; e < CPT; ++e) zr[e] = dd_fma_dd(zr[e], av[e], res);
    }
    if (lambda > 0.0) {
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int col = col_of<CPT>(tid, e);
            if (col < L && (col % nblocks) == block) {
                // row m + col: residual 0 - lambda x_col, contributes lambda * residual
                dd res = two_prod(-lambda, xr[e]);
                zr[e] = dd_fma_dd(zr[e], lambda, res);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int col = col_of<CPT>(tid, e);
        if (col < L) {
            hpart_hi[(int64_t)block * L + col] = zr[e].hi;
            hpart_lo[(int64_t)block * L + col] = zr[e].lo;
        }
    }
}

// h = T^T (b - T x) in double-double over the narrow-row layout of
// sweep_narrow_body (LPR lanes a row, 8 columns a lane, L <= 8 LPR, lambda
// = 0): a row's product T_j x is summed over its lanes in double-double
// and taken from the row's first lane (so every lane uses the same bits),
// each lane keeps the residual's contributions to its columns, and these
// are summed over the rows of a wave (shuffles) and then over the waves in
// wave order (LDS).  Offsets of T must fit in 31 bits, as for the sweep.
template <int LPR>
__device__ __forceinline__ void resid_dd_narrow_body(const double *__restrict__ T, int64_t ldt, int64_t rows,
                                                     int L, int64_t rows_per_block,
                                                     const double *__restrict__ b,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ hpart_hi,
                                                     double *__restrict__ hpart_lo, const int block,
                                                     double (*__restrict__ rh)[8 * 64],
                                                     double (*__restrict__ rl)[8 * 64]) {
    constexpr int CPT = 8, RPW = 64 / LPR, NW = NT / 64, STEP = NW * RPW;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int sl = lane % LPR, rw = lane / LPR;
    double xr[CPT];
    dd zr[CPT];
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int col = 2 * sl + 2 * LPR * (e >> 1) + (e & 1);
        xr[e] = col < L ? x[col] : 0.0;
        zr[e] = {0.0, 0.0};
    }
    const int64_t r0 = (int64_t)block * rows_per_block;
    const int64_t r1 = min(rows, r0 + rows_per_block);
    for (int64_t j0 = r0; j0 < r1; j0 += STEP) {
        const int64_t row = j0 + wid * RPW + rw;
        const bool valid = row < r1;
        const double *__restrict__ trow = T + (valid ? row : r0) * ldt;
        double av[CPT];
        dd p = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int col = 2 * sl + 2 * LPR * (e >> 1) + (e & 1);
            av[e] = (valid && col < L) ? trow[col] : 0.0;
            p = dd_fma(p, av[e], xr[e]);
        }
#pragma unroll
        for (int o = 1; o < LPR; o <<= 1) p = dd_add(p, dd{__shfl_xor(p.hi, o, 64), __shfl_xor(p.lo, o, 64)});
        p.hi = __shfl(p.hi, rw * LPR, 64);
        p.lo = __shfl(p.lo, rw * LPR, 64);
        const dd res = valid ? dd_add(dd{b[row], 0.0}, dd{-p.hi, -p.lo}) : dd{0.0, 0.0};
#pragma unroll
        for (int e = 0; e < CPT; ++e) zr[e] = dd_fma_dd(zr[e], av[e], res);
    }
#pragma unroll
    for (int o = LPR; o < 64; o <<= 1)
#pragma unroll
        for (int e = 0; e < CPT; ++e)
            zr[e] = dd_add(zr[e], dd{__shfl_xor(zr[e].hi, o, 64), __shfl_xor(zr[e].lo, o, 64)});
    if (rw == 0) {
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int col = 2 * sl + 2 * LPR * (e >> 1) + (e & 1);
            if (col < L) {
                rh[wid][col] = zr[e].hi;
                rl[wid][col] = zr[e].lo;
            }
        }
    }
    __syncthreads();
    for (int col = tid; col < L; col += NT) {
        dd t = {rh[0][col], rl[0][col]};
#pragma unroll
        for (int w = 1; w < NW; ++w) t = dd_add(t, dd{rh[w][col], rl[w][col]});
        hpart_hi[(int64_t)block * L + col] = t.hi;
        hpart_lo[(int64_t)block * L + col] = t.lo;
    }
}

template <int CPT, typename TT>
__global__ void __launch_bounds__(NT)
resid_dd_tall_kernel(const TT *__restrict__ T, int64_t ldt, int64_t rows, int L, int nblocks,
                     int64_t rows_per_block, const double *__restrict__ b,
                     const double *__restrict__ x, double lambda, double *__restrict__ hpart_hi,
                     double *__restrict__ hpart_lo) {
    resid_dd_tall_body<CPT, TT>(T, ldt, rows, L, nblocks, rows_per_block, b, x, lambda, hpart_hi, hpart_lo,
                                (int)blockIdx.x);
}

// Fat: z = T^T x = A x in double-double (rows of T weighted by x).
template <int CPT, typename TT>
__global__ void __launch_bounds__(NT)
ax_dd_fat_kernel(const TT *__restrict__ T, int64_t ldt, int64_t rows, int L,
                 int64_t rows_per_block, const double *__restrict__ x,
                 double *__restrict__ zpart_hi, double *__restrict__ zpart_lo) {
    const int tid = threadIdx.x;
    dd zr[CPT];
#pragma unroll
    for (int e = 0; e < CPT; ++e) zr[e] = {0.0, 0.0};
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(rows, r0 + rows_per_block);
    for (int64_t row = r0; row < r1; ++row) {
        const TT *trow = T + row * ldt;
        const double xv = x[row];
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int col = col_of<CPT>(tid, e);
            if (col < L) zr[e] = dd_fma(zr[e], (double)trow[col], xv);
        }
    }
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int col = col_of<CPT>(tid, e);
        if (col < L) {
            zpart_hi[(int64_t)blockIdx.x * L + col] = zr[e].hi;
            zpart_lo[(int64_t)blockIdx.x * L + col] = zr[e].lo;
        }
    }
}

// out = sum over nb partials (double-double), optionally out = bvec - sum.
__global__ void __launch_bounds__(256)
reduce_dd_kernel(const double *__restrict__ phi, const double *__restrict__ plo, int nb, int L,
                 const double *__restrict__ bvec, double *__restrict__ out_hi,
                 double *__restrict__ out_lo, double lambda = 0.0,
                 const double *__restrict__ rho = nullptr) {
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= L) return;
    dd t = {0.0, 0.0};
    for (int b = 0; b < nb; ++b) t = dd_add(t, dd{phi[(int64_t)b * L + col], plo[(int64_t)b * L + col]});
    // the under-determined Tikhonov form: [A, lambda I] [x; rho] = A x + lambda rho
    if (rho) t = dd_fma(t, lambda, rho[col]);
    if (bvec) t = dd_add(dd{bvec[col], 0.0}, dd{-t.hi, -t.lo});
    out_hi[col] = t.hi;
    if (out_lo) out_lo[col] = t.lo;
}

// y = M^T v for row-major M (nrows x ncols, ld) with v = vhi + vlo in
// double-double accumulation; one wavefront per output column chunk.
__global__ void __launch_bounds__(256)
gemv_t_dd_kernel(const double *__restrict__ M, int64_t ld, int64_t nrows, int64_t ncols,
                 const double *__restrict__ vhi, const double *__restrict__ vlo,
                 double *__restrict__ y) {
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= ncols) return;
    const int lane = threadIdx.x & 63;
    dd t = {0.0, 0.0};
    for (int64_t i = lane; i < nrows; i += 64) t = dd_fma_dd(t, M[i * ld + c], dd{vhi[i], vlo[i]});
    t = wave_sum_dd(t);
    if (lane == 0) y[c] = t.hi + t.lo;
}

// CG on K^T K z = c: given t = K^T K p (sweep) and acc0 = ||K p||^2.
__device__ __forceinline__ void cg_step_body(const double *__restrict__ t, int64_t r, double *__restrict__ z,
                                             double *__restrict__ res, double *__restrict__ p, State *st) {
    if (st->done) return;
    __shared__ double scratch[SNT / 64];
    const double pbp = st->acc[0];
    const double rs = st->cg_rs;
    const double a = pbp > 0.0 ? rs / pbp : 0.0;
    double part = 0.0;
    for (int64_t i = threadIdx.x; i < r; i += SNT) {
        z[i] += a * p[i];
        const double ri = res[i] - a * t[i];
        res[i] = ri;
        part += ri * ri;
    }
    const double rs_new = block_sum<SNT>(part, scratch);
    const double bta = rs > 0.0 ? rs_new / rs : 0.0;
    for (int64_t i = threadIdx.x; i < r; i += SNT) p[i] = res[i] + bta * p[i];
    if (threadIdx.x == 0) {
        st->cg_rs = rs_new;
        const int it = st->iters + 1;
        st->iters = it;
        const bool conv = sqrt(rs_new) <= st->cg_stop || pbp <= 0.0;
        st->converged = conv ? 1 : 0;
        st->done = (conv || it >= st->maxiter) ? 1 : 0;
    }
}

__global__ void __launch_bounds__(SNT)
cg_step_kernel(const double *__restrict__ t, int64_t r, double *__restrict__ z,
               double *__restrict__ res, double *__restrict__ p, State *st) {
    cg_step_body(t, r, z, res, p, st);
}

__device__ __forceinline__ void cg_init_body(const double *__restrict__ c, int64_t r, double *__restrict__ z,
                                             double *__restrict__ res, double *__restrict__ p, double rtol,
                                             int maxiter, State *st) {
    __shared__ double scratch[SNT / 64];
    double part = 0.0;
    for (int64_t i = threadIdx.x; i < r; i += SNT) {
        z[i] = 0.0;
        res[i] = c[i];
        p[i] = c[i];
        part += c[i] * c[i];
    }
    const double rs = block_sum<SNT>(part, scratch);
    if (threadIdx.x == 0) {
        State s0 = {};
        s0.maxiter = maxiter;
        s0.cg_rs = rs;
        s0.cg_stop = rtol * sqrt(rs);
        s0.done = rs == 0.0 ? 1 : 0;
        s0.converged = s0.done;
        *st = s0;
    }
}

__global__ void __launch_bounds__(SNT)
cg_init_kernel(const double *__restrict__ c, int64_t r, double *__restrict__ z,
               double *__restrict__ res, double *__restrict__ p, double rtol, int maxiter,
               State *st) {
    cg_init_body(c, r, z, res, p, rtol, maxiter, st);
}

// ------------------------------------------------------------ sparse passes
//
// For sparse T a sweep is two passes: a row pass over CSR(T) forms
// q_j = T_j w and the row-local update of the same operation as the dense
// sweep, storing c_j in the long vector; a column pass over CSR(T^T) forms
// z = T^T c by gathering c.  Both run in a fixed order (no atomics).

constexpr int CRP_NT = 256;  // threads of the row pass
constexpr int CRP_G = 8;     // lanes per row
constexpr int CCP_NT = 256;  // column pass: one wavefront per column

struct CsrArgs {
    CsrMat t;                 // CSR(T)
    int64_t K, total;         // rows of T; rows including the Tikhonov rows
    int64_t rows_per_block;
    const double *w;
    double *y, *xv, *wv;
    double *spart;            // nblocks x 4
    State *st;
    double lambda, alpha, beta;
};

__device__ __forceinline__ double group8_sum(double v) {
    v += __shfl_xor(v, 4, CRP_G);
    v += __shfl_xor(v, 2, CRP_G);
    v += __shfl_xor(v, 1, CRP_G);
    return v;
}

__device__ __forceinline__ dd group8_sum_dd(dd v) {
#pragma unroll
    for (int m = 4; m >= 1; m >>= 1) {
        const dd o{__shfl_xor(v.hi, m, CRP_G), __shfl_xor(v.lo, m, CRP_G)};
        v = dd_add(v, o);
    }
    return v;
}

// The scalars of the current iteration that the row-local update needs.
struct RowScalars {
    double coef = 0.0, inv_alpha = 0.0, beta = 0.0, phi_rho = 0.0, theta_rho = 0.0;
    int pending = 0;
};

template <int OP>
__device__ __forceinline__ RowScalars row_scalars(const CsrArgs &a) {
    RowScalars r;
    if (OP == OP_LSQR_TALL) r.coef = a.st->coef;
    if (OP == OP_CS_TALL) r.coef = a.alpha;
    if (OP == OP_LSQR_FAT) {
        r.inv_alpha = a.st->inv_alpha;
        r.beta = a.st->beta;
        r.phi_rho = a.st->phi_rho;
        r.theta_rho = a.st->theta_rho;
        r.pending = a.st->pending;
    }
    return r;
}

// The row-local part of a pass, given q = T_row w: the same update as the
// dense sweep's, with the partial norms in acc0 .. acc3.
template <int OP>
__device__ __forceinline__ void row_local(const CsrArgs &a, const RowScalars &sc, int64_t row,
                                          double q, double &acc0, double &acc1, double &acc2,
                                          double &acc3) {
    const double coef = sc.coef, inv_alpha = sc.inv_alpha, beta = sc.beta;
    const double phi_rho = sc.phi_rho, theta_rho = sc.theta_rho;
    const int pending = sc.pending;
    {
        if (OP == OP_ATB) {
            const double c = a.y[row];
            acc0 += c * c;
        } else if (OP == OP_LSQR_TALL) {
            const double c = q - coef * a.y[row];
            a.y[row] = c;
            acc0 += c * c;
        } else if (OP == OP_CS_TALL) {
            const double c = a.y[row] - coef * q;
            a.y[row] = c;
            acc0 += c * c;
        } else if (OP == OP_NORMAL) {
            a.y[row] = q;
            acc0 += q * q;
        } else if (OP == OP_LSQR_FAT) {
            const double v = a.y[row] * inv_alpha;
            const double c = q - beta * v;
            if (pending == 1) {
                a.wv[row] = v;
                acc3 += v * v;
            } else if (pending == 2) {
                const double xo = a.xv[row] + phi_rho * a.wv[row];
                const double wn = v - theta_rho * a.wv[row];
                a.xv[row] = xo;
                a.wv[row] = wn;
                acc1 += xo * xo;
                acc2 += xo * wn;
                acc3 += wn * wn;
            }
            a.y[row] = c;
            acc0 += c * c;
        } else {  // OP_CS_FAT
            const double c = a.beta * a.y[row] + q;
            a.y[row] = c;
            a.xv[row] += a.alpha * c;
            acc0 += c * c;
        }
    }
}

// The workgroup's partial norms into spart (fixed order).
__device__ __forceinline__ void store_row_partials(const CsrArgs &a, double acc0, double acc1,
                                                   double acc2, double acc3) {
    __shared__ double red[CRP_NT / 64][4];
    const int tid = threadIdx.x;
    acc0 = wave_sum(acc0);
    acc1 = wave_sum(acc1);
    acc2 = wave_sum(acc2);
    acc3 = wave_sum(acc3);
    const int lane = tid & 63, wid = tid >> 6;
    if (lane == 0) {
        red[wid][0] = acc0; red[wid][1] = acc1; red[wid][2] = acc2; red[wid][3] = acc3;
    }
    __syncthreads();
    if (tid < 4) {
        double t = 0.0;
        for (int w = 0; w < CRP_NT / 64; ++w) t += red[w][tid];
        a.spart[(int64_t)blockIdx.x * 4 + tid] = t;
    }
}

template <int OP>
__global__ void __launch_bounds__(CRP_NT) csr_row_pass_kernel(CsrArgs a) {
    if (a.st->done) return;
    const int tid = threadIdx.x, g = tid / CRP_G, l = tid % CRP_G;
    constexpr int NG = CRP_NT / CRP_G;
    const RowScalars sc = row_scalars<OP>(a);
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r1 = min(a.total, r0 + a.rows_per_block);
    for (int64_t row = r0 + g; row < r1; row += NG) {
        double q = 0.0;
        if (OP != OP_ATB) {
            if (row < a.K) {
                const int64_t e0 = a.t.ptr[row], e1 = a.t.ptr[row + 1];
                // the row's first 4 CRP_G entries: indices and values, then
                // the gathered w, all requested before any is used (the
                // summation order is that of the plain loop)
                constexpr int U = 4;
                int32_t ix[U];
                double vv[U], ww[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t e = e0 + l + CRP_G * u;
                    ix[u] = e < e1 ? a.t.idx[e] : -1;
                    vv[u] = e < e1 ? a.t.val[e] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) ww[u] = ix[u] >= 0 ? a.w[ix[u]] : 0.0;
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (ix[u] >= 0) q += vv[u] * ww[u];
                for (int64_t e = e0 + l + CRP_G * U; e < e1; e += CRP_G) q += a.t.val[e] * a.w[a.t.idx[e]];
                q = group8_sum(q);
            } else {
                q = a.lambda * a.w[row - a.K];
            }
        }
        if (l != 0) continue;
        row_local<OP>(a, sc, row, q, acc0, acc1, acc2, acc3);
    }
    store_row_partials(a, acc0, acc1, acc2, acc3);
}

// Row pass of an operator T: q = T w was formed by the caller's product
// (qv, K rows); the Tikhonov rows give lambda w.  One thread per row.
template <int OP>
__global__ void __launch_bounds__(CRP_NT) op_row_pass_kernel(CsrArgs a, const double *__restrict__ qv) {
    if (a.st->done) return;
    const RowScalars sc = row_scalars<OP>(a);
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r1 = min(a.total, r0 + a.rows_per_block);
    for (int64_t row = r0 + threadIdx.x; row < r1; row += CRP_NT) {
        double q = 0.0;
        if (OP != OP_ATB) q = row < a.K ? qv[row] : a.lambda * a.w[row - a.K];
        row_local<OP>(a, sc, row, q, acc0, acc1, acc2, acc3);
    }
    store_row_partials(a, acc0, acc1, acc2, acc3);
}

// Column pass over segments: zseg_g = sum of T(k, j) y_k over segment g
// (at most SparseView::kColSeg entries of column j of T), one wavefront per
// segment.
__global__ void __launch_bounds__(CCP_NT)
csr_col_seg_kernel(CsrMat ct, const int32_t *__restrict__ seg_row,
                   const int32_t *__restrict__ row_seg, int64_t nseg, const double *__restrict__ y,
                   double *__restrict__ zseg, const State *st) {
    if (st && st->done) return;
    const int64_t g = (int64_t)blockIdx.x * (CCP_NT / 64) + (threadIdx.x >> 6);
    if (g >= nseg) return;
    const int lane = threadIdx.x & 63;
    const int j = seg_row[g];
    const int64_t e0 = ct.ptr[j] + (g - row_seg[j]) * SparseView::kColSeg;
    const int64_t e1 = min(e0 + SparseView::kColSeg, ct.ptr[j + 1]);
    // a segment holds at most 8 entries per lane: every index and value is
    // loaded first, then every gathered y, so the lane waits for two load
    // latencies rather than two per entry
    constexpr int U = (int)(SparseView::kColSeg / 64);
    int32_t ix[U];
    double vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t e = e0 + lane + 64 * u;
        ix[u] = e < e1 ? ct.idx[e] : -1;
        vv[u] = e < e1 ? ct.val[e] : 0.0;
    }
    double yy[U];
#pragma unroll
    for (int u = 0; u < U; ++u) yy[u] = ix[u] >= 0 ? y[ix[u]] : 0.0;
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) t += vv[u] * yy[u];
    t = wave_sum(t);
    if (lane == 0) zseg[g] = t;
}

// z_j = the segments of column j summed (+ lambda y_{K+j}): one wavefront
// per column, lane l summing segments l, l + 64, ... in order, then the
// wavefront's fixed butterfly, so a column of many segments (a long row of
// a fat A) does not serialise one thread.
__global__ void __launch_bounds__(256)
csr_col_combine_kernel(const int32_t *__restrict__ row_seg, int64_t d,
                       const double *__restrict__ zseg, const double *__restrict__ y, double lambda,
                       int64_t K, double *__restrict__ z, const State *st) {
    if (st && st->done) return;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= d) return;
    const int lane = threadIdx.x & 63;
    double t = 0.0;
    for (int g = row_seg[j] + lane; g < row_seg[j + 1]; g += 64) t += zseg[g];
    t = wave_sum(t);
    if (lane == 0) z[j] = lambda > 0.0 ? t + lambda * y[K + j] : t;
}

// st->acc = sums of the row-pass partials (fixed order).
__global__ void __launch_bounds__(256)
reduce_spart_kernel(const double *__restrict__ spart, int nb, State *st) {
    if (st->done) return;
    __shared__ double red[4][4];
    const int tid = threadIdx.x, k = tid & 3, part = tid >> 2;  // 64 partial sums per accumulator
    double t = 0.0;
    for (int b = part; b < nb; b += 64) t += spart[b * 4 + k];
    // reduce over the 64 threads with the same k: lanes k, k+4, ... within
    // each wavefront, then across the 4 wavefronts
    for (int m = 32; m >= 4; m >>= 1) t += __shfl_xor(t, m);
    if ((tid & 63) < 4) red[tid >> 6][k] = t;
    __syncthreads();
    if (tid < 4) st->acc[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
}

// Tall refinement, rows: res_k = b_k - T_k x (k < K) and res_{K+j} =
// -lambda x_j, in double-double.
__global__ void __launch_bounds__(CRP_NT)
csr_resid_rows_dd_kernel(CsrMat t, int64_t K, int64_t total, int64_t rows_per_block,
                         const double *__restrict__ b, const double *__restrict__ x,
                         double lambda, double *__restrict__ rhi, double *__restrict__ rlo) {
    const int tid = threadIdx.x, g = tid / CRP_G, l = tid % CRP_G;
    constexpr int NG = CRP_NT / CRP_G;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(total, r0 + rows_per_block);
    for (int64_t row = r0 + g; row < r1; row += NG) {
        dd res;
        if (row < K) {
            dd p = {0.0, 0.0};
            const int64_t e0 = t.ptr[row], e1 = t.ptr[row + 1];
            for (int64_t e = e0 + l; e < e1; e += CRP_G) p = dd_fma(p, t.val[e], x[t.idx[e]]);
            p = group8_sum_dd(p);
            res = dd_add(dd{b[row], 0.0}, dd{-p.hi, -p.lo});
        } else {
            res = two_prod(-lambda, x[row - K]);
        }
        if (l == 0) {
            rhi[row] = res.hi;
            rlo[row] = res.lo;
        }
    }
}

// Column pass in double-double: out_j = sum_k T(k, j) (yhi_k + ylo_k)
// (+ lambda (yhi + ylo)_{K+j}); ylo may be NULL.
__global__ void __launch_bounds__(CCP_NT)
csr_col_pass_dd_kernel(CsrMat ct, const double *__restrict__ yhi, const double *__restrict__ ylo,
                       double lambda, int64_t K, double *__restrict__ out_hi,
                       double *__restrict__ out_lo) {
    const int64_t j = (int64_t)blockIdx.x * (CCP_NT / 64) + (threadIdx.x >> 6);
    if (j >= ct.nrows) return;
    const int lane = threadIdx.x & 63;
    dd t = {0.0, 0.0};
    const int64_t e0 = ct.ptr[j], e1 = ct.ptr[j + 1];
    for (int64_t e = e0 + lane; e < e1; e += 64) {
        const int32_t k = ct.idx[e];
        t = dd_fma_dd(t, ct.val[e], dd{yhi[k], ylo ? ylo[k] : 0.0});
    }
    t = wave_sum_dd(t);
    if (lane == 0) {
        if (lambda > 0.0) t = dd_fma_dd(t, lambda, dd{yhi[K + j], ylo ? ylo[K + j] : 0.0});
        out_hi[j] = t.hi;
        if (out_lo) out_lo[j] = t.lo;
    }
}

// ------------------------------------------------------------ host driver

int grid1(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 4096)); }

struct Ctx {
    const IterProblem &pb;
    hipStream_t st;
    int L;
    int nblocks;
    int64_t rows_per_block;
    int cpt, R;
    int narrow = 0;  // lanes per row of the narrow tall sweep (0: the wide sweep)
    int ngroups, chunk;
    DevBuf zpart, spart, zred, sred, z, stbuf, Pt;
    DevBuf zseg;  // sparse: per-segment column sums
    DevBuf qv;    // operator: T w from the caller's product
    State *state;
    const double *Ptp;  // P^T, r x L row-major (ld L)
    // optional per-launch timing of the sweep kernel
    bool profile = false;
    std::vector<hipEvent_t> ev;
    // precision form: sweeps read the FP64 T instead of its FP32 copy
    bool force_f64 = false;

    // event pairs of launches that found the done flag set (no pass over A)
    std::vector<hipEvent_t> ev_noop;

    ~Ctx() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        for (hipEvent_t e : ev_noop) (void)hipEventDestroy(e);
    }

    // Sweeps timed so far; with prof_keep, the launches of a convergence-
    // checked loop past its last iteration (the rest of its last chunk,
    // which return at once on the done flag) are left out of the sweep
    // timing and count.
    size_t prof_mark() const { return ev.size() / 2; }
    void prof_keep(size_t mark, int64_t real) {
        if (!profile) return;
        const size_t end = std::min(ev.size() / 2, mark + (size_t)std::max<int64_t>(real, 0));
        for (size_t i = 2 * end; i < ev.size(); ++i) ev_noop.push_back(ev[i]);
        ev.resize(2 * end);
    }

    double sweep_kernel_ms() {
        double t = 0.0;
        for (size_t i = 0; i + 1 < ev.size(); i += 2) {
            LSRN_HIP(hipEventSynchronize(ev[i + 1]));
            float ms = 0.f;
            LSRN_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            t += ms;
        }
        return t;
    }

    Ctx(const IterProblem &p, hipStream_t s, bool autotune = false) : pb(p), st(s) {
        L = (int)pb.cols;
        if (pb.sp || pb.op) {
            // sparse: row-pass workgroups over the rows of T and the Tikhonov rows
            cpt = 0; R = 1;
            const int64_t total = pb.rows + (pb.lambda > 0.0 ? pb.cols : 0);
            const int64_t want = 4 * (int64_t)device_cus();
            nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, ceil_div(total, CRP_NT / CRP_G)));
            rows_per_block = ceil_div(total, nblocks);
            nblocks = (int)std::max<int64_t>(1, ceil_div(total, rows_per_block));
            chunk = 16;
            ngroups = 1;
            spart.alloc((size_t)nblocks * 4 * sizeof(double));
            z.alloc((size_t)L * sizeof(double));
            if (pb.sp) zseg.alloc((size_t)pb.sp->nseg * sizeof(double));
            else qv.alloc((size_t)pb.rows * sizeof(double));
            stbuf.alloc(sizeof(State));
            state = stbuf.as<State>();
            Pt.alloc((size_t)std::max<int64_t>(pb.r, 1) * L * sizeof(double));
            transpose(L, pb.r, pb.P, pb.ldp, Pt.as<double>(), st);
            Ptp = Pt.as<double>();
            return;
        }
        if (L <= 512) { cpt = 2; R = 8; }
        else if (L <= 1024) { cpt = 4; R = 4; }
        else if (L <= 2048) { cpt = 8; R = 4; }
        else if (L <= 4096) { cpt = 16; R = 2; }
        else fail(LSRN_E_UNSUPPORTED, "dense iteration supports min(m, n) <= 4096");
        // narrow tall rows: LPR lanes per row instead of the whole workgroup
        if (pb.tall && L <= 256 && (pb.rows + 512) * pb.ldt < ((int64_t)1 << 28))
            for (int l = 2; l <= 32 && !narrow; l *= 2)
                if (L <= 8 * l) narrow = l;
        // workgroups per compute unit: a recorded (tuned) value for this
        // shape key, else 2; with autotune and no record, every candidate is
        // timed below on this problem and the fastest recorded
        TuneKey key;
        key.phase = TUNE_SWEEP;
        key.dtype = pb.T32 ? 1 : 0;
        key.rows_log2 = rows_bucket(pb.rows);
        key.cols = L;
        int per_cu = 2;
        const bool recorded = tune_lookup(key, per_cu);
        const bool tune = autotune && !recorded;
        chunk = 16;
        shape(tune ? kMaxPerCu : per_cu);
        zpart.alloc((size_t)nblocks * L * sizeof(double));
        spart.alloc((size_t)nblocks * 4 * sizeof(double));
        zred.alloc((size_t)ngroups * L * sizeof(double));
        sred.alloc((size_t)ngroups * 4 * sizeof(double));
        z.alloc((size_t)L * sizeof(double));
        stbuf.alloc(sizeof(State));
        state = stbuf.as<State>();
        // P^T (r x L) for the t = P^T z products
        Pt.alloc((size_t)std::max<int64_t>(pb.r, 1) * L * sizeof(double));
        transpose(L, pb.r, pb.P, pb.ldp, Pt.as<double>(), st);
        Ptp = Pt.as<double>();
        if (tune) per_cu = tune_sweep(key);
        shape(per_cu);
    }

    static constexpr int kMaxPerCu = 4;

    // Dense sweep launch shape for `per_cu` workgroups per compute unit.
    void shape(int per_cu) {
        const int64_t want = (int64_t)per_cu * device_cus();
        nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, ceil_div(pb.rows, R)));
        rows_per_block = round_up(ceil_div(pb.rows, nblocks), R);
        nblocks = (int)std::max<int64_t>(1, ceil_div(pb.rows, rows_per_block));
        ngroups = (int)ceil_div(nblocks, chunk);
    }

    // Time the normal-equation sweep (one pass over A, the iterations' pass)
    // for 1 .. kMaxPerCu workgroups per compute unit on this problem,
    // record the fastest for the shape key and return it.
    int tune_sweep(const TuneKey &key) {
        DevBuf wb((size_t)L * sizeof(double)), yb((size_t)pb.rows * sizeof(double));
        fill_kernel<<<grid1(L), 256, 0, st>>>(L, 0.0, wb.as<double>());
        LSRN_HIP(hipGetLastError());
        hipEvent_t e0, e1;
        LSRN_HIP(hipEventCreate(&e0));
        LSRN_HIP(hipEventCreate(&e1));
        int best = 2;
        float best_ms = 0.f;
        for (int c = 1; c <= kMaxPerCu; ++c) {
            shape(c);
            reset_state(1);
            sweep(OP_NORMAL, wb.as<double>(), yb.as<double>(), nullptr, nullptr);
            LSRN_HIP(hipEventRecord(e0, st));
            for (int k = 0; k < 3; ++k) sweep(OP_NORMAL, wb.as<double>(), yb.as<double>(), nullptr, nullptr);
            LSRN_HIP(hipEventRecord(e1, st));
            LSRN_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            LSRN_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (c == 1 || ms < best_ms) {
                best = c;
                best_ms = ms;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        tune_store(key, best);
        return best;
    }

    void reset_state(int maxiter) {
        set_state_kernel<<<1, 1, 0, st>>>(state, maxiter);
        LSRN_HIP(hipGetLastError());
    }

    template <int CPT, int RR, bool F32>
    void sweep_tf(int op, SweepArgs &a) {
        switch (op) {
            case OP_ATB: sweep_kernel<CPT, RR, OP_ATB, F32><<<nblocks, NT, 0, st>>>(a); break;
            case OP_LSQR_TALL: sweep_kernel<CPT, RR, OP_LSQR_TALL, F32><<<nblocks, NT, 0, st>>>(a); break;
            case OP_CS_TALL: sweep_kernel<CPT, RR, OP_CS_TALL, F32><<<nblocks, NT, 0, st>>>(a); break;
            case OP_NORMAL: sweep_kernel<CPT, RR, OP_NORMAL, F32><<<nblocks, NT, 0, st>>>(a); break;
            case OP_LSQR_FAT: sweep_kernel<CPT, RR, OP_LSQR_FAT, F32><<<nblocks, NT, 0, st>>>(a); break;
            default: sweep_kernel<CPT, RR, OP_CS_FAT, F32><<<nblocks, NT, 0, st>>>(a); break;
        }
    }
    template <int LPR>
    void sweep_narrow_l(int op, SweepArgs &a) {
        switch (op) {
            case OP_ATB: sweep_narrow_kernel<LPR, OP_ATB><<<nblocks, NT, 0, st>>>(a); break;
            case OP_LSQR_TALL: sweep_narrow_kernel<LPR, OP_LSQR_TALL><<<nblocks, NT, 0, st>>>(a); break;
            case OP_CS_TALL: sweep_narrow_kernel<LPR, OP_CS_TALL><<<nblocks, NT, 0, st>>>(a); break;
            default: sweep_narrow_kernel<LPR, OP_NORMAL><<<nblocks, NT, 0, st>>>(a); break;
        }
    }
    void sweep_narrow(int op, SweepArgs &a) {
        switch (narrow) {
            case 2: sweep_narrow_l<2>(op, a); break;
            case 4: sweep_narrow_l<4>(op, a); break;
            case 8: sweep_narrow_l<8>(op, a); break;
            case 16: sweep_narrow_l<16>(op, a); break;
            default: sweep_narrow_l<32>(op, a); break;
        }
    }
    template <int CPT, int RR>
    void sweep_t(int op, SweepArgs &a) {
        if (a.T32) sweep_tf<CPT, RR, true>(op, a);
        else sweep_tf<CPT, RR, false>(op, a);
    }

    // One pass: z = sum_j op_j T_j, st->acc = reduced accumulators.
    void sweep(int op, const double *w, double *y, double *xv, double *wv, double alpha = 0.0,
               double beta = 0.0) {
        if (pb.sp) {
            sweep_sparse(op, w, y, xv, wv, alpha, beta);
            return;
        }
        if (pb.op) {
            sweep_op(op, w, y, xv, wv, alpha, beta);
            return;
        }
        SweepArgs a;
        a.T = pb.T; a.T32 = force_f64 ? nullptr : pb.T32; a.ldt = pb.ldt; a.rows = pb.rows; a.L = L;
        a.nblocks = nblocks;
        a.rows_per_block = rows_per_block; a.w = w; a.zpart = zpart.as<double>();
        a.spart = spart.as<double>(); a.y = y; a.xv = xv; a.wv = wv; a.st = state;
        a.lambda = pb.lambda; a.alpha = alpha; a.beta = beta;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (profile) {
            LSRN_HIP(hipEventCreate(&e0));
            LSRN_HIP(hipEventCreate(&e1));
            ev.push_back(e0);
            ev.push_back(e1);
            LSRN_HIP(hipEventRecord(e0, st));
        }
        if (narrow && !a.T32 && a.lambda == 0.0 &&
            (op == OP_ATB || op == OP_LSQR_TALL || op == OP_CS_TALL || op == OP_NORMAL)) sweep_narrow(op, a);
        else if (cpt == 2) sweep_t<2, 8>(op, a);
        else if (cpt == 4) sweep_t<4, 4>(op, a);
        else if (cpt == 8) sweep_t<8, 4>(op, a);
        else sweep_t<16, 2>(op, a);
        LSRN_HIP(hipGetLastError());
        if (profile) LSRN_HIP(hipEventRecord(e1, st));
        dim3 g1((unsigned)ceil_div(L, 256), (unsigned)ngroups);
        reduce_stage1_kernel<<<g1, 256, 0, st>>>(zpart.as<double>(), spart.as<double>(), nblocks, L,
                                                 chunk, zred.as<double>(), sred.as<double>(), state);
        reduce_stage2_kernel<<<(unsigned)ceil_div(L, 256), 256, 0, st>>>(
            zred.as<double>(), sred.as<double>(), ngroups, L, z.as<double>(), state);
        LSRN_HIP(hipGetLastError());
    }

    // Sparse sweep: row pass (q, row-local update, partial norms), column
    // pass z = T^T c, and the partial norms reduced into st->acc.
    void sweep_sparse(int op, const double *w, double *y, double *xv, double *wv, double alpha,
                      double beta) {
        CsrArgs a;
        a.t = pb.sp->rows; a.K = pb.rows;
        a.total = pb.rows + (pb.lambda > 0.0 ? pb.cols : 0);
        a.rows_per_block = rows_per_block; a.w = w; a.y = y; a.xv = xv; a.wv = wv;
        a.spart = spart.as<double>(); a.st = state; a.lambda = pb.lambda; a.alpha = alpha; a.beta = beta;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (profile) {
            LSRN_HIP(hipEventCreate(&e0));
            LSRN_HIP(hipEventCreate(&e1));
            ev.push_back(e0);
            ev.push_back(e1);
            LSRN_HIP(hipEventRecord(e0, st));
        }
        switch (op) {
            case OP_ATB: csr_row_pass_kernel<OP_ATB><<<nblocks, CRP_NT, 0, st>>>(a); break;
            case OP_LSQR_TALL: csr_row_pass_kernel<OP_LSQR_TALL><<<nblocks, CRP_NT, 0, st>>>(a); break;
            case OP_CS_TALL: csr_row_pass_kernel<OP_CS_TALL><<<nblocks, CRP_NT, 0, st>>>(a); break;
            case OP_NORMAL: csr_row_pass_kernel<OP_NORMAL><<<nblocks, CRP_NT, 0, st>>>(a); break;
            case OP_LSQR_FAT: csr_row_pass_kernel<OP_LSQR_FAT><<<nblocks, CRP_NT, 0, st>>>(a); break;
            default: csr_row_pass_kernel<OP_CS_FAT><<<nblocks, CRP_NT, 0, st>>>(a); break;
        }
        csr_col_seg_kernel<<<(unsigned)ceil_div(pb.sp->nseg, CCP_NT / 64), CCP_NT, 0, st>>>(
            pb.sp->cols, pb.sp->seg_row.as<int32_t>(), pb.sp->row_seg.as<int32_t>(), pb.sp->nseg, y,
            zseg.as<double>(), state);
        csr_col_combine_kernel<<<(unsigned)ceil_div(L, 4), 256, 0, st>>>(
            pb.sp->row_seg.as<int32_t>(), L, zseg.as<double>(), y, pb.lambda, pb.rows, z.as<double>(),
            state);
        LSRN_HIP(hipGetLastError());
        if (profile) LSRN_HIP(hipEventRecord(e1, st));
        reduce_spart_kernel<<<1, 256, 0, st>>>(spart.as<double>(), nblocks, state);
        LSRN_HIP(hipGetLastError());
    }

    // Operator sweep: q = T w by the caller's product, the row pass on q,
    // z = T^T y by the caller's product (+ lambda y of the Tikhonov rows).
    // The products run even after the device-side done flag is set; the
    // library's kernels then leave every vector unchanged.
    void sweep_op(int op, const double *w, double *y, double *xv, double *wv, double alpha,
                  double beta) {
        CsrArgs a;
        a.K = pb.rows;
        a.total = pb.rows + (pb.lambda > 0.0 ? pb.cols : 0);
        a.rows_per_block = rows_per_block; a.w = w; a.y = y; a.xv = xv; a.wv = wv;
        a.spart = spart.as<double>(); a.st = state; a.lambda = pb.lambda; a.alpha = alpha; a.beta = beta;
        if (op != OP_ATB) pb.op->apply_t(0, 1, w, L, qv.as<double>(), pb.rows, st);
        const double *q = qv.as<double>();
        switch (op) {
            case OP_ATB: op_row_pass_kernel<OP_ATB><<<nblocks, CRP_NT, 0, st>>>(a, q); break;
            case OP_LSQR_TALL: op_row_pass_kernel<OP_LSQR_TALL><<<nblocks, CRP_NT, 0, st>>>(a, q); break;
            case OP_CS_TALL: op_row_pass_kernel<OP_CS_TALL><<<nblocks, CRP_NT, 0, st>>>(a, q); break;
            case OP_NORMAL: op_row_pass_kernel<OP_NORMAL><<<nblocks, CRP_NT, 0, st>>>(a, q); break;
            case OP_LSQR_FAT: op_row_pass_kernel<OP_LSQR_FAT><<<nblocks, CRP_NT, 0, st>>>(a, q); break;
            default: op_row_pass_kernel<OP_CS_FAT><<<nblocks, CRP_NT, 0, st>>>(a, q); break;
        }
        LSRN_HIP(hipGetLastError());
        pb.op->apply_t(1, 1, y, pb.rows, z.as<double>(), L, st);
        if (pb.lambda > 0.0) {
            axpby_kernel<<<grid1(L), 256, 0, st>>>(L, pb.lambda, y + pb.rows, 1.0, z.as<double>());
            LSRN_HIP(hipGetLastError());
        }
        reduce_spart_kernel<<<1, 256, 0, st>>>(spart.as<double>(), nblocks, state);
        LSRN_HIP(hipGetLastError());
    }

    // out (length rows_of_M) = M x.
    void gemv(const double *M, int64_t ld, int64_t nrows, int64_t ncols, const double *x,
              double *out, bool honour_done = true) {
        if (nrows <= 0) return;
        gemv_kernel<<<(unsigned)ceil_div(nrows, 4), 256, 0, st>>>(M, ld, nrows, ncols, x, out,
                                                                   honour_done ? state : nullptr);
        LSRN_HIP(hipGetLastError());
    }

    State host_state() {
        State h;
        LSRN_HIP(hipMemcpyAsync(&h, state, sizeof(State), hipMemcpyDeviceToHost, st));
        LSRN_HIP(hipStreamSynchronize(st));
        return h;
    }

    // A chunk of iterations (kernel launches only, their arguments fixed) is
    // captured once into a HIP graph and replayed: one launch per chunk
    // instead of one per kernel.  Per-launch timing needs the eager path.
    bool use_graphs = false;
    template <class F>
    void run_chunk(hipGraphExec_t &exec, F &&body) {
        if (!use_graphs) {
            body();
            return;
        }
        if (!exec) {
            hipGraph_t graph = nullptr;
            LSRN_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            try {
                body();
            } catch (...) {
                (void)hipStreamEndCapture(st, &graph);
                if (graph) (void)hipGraphDestroy(graph);
                throw;
            }
            LSRN_HIP(hipStreamEndCapture(st, &graph));
            const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            LSRN_HIP(e);
        }
        LSRN_HIP(hipGraphLaunch(exec, st));
    }
};

struct GraphExec {
    hipGraphExec_t g = nullptr;
    ~GraphExec() {
        if (g) (void)hipGraphExecDestroy(g);
    }
};

int64_t default_maxiter(const IterProblem &pb, const lsrn_options &opt, double &sl, double &su) {
    const double lo = std::sqrt((double)pb.s) - std::sqrt((double)pb.r) - opt.t_margin;
    const double hi = std::sqrt((double)pb.s) + std::sqrt((double)pb.r) + opt.t_margin;
    sl = su = 0.0;
    int64_t cs = -1;
    if (lo > 0.0) {
        su = 1.0 / lo;
        sl = 1.0 / hi;
        const double rate = (su - sl) / (su + sl);
        cs = rate > 0.0 ? (int64_t)std::ceil((std::log(opt.tol) - std::log(2.0)) / std::log(rate)) + 1 : 1;
    }
    if (opt.max_iter > 0) return opt.max_iter;
    return cs > 0 ? cs + 10 : 10 * pb.cols + 100;
}

// Chebyshev step lengths of Alg. 3 (k = 0 .. K); alpha_1 = 1/(d - c^2/(2d)).
void cs_schedule(double sl, double su, double eps, std::vector<double> &al, std::vector<double> &be) {
    const double d = 0.5 * (su * su + sl * sl), c = 0.5 * (su * su - sl * sl);
    const double rate = (su - sl) / (su + sl);
    const int64_t iters = rate > 0.0 ? (int64_t)std::ceil((std::log(eps) - std::log(2.0)) / std::log(rate)) + 1 : 1;
    al.resize((size_t)iters);
    be.resize((size_t)iters);
    double alpha = 0.0, beta = 0.0;
    for (int64_t k = 0; k < iters; ++k) {
        if (k == 0) { beta = 0.0; alpha = 1.0 / d; }
        else if (k == 1) { beta = 0.5 * (c / d) * (c / d); alpha = 1.0 / (d - c * c / (2.0 * d)); }
        else { beta = (alpha * c / 2.0) * (alpha * c / 2.0); alpha = 1.0 / (d - alpha * c * c / 4.0); }
        al[(size_t)k] = alpha;
        be[(size_t)k] = beta;
    }
}

// The check after a Chebyshev run (Alg. 3), which is exact only when the
// singular values of the preconditioned operator K lie in [sigma_L,
// sigma_U] -- Theorem 3 gives that with a probability, not always.  Within
// the bounds the gradient of the normal equations after the run is the
// Chebyshev residual polynomial applied to the starting one, of norm at
// most eps times it (tall: g = K^T r against g0 = K^T b^; fat: the residual
// of the consistent K x = c against c).  The run passes when
//   ||g|| <= 2 max(eps, 2^-27) ||g0||;
// the floor 2^-27 (about sqrt(u)) stays above the rounding of the products
// K y = A (N y), whose relative size grows with kappa(A), while a run
// outside the bounds grows the gradient instead of shrinking it.
bool cs_passes(double gn, double g0, double eps) {
    const double floor_rel = std::ldexp(1.0, -27);
    return std::isfinite(gn) && gn <= 2.0 * std::max(eps, floor_rel) * g0;
}

double host_norm(const double *d, int64_t n, hipStream_t st);

constexpr int CHUNK = 8;  // iterations enqueued between convergence checks

// ---- tall: K = [A; lambda I] N
struct TallSolver {
    Ctx &cx;
    int64_t M, r;  // long length (rows + Tikhonov rows), short length
    DevBuf ulong, v, wdir, y, t, wN;

    explicit TallSolver(Ctx &c) : cx(c) {
        M = cx.pb.rows + (cx.pb.lambda > 0.0 ? cx.pb.cols : 0);
        r = cx.pb.r;
        ulong.alloc((size_t)M * sizeof(double));
        v.alloc((size_t)r * sizeof(double));
        wdir.alloc((size_t)r * sizeof(double));
        y.alloc((size_t)r * sizeof(double));
        t.alloc((size_t)r * sizeof(double));
        wN.alloc((size_t)cx.L * sizeof(double));
    }

    void load_rhs(const double *b) {
        LSRN_HIP(hipMemcpyAsync(ulong.as<double>(), b, (size_t)cx.pb.rows * sizeof(double),
                                hipMemcpyDeviceToDevice, cx.st));
        if (M > cx.pb.rows)
            fill_kernel<<<grid1(M - cx.pb.rows), 256, 0, cx.st>>>(M - cx.pb.rows, 0.0,
                                                                  ulong.as<double>() + cx.pb.rows);
    }

    // t = N^T [A; lambda I]^T u
    void at(const double *ulong_in) {
        cx.sweep(OP_ATB, nullptr, const_cast<double *>(ulong_in), nullptr, nullptr);
        cx.gemv(cx.Ptp, cx.L, r, cx.L, cx.z.as<double>(), t.as<double>());
    }

    int64_t lsqr(int64_t maxiter, double tol, bool &converged) {
        const size_t mk = cx.prof_mark();
        cx.reset_state((int)maxiter);
        at(ulong.as<double>());
        lsqr_tall_init_kernel<<<1, SNT, 0, cx.st>>>(t.as<double>(), r, v.as<double>(),
                                                    wdir.as<double>(), y.as<double>(), cx.state);
        LSRN_HIP(hipGetLastError());
        State h = cx.host_state();
        GraphExec graph;
        while (!h.done) {
            cx.run_chunk(graph.g, [&] {
                for (int k = 0; k < CHUNK; ++k) {
                    cx.gemv(cx.pb.P, cx.pb.ldp, cx.L, r, v.as<double>(), wN.as<double>());
                    cx.sweep(OP_LSQR_TALL, wN.as<double>(), ulong.as<double>(), nullptr, nullptr);
                    cx.gemv(cx.Ptp, cx.L, r, cx.L, cx.z.as<double>(), t.as<double>());
                    lsqr_tall_step_kernel<<<1, SNT, 0, cx.st>>>(t.as<double>(), r, v.as<double>(),
                                                                wdir.as<double>(), y.as<double>(),
                                                                tol, cx.state);
                }
                LSRN_HIP(hipGetLastError());
            });
            h = cx.host_state();
        }
        cx.prof_keep(mk, 1 + h.iters);  // the start sweep and one per iteration
        converged = h.converged != 0;
        return h.iters;
    }

    // Alg. 3 on K y = b^ (K = [A; lambda I] N).  With `checked`, the result
    // is tested afterwards (cs_passes) and, if the test fails, LSQR is
    // restarted from it; `fell_back` reports that.
    int64_t cs(const double *b, double sl, double su, double eps, bool checked, int64_t maxiter,
               double tol, bool &converged, bool &fell_back) {
        std::vector<double> al, be;
        cs_schedule(sl, su, eps, al, be);
        cx.reset_state(0);
        // r = b^, t = K^T r; v = 0, y = 0
        const double bn = checked ? host_norm(ulong.as<double>(), M, cx.st) : 0.0;
        at(ulong.as<double>());
        const double g0 = checked ? host_norm(t.as<double>(), r, cx.st) : 0.0;
        fill_kernel<<<grid1(r), 256, 0, cx.st>>>(r, 0.0, v.as<double>());
        fill_kernel<<<grid1(r), 256, 0, cx.st>>>(r, 0.0, y.as<double>());
        for (size_t k = 0; k < al.size(); ++k) {
            cs_short_kernel<<<grid1(r), 256, 0, cx.st>>>(r, v.as<double>(), t.as<double>(),
                                                         y.as<double>(), al[k], be[k]);
            cx.gemv(cx.pb.P, cx.pb.ldp, cx.L, r, v.as<double>(), wN.as<double>());
            const bool last = k + 1 == al.size();
            cx.sweep(OP_CS_TALL, wN.as<double>(), ulong.as<double>(), nullptr, nullptr, al[k]);
            if (!last) cx.gemv(cx.Ptp, cx.L, r, cx.L, cx.z.as<double>(), t.as<double>());
        }
        LSRN_HIP(hipGetLastError());
        converged = true;
        fell_back = false;
        const int64_t iters = (int64_t)al.size();
        if (!checked) return iters;
        // the last sweep left z = T^T r (r = b^ - K y, the recurrence's
        // residual in ulong) and ||r||^2 in acc0: g = K^T r costs one gemv
        cx.gemv(cx.Ptp, cx.L, r, cx.L, cx.z.as<double>(), t.as<double>(), false);
        const double gn = host_norm(t.as<double>(), r, cx.st);
        if (cs_passes(gn, g0, eps)) return iters;
        const double rn = std::sqrt(std::max(0.0, cx.host_state().acc[0]));
        // LSQR on K dy = r from dy = 0 (ulong holds r), then y += dy; a
        // divergent run (residual above ||b^||) is dropped: y = 0, r = b^
        fell_back = true;
        DevBuf ycs((size_t)r * sizeof(double));
        if (std::isfinite(rn) && rn <= bn) {
            LSRN_HIP(hipMemcpyAsync(ycs.as<double>(), y.as<double>(), (size_t)r * sizeof(double),
                                    hipMemcpyDeviceToDevice, cx.st));
        } else {
            fill_kernel<<<grid1(r), 256, 0, cx.st>>>(r, 0.0, ycs.as<double>());
            load_rhs(b);
        }
        const int64_t more = lsqr(maxiter, tol, converged);
        axpby_kernel<<<grid1(r), 256, 0, cx.st>>>(r, 1.0, ycs.as<double>(), 1.0, y.as<double>());
        LSRN_HIP(hipGetLastError());
        LSRN_HIP(hipStreamSynchronize(cx.st));  // before ycs is freed
        return iters + more;
    }

    void x_from_y(double *x) { cx.gemv(cx.pb.P, cx.pb.ldp, cx.L, r, y.as<double>(), x, false); }
};

// ---- fat: K = M^T A, T = A^T (rows = n)
struct FatSolver {
    Ctx &cx;
    int64_t n, r;
    DevBuf vt, wdir, u, t, wM;
    double *x;

    // xout holds rows (+ L with Tikhonov rows) entries: x, or x^ = [x; rho]
    FatSolver(Ctx &c, double *xout) : cx(c), x(xout) {
        n = cx.pb.rows + (cx.pb.lambda > 0.0 ? cx.L : 0);
        r = cx.pb.r;
        vt.alloc((size_t)n * sizeof(double));
        wdir.alloc((size_t)n * sizeof(double));
        u.alloc((size_t)r * sizeof(double));
        t.alloc((size_t)r * sizeof(double));
        wM.alloc((size_t)cx.L * sizeof(double));
    }

    // LSQR on M^T A x = c with c given in t.
    int64_t lsqr(int64_t maxiter, double tol, bool &converged) {
        fill_kernel<<<grid1(n), 256, 0, cx.st>>>(n, 0.0, x);
        fill_kernel<<<grid1(n), 256, 0, cx.st>>>(n, 0.0, vt.as<double>());
        const size_t mk = cx.prof_mark();
        cx.reset_state((int)maxiter);
        lsqr_fat_init_kernel<<<1, SNT, 0, cx.st>>>(t.as<double>(), r, u.as<double>(), cx.state);
        // start sweep: v~_1 = A^T M u_1
        cx.gemv(cx.pb.P, cx.pb.ldp, cx.L, r, u.as<double>(), wM.as<double>());
        cx.sweep(OP_LSQR_FAT, wM.as<double>(), vt.as<double>(), x, wdir.as<double>());
        cx.gemv(cx.Ptp, cx.L, r, cx.L, cx.z.as<double>(), t.as<double>());
        lsqr_fat_step_kernel<<<1, SNT, 0, cx.st>>>(t.as<double>(), r, u.as<double>(), 1, tol, cx.state);
        LSRN_HIP(hipGetLastError());
        State h = cx.host_state();
        GraphExec graph;
        while (!h.done) {
            cx.run_chunk(graph.g, [&] {
                for (int k = 0; k < CHUNK; ++k) {
                    cx.gemv(cx.pb.P, cx.pb.ldp, cx.L, r, u.as<double>(), wM.as<double>());
                    cx.sweep(OP_LSQR_FAT, wM.as<double>(), vt.as<double>(), x, wdir.as<double>());
                    cx.gemv(cx.Ptp, cx.L, r, cx.L, cx.z.as<double>(), t.as<double>());
                    lsqr_fat_step_kernel<<<1, SNT, 0, cx.st>>>(t.as<double>(), r, u.as<double>(), 0,
                                                               tol, cx.state);
                }
                LSRN_HIP(hipGetLastError());
            });
            h = cx.host_state();
        }
        cx.prof_keep(mk, 1 + h.iters);  // the start sweep and one per iteration
        lsqr_fat_finish_kernel<<<grid1(n), 256, 0, cx.st>>>(n, x, wdir.as<double>(), cx.state);
        LSRN_HIP(hipGetLastError());
        converged = h.converged != 0;
        return h.iters;
    }

    // Alg. 3 on M^T A x = c (c in t): x, v long; residual short.  With
    // `checked`, the short residual is tested afterwards (cs_passes) and, if
    // the test fails, LSQR is restarted from x; `fell_back` reports that.
    int64_t cs(double sl, double su, double eps, bool checked, int64_t maxiter, double tol,
               bool &converged, bool &fell_back) {
        std::vector<double> al, be;
        cs_schedule(sl, su, eps, al, be);
        cx.reset_state(0);
        fill_kernel<<<grid1(n), 256, 0, cx.st>>>(n, 0.0, x);
        fill_kernel<<<grid1(n), 256, 0, cx.st>>>(n, 0.0, vt.as<double>());
        double *res = u.as<double>();
        LSRN_HIP(hipMemcpyAsync(res, t.as<double>(), (size_t)r * sizeof(double),
                                hipMemcpyDeviceToDevice, cx.st));
        const double c0 = checked ? host_norm(res, r, cx.st) : 0.0;
        DevBuf csave(checked ? (size_t)r * sizeof(double) : 0);
        if (checked)
            LSRN_HIP(hipMemcpyAsync(csave.as<double>(), res, (size_t)r * sizeof(double),
                                    hipMemcpyDeviceToDevice, cx.st));
        for (size_t k = 0; k < al.size(); ++k) {
            cx.gemv(cx.pb.P, cx.pb.ldp, cx.L, r, res, wM.as<double>());
            cx.sweep(OP_CS_FAT, wM.as<double>(), vt.as<double>(), x, nullptr, al[k], be[k]);
            cx.gemv(cx.Ptp, cx.L, r, cx.L, cx.z.as<double>(), t.as<double>());
            axpby_kernel<<<grid1(r), 256, 0, cx.st>>>(r, -al[k], t.as<double>(), 1.0, res);
        }
        LSRN_HIP(hipGetLastError());
        converged = true;
        fell_back = false;
        const int64_t iters = (int64_t)al.size();
        if (!checked) return iters;
        // K x = c is consistent: the residual c - K x (by the recurrence, in
        // res) is what the Chebyshev polynomial bounds
        const double rn = host_norm(res, r, cx.st);
        if (cs_passes(rn, c0, eps)) return iters;
        // LSQR on K dx = res from dx = 0, then x += dx; a divergent run
        // (residual above ||c||) is dropped: x = 0 and LSQR solves K x = c
        fell_back = true;
        DevBuf xcs((size_t)n * sizeof(double));
        const bool keep = std::isfinite(rn) && rn <= c0;
        if (keep)
            LSRN_HIP(hipMemcpyAsync(xcs.as<double>(), x, (size_t)n * sizeof(double),
                                    hipMemcpyDeviceToDevice, cx.st));
        else
            fill_kernel<<<grid1(n), 256, 0, cx.st>>>(n, 0.0, xcs.as<double>());
        LSRN_HIP(hipMemcpyAsync(t.as<double>(), keep ? res : csave.as<double>(),
                                (size_t)r * sizeof(double), hipMemcpyDeviceToDevice, cx.st));
        const int64_t more = lsqr(maxiter, tol, converged);
        axpby_kernel<<<grid1(n), 256, 0, cx.st>>>(n, 1.0, xcs.as<double>(), 1.0, x);
        LSRN_HIP(hipGetLastError());
        LSRN_HIP(hipStreamSynchronize(cx.st));  // before xcs is freed
        return iters + more;
    }
};

// The residual passes read the FP64 T, or the FP32 T when the problem's
// matrix is stored in FP32 (then its values are exact in FP64).
template <int CPT>
void launch_resid_tall(Ctx &cx, const double *b, const double *x, double *hi, double *lo) {
    if (cx.pb.T)
        resid_dd_tall_kernel<CPT, double><<<cx.nblocks, NT, 0, cx.st>>>(
            cx.pb.T, cx.pb.ldt, cx.pb.rows, cx.L, cx.nblocks, cx.rows_per_block, b, x, cx.pb.lambda, hi, lo);
    else
        resid_dd_tall_kernel<CPT, float><<<cx.nblocks, NT, 0, cx.st>>>(
            cx.pb.T32, cx.pb.ldt, cx.pb.rows, cx.L, cx.nblocks, cx.rows_per_block, b, x, cx.pb.lambda, hi, lo);
}

template <int CPT>
void launch_ax_fat(Ctx &cx, const double *x, double *hi, double *lo) {
    if (cx.pb.T)
        ax_dd_fat_kernel<CPT, double><<<cx.nblocks, NT, 0, cx.st>>>(cx.pb.T, cx.pb.ldt, cx.pb.rows, cx.L,
                                                                    cx.rows_per_block, x, hi, lo);
    else
        ax_dd_fat_kernel<CPT, float><<<cx.nblocks, NT, 0, cx.st>>>(cx.pb.T32, cx.pb.ldt, cx.pb.rows, cx.L,
                                                                   cx.rows_per_block, x, hi, lo);
}

double host_norm(const double *d, int64_t n, hipStream_t st) {
    std::vector<double> h((size_t)n);
    LSRN_HIP(hipMemcpyAsync(h.data(), d, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st));
    LSRN_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (double v : h) s += v * v;
    return std::sqrt(s);
}

}  // namespace

namespace {

IterResult iterate_on(const IterProblem &pb, const double *b, double *x, const lsrn_options &opt,
                      hipStream_t st) {
    IterResult res;
    Ctx cx(pb, st, opt.autotune != 0);
    cx.profile = opt.profile != 0;
    // the caller's products of an operator may do anything on the stream
    cx.use_graphs = !cx.profile && st != nullptr && graphs_allowed() && !pb.op;
    double sl = 0.0, su = 0.0;
    const int64_t maxiter = default_maxiter(pb, opt, sl, su);
    res.sigma_l = sl;
    res.sigma_u = su;
    const bool cs = opt.method == LSRN_CHEBYSHEV;
    if (cs && su <= 0.0)
        fail(LSRN_E_UNSUPPORTED, "Chebyshev bounds need sqrt(s) - sqrt(r) - t > 0");

    hipEvent_t e0, e1, e2;
    LSRN_HIP(hipEventCreate(&e0));
    LSRN_HIP(hipEventCreate(&e1));
    LSRN_HIP(hipEventCreate(&e2));
    LSRN_HIP(hipEventRecord(e0, st));
    const int64_t L = pb.cols, r = pb.r;
    bool conv = true;

    if (pb.tall) {
        TallSolver ts(cx);
        ts.load_rhs(b);
        // the precision form's main solve runs on fl32(A): no point in going
        // below 1e-8 before the refinement
        // the precision form: FP32 sweeps solve the problem of fl32(A), and
        // refinement with them contracts only while kappa(A) 2^-24 << 1.
        // The sketch's sigma_max / sigma_min_kept (at most about
        // (1 + sqrt(r/s)) / (1 - sqrt(r/s)) times kappa(A), Sec. 4.2) over
        // 2^24 above 1/2 means they cannot: the sweeps then read the FP64 A
        // from the start and only the sketch stays BF16.
        if (pb.T && pb.T32 && pb.kappa_sketch * std::ldexp(1.0, -24) > 0.5) cx.force_f64 = true;
        const double tol_main = (pb.T && pb.T32 && !cx.force_f64) ? std::max(opt.tol, 1e-8) : opt.tol;
        bool fb = false;
        // a restart after a failed check gets a cap not taken from the bounds
        // the check found wrong
        const int64_t cap_fb = opt.max_iter > 0 ? opt.max_iter : 4 * maxiter;
        res.iters = cs ? ts.cs(b, sl, su, opt.tol, true, cap_fb, opt.tol, conv, fb)
                       : ts.lsqr(maxiter, tol_main, conv);
        res.cs_fallbacks += fb ? 1 : 0;
        ts.x_from_y(x);
        LSRN_HIP(hipEventRecord(e1, st));
        LSRN_HIP(hipStreamSynchronize(st));
        // refinement: (A N)^T (A N) dy = N^T h, h = A^T (b - A x) - lambda^2 x in dd
        if (opt.refine > 0) {
            const int64_t total = pb.rows + (pb.lambda > 0.0 ? L : 0);
            const size_t hlen = pb.sp ? (size_t)total : (size_t)cx.nblocks * L;
            DevBuf hhi(hlen * sizeof(double)), hlo(hlen * sizeof(double));
            DevBuf h((size_t)L * sizeof(double)), c((size_t)r * sizeof(double));
            DevBuf zc((size_t)r * sizeof(double)), rc((size_t)r * sizeof(double)), pc((size_t)r * sizeof(double));
            DevBuf dx((size_t)L * sizeof(double));
            // the sparse normal-equation sweep stores T p here for its column pass
            DevBuf ybuf(pb.sp ? (size_t)(pb.rows + L) * sizeof(double) : 0);
            GraphExec cg_graph;  // the CG chunk keeps its buffers across refinement steps
            bool refine_conv = true;
            double dn_prev = 0.0;
            // the precision form: once its FP32 sweeps stop shrinking the
            // corrections (or the step budget is spent) the refinement goes on
            // with sweeps over the FP64 A, a few steps more at most
            int budget = opt.refine;
            for (int step = 0; step < budget; ++step) {
                if (pb.sp) {
                    // rows: res = b^ - T^ x (dd); columns: h = T^^T res (dd), rounded
                    csr_resid_rows_dd_kernel<<<cx.nblocks, CRP_NT, 0, st>>>(
                        pb.sp->rows, pb.rows, total, cx.rows_per_block, b, x, pb.lambda,
                        hhi.as<double>(), hlo.as<double>());
                    csr_col_pass_dd_kernel<<<(unsigned)ceil_div(L, CCP_NT / 64), CCP_NT, 0, st>>>(
                        pb.sp->cols, hhi.as<double>(), hlo.as<double>(), pb.lambda, pb.rows,
                        h.as<double>(), nullptr);
                    LSRN_HIP(hipGetLastError());
                } else {
                    if (cx.cpt == 2) launch_resid_tall<2>(cx, b, x, hhi.as<double>(), hlo.as<double>());
                    else if (cx.cpt == 4) launch_resid_tall<4>(cx, b, x, hhi.as<double>(), hlo.as<double>());
                    else if (cx.cpt == 8) launch_resid_tall<8>(cx, b, x, hhi.as<double>(), hlo.as<double>());
                    else launch_resid_tall<16>(cx, b, x, hhi.as<double>(), hlo.as<double>());
                    LSRN_HIP(hipGetLastError());
                    reduce_dd_kernel<<<(unsigned)ceil_div(L, 256), 256, 0, st>>>(
                        hhi.as<double>(), hlo.as<double>(), cx.nblocks, (int)L, nullptr, h.as<double>(), nullptr);
                }
                cx.gemv(cx.Ptp, L, r, L, h.as<double>(), c.as<double>(), false);
                const int cg_max = 200;
                cg_init_kernel<<<1, SNT, 0, st>>>(c.as<double>(), r, zc.as<double>(), rc.as<double>(),
                                                  pc.as<double>(), opt.refine_tol, cg_max, cx.state);
                State hs = cx.host_state();
                const size_t mk = cx.prof_mark();
                while (!hs.done) {
                    cx.run_chunk(cg_graph.g, [&] {
                        for (int k = 0; k < CHUNK; ++k) {
                            cx.gemv(pb.P, pb.ldp, L, r, pc.as<double>(), ts.wN.as<double>());
                            cx.sweep(OP_NORMAL, ts.wN.as<double>(), ybuf.as<double>(), nullptr, nullptr);
                            cx.gemv(cx.Ptp, L, r, L, cx.z.as<double>(), ts.t.as<double>());
                            cg_step_kernel<<<1, SNT, 0, st>>>(ts.t.as<double>(), r, zc.as<double>(),
                                                              rc.as<double>(), pc.as<double>(),
                                                              cx.state);
                        }
                        LSRN_HIP(hipGetLastError());
                    });
                    hs = cx.host_state();
                }
                cx.prof_keep(mk, hs.iters);
                res.refine_iters += hs.iters;
                refine_conv = hs.converged != 0;
                cx.gemv(pb.P, pb.ldp, L, r, zc.as<double>(), dx.as<double>(), false);
                axpby_kernel<<<grid1(L), 256, 0, st>>>(L, 1.0, dx.as<double>(), 1.0, x);
                LSRN_HIP(hipGetLastError());
                ++res.refine_steps;
                if (cx.force_f64) ++res.fp64_refine_steps;
                const double dn = host_norm(dx.as<double>(), L, st), xn = host_norm(x, L, st);
                const bool stalled = step > 0 && dn > 0.5 * dn_prev;
                dn_prev = dn;
                if (pb.T && pb.T32) {
                    // the precision form's main LSQR runs on fl32(A): its
                    // answer is settled by the refinement, whose last
                    // correction must have become negligible
                    conv = dn <= std::max(opt.tol, 1e-12) * xn;
                    if (conv) break;
                    if (!cx.force_f64 && (stalled || step + 1 == budget)) {
                        cx.force_f64 = true;
                        if (cg_graph.g) {
                            LSRN_HIP(hipGraphExecDestroy(cg_graph.g));
                            cg_graph.g = nullptr;
                        }
                        budget = step + 1 + 3;
                        dn_prev = std::numeric_limits<double>::infinity();
                        continue;
                    }
                    if (cx.force_f64 && stalled) break;
                    continue;
                }
                // stop at convergence, or once the corrections stop shrinking
                // (the floor of the inner arithmetic is reached)
                if (dn <= 1e-15 * xn || stalled) break;
            }
            // with refinement the answer is the refined one: the solve has
            // converged when the last correction's solve met its rule, even
            // if the main LSQR stopped at its cap (at kappa(A) near 1/u^(1/2)
            // its normal-equation test can sit at the rounding floor)
            if (!(pb.T && pb.T32)) conv = refine_conv;
        }
        LSRN_HIP(hipStreamSynchronize(st));  // before the solver's buffers are freed
    } else {
        // with lambda > 0 (the under-determined Tikhonov form [A, lambda I_m],
        // Sec. 5) the unknown is x^ = [x; rho], rows + L long; x is its head
        const int64_t nl = pb.rows + (pb.lambda > 0.0 ? L : 0);
        DevBuf xhat(nl > pb.rows ? (size_t)nl * sizeof(double) : 0);
        double *const xh = nl > pb.rows ? xhat.as<double>() : x;
        FatSolver fs(cx, xh);
        // c = M^T b
        cx.gemv(cx.Ptp, L, r, L, b, fs.t.as<double>(), false);
        bool fb = false;
        const int64_t cap_fb = opt.max_iter > 0 ? opt.max_iter : 4 * maxiter;
        res.iters = cs ? fs.cs(sl, su, opt.tol, true, cap_fb, opt.tol, conv, fb)
                       : fs.lsqr(maxiter, opt.tol, conv);
        res.cs_fallbacks += fb ? 1 : 0;
        LSRN_HIP(hipEventRecord(e1, st));
        if (opt.refine > 0) {
            const int64_t n = nl;
            double *const x = xh;
            const size_t zlen = pb.sp ? (size_t)L : (size_t)cx.nblocks * L;
            DevBuf zhi(zlen * sizeof(double)), zlo(zlen * sizeof(double));
            DevBuf thi((size_t)L * sizeof(double)), tlo((size_t)L * sizeof(double));
            DevBuf xsave((size_t)n * sizeof(double));
            double dn_prev = 0.0;
            for (int step = 0; step < opt.refine; ++step) {
                if (pb.sp) {
                    // A x (+ lambda rho) per row of A, in double-double
                    csr_col_pass_dd_kernel<<<(unsigned)ceil_div(L, CCP_NT / 64), CCP_NT, 0, st>>>(
                        pb.sp->cols, x, nullptr, pb.lambda, pb.rows, zhi.as<double>(), zlo.as<double>());
                } else {
                    if (cx.cpt == 2) launch_ax_fat<2>(cx, x, zhi.as<double>(), zlo.as<double>());
                    else if (cx.cpt == 4) launch_ax_fat<4>(cx, x, zhi.as<double>(), zlo.as<double>());
                    else if (cx.cpt == 8) launch_ax_fat<8>(cx, x, zhi.as<double>(), zlo.as<double>());
                    else launch_ax_fat<16>(cx, x, zhi.as<double>(), zlo.as<double>());
                }
                LSRN_HIP(hipGetLastError());
                const bool add_rho = !pb.sp && pb.lambda > 0.0;
                reduce_dd_kernel<<<(unsigned)ceil_div(L, 256), 256, 0, st>>>(
                    zhi.as<double>(), zlo.as<double>(), pb.sp ? 1 : cx.nblocks, (int)L, b,
                    thi.as<double>(), tlo.as<double>(), pb.lambda, add_rho ? x + pb.rows : nullptr);
                // e = M^T (b - A x - lambda rho) with dd accumulation
                gemv_t_dd_kernel<<<(unsigned)ceil_div(r, 4), 256, 0, st>>>(
                    pb.P, pb.ldp, L, r, thi.as<double>(), tlo.as<double>(), fs.t.as<double>());
                LSRN_HIP(hipGetLastError());
                LSRN_HIP(hipMemcpyAsync(xsave.as<double>(), x, (size_t)n * sizeof(double),
                                        hipMemcpyDeviceToDevice, st));
                bool c2 = true;
                // the correction needs only refine_tol relative accuracy:
                // the error left after it is that times the error before
                const double ctol = std::max(opt.tol, opt.refine_tol);
                bool fb2 = false;
                res.refine_iters += cs ? fs.cs(sl, su, ctol, true, cap_fb, ctol, c2, fb2)
                                       : fs.lsqr(maxiter, ctol, c2);
                res.cs_fallbacks += fb2 ? 1 : 0;
                conv = c2;  // the refined answer: its last correction's solve decides
                // fs wrote the correction into x; x = xsave + dx
                const double dn = host_norm(x, n, st);
                axpby_kernel<<<grid1(n), 256, 0, st>>>(n, 1.0, xsave.as<double>(), 1.0, x);
                LSRN_HIP(hipGetLastError());
                ++res.refine_steps;
                const double xn = host_norm(x, n, st);
                // stop at convergence, or once the corrections stop shrinking
                // (the floor of the inner arithmetic is reached)
                if (dn <= 1e-15 * xn || (step > 0 && dn > 0.5 * dn_prev)) break;
                dn_prev = dn;
            }
        }
        if (xh != x)
            LSRN_HIP(hipMemcpyAsync(x, xh, (size_t)pb.rows * sizeof(double), hipMemcpyDeviceToDevice, st));
        LSRN_HIP(hipStreamSynchronize(st));  // before the solver's buffers are freed
    }
    LSRN_HIP(hipEventRecord(e2, st));
    LSRN_HIP(hipEventSynchronize(e2));
    float ms1 = 0.f, ms2 = 0.f;
    LSRN_HIP(hipEventElapsedTime(&ms1, e0, e1));
    LSRN_HIP(hipEventElapsedTime(&ms2, e1, e2));
    res.t_iter_ms = ms1;
    res.t_refine_ms = ms2;
    res.converged = conv;
    if (cx.profile) {
        res.t_sweep_kernel_ms = cx.sweep_kernel_ms();
        res.sweep_kernels = (int64_t)cx.ev.size() / 2;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    return res;
}

}  // namespace

IterResult iterate(const IterProblem &pb, const double *b, double *x, const lsrn_options &opt,
                   hipStream_t st) {
    // an operator's products are promised the caller's stream, and its
    // iterations are never captured
    if (st || pb.op) return iterate_on(pb, b, x, opt, st);
    // the null stream cannot be captured into graphs: run on a stream of our
    // own (default priority) after the caller's work on the null stream
    LSRN_HIP(hipStreamSynchronize(nullptr));
    hipStream_t own = nullptr;
    LSRN_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    try {
        IterResult r = iterate_on(pb, b, x, opt, own);
        LSRN_HIP(hipStreamSynchronize(own));
        (void)hipStreamDestroy(own);
        return r;
    } catch (...) {
        (void)hipStreamSynchronize(own);
        (void)hipStreamDestroy(own);
        throw;
    }
}

void OpView::apply_t(int t, int64_t k, const double *in, int64_t ldin, double *out, int64_t ldout,
                     hipStream_t st) const {
    // T = A (m >= n) or A^T: T in is A in or A^T in
    const int trans = (m >= n) ? t : 1 - t;
    if (fn(ctx, trans, k, in, ldin, out, ldout, (void *)st) != 0)
        fail(LSRN_E_INVALID, "the operator's product routine returned an error");
    LSRN_HIP(hipGetLastError());
}

// ------------------------------------------------------- batched LSQR
//
// Many tall problems with min(m, n) <= 512 iterate together: every launch
// below covers the whole batch, one work item per (problem, row block),
// (problem, column chunk), (problem, row group) or problem, found from a
// prefix table; a problem whose done flag is set leaves the work items of
// its kernels empty.  One chunk of iterations (five launches each) is
// replayed as a HIP graph.

namespace {

constexpr int BCPT = 2, BR = 8;          // the sweep variant for L <= 512
constexpr int B_RED_COLS = 32;           // columns of z per reduction workgroup
constexpr int B_RED_GROUPS = 256 / B_RED_COLS;  // partial groups per reduction workgroup
constexpr int B_CHUNK = 16;  // batched iterations enqueued between done-flag checks

// Rows per workgroup of a problem's batched sweeps, from its own row count
// alone (so its bits do not depend on the rest of the batch): about 512
// workgroups for a tall problem, 128 to 512 rows each (fewer rows left the
// per-workgroup set-up dominant on problems of a few thousand rows).
int64_t batch_rows_per_block(int64_t rows) {
    return std::min<int64_t>(512, std::max<int64_t>(128, round_up(ceil_div(rows, 512), 64)));
}

struct BatchItem {
    SweepArgs sw;  // T, ldt, rows, L, nblocks, rows_per_block, w = wN, zpart, spart, y = u, st
    const double *P;
    int64_t ldp;
    const double *Pt;  // r x L
    int64_t r, L;
    double *v, *wdir, *yv, *t, *z, *x;
    double tol;
    int lpr;  // lanes per row of the narrow sweep (0: the wide sweep)
    // refinement: the right-hand side, h = A^T (b - A x) (double-double
    // partials per row block, then rounded), c = N^T h, and the CG vectors
    const double *bvec;
    double *hhi, *hlo, *h, *c, *zc, *rc, *pc;
    double rtol;
    int refine;  // this problem's refinement steps (its buffers exist only if > 0)
    // Chebyshev (Alg. 3): cs = 1, the run's ncs steps (alpha_k at sched[k],
    // beta_k at sched[ncs + k]), the iterate kept for an LSQR restart, and
    // csn = {|N^T A^T b|, |N^T A^T r| after the run, |b|} for the check
    int cs, ncs;
    const double *sched;
    double *ycs, *csn;
};

__device__ __forceinline__ int find_item(const int *__restrict__ off, int n, int g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int OP>
__global__ void __launch_bounds__(NT, 2)
batch_sweep_kernel(const BatchItem *__restrict__ it, const int *__restrict__ off, int n) {
    __shared__ double zred[(NT / 64) * 64 * 8];
    __shared__ double accred[NT / 64];
    const int p = find_item(off, n, (int)blockIdx.x);
    const int blk = (int)blockIdx.x - off[p];
    switch (it[p].lpr) {
        case 2: sweep_narrow_body<2, OP>(it[p].sw, blk, zred, accred); break;
        case 4: sweep_narrow_body<4, OP>(it[p].sw, blk, zred, accred); break;
        case 8: sweep_narrow_body<8, OP>(it[p].sw, blk, zred, accred); break;
        case 16: sweep_narrow_body<16, OP>(it[p].sw, blk, zred, accred); break;
        case 32: sweep_narrow_body<32, OP>(it[p].sw, blk, zred, accred); break;
        case 64: sweep_narrow_body<64, OP>(it[p].sw, blk, zred, accred); break;
        default: sweep_body<BCPT, BR, OP, false>(it[p].sw, blk); break;
    }
}

// Sum over the partials k = g, g + 8, ... of column col: four independent
// chains (k = g + 8 (4 q + u), u = 0..3), added as (c0 + c1) + (c2 + c3).
__device__ __forceinline__ double batch_col_sum(const double *__restrict__ zp, int64_t L, int col, int nb,
                                                int g) {
    double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
    constexpr int S = B_RED_GROUPS;
    int k = g;
    for (; k + 3 * S < nb; k += 4 * S) {
        c0 += zp[(int64_t)k * L + col];
        c1 += zp[(int64_t)(k + S) * L + col];
        c2 += zp[(int64_t)(k + 2 * S) * L + col];
        c3 += zp[(int64_t)(k + 3 * S) * L + col];
    }
    if (k < nb) c0 += zp[(int64_t)k * L + col];
    if (k + S < nb) c1 += zp[(int64_t)(k + S) * L + col];
    if (k + 2 * S < nb) c2 += zp[(int64_t)(k + 2 * S) * L + col];
    return (c0 + c1) + (c2 + c3);
}

// z_p = sum of the row-block partials, st_p->acc = sum of the scalar
// partials.  A workgroup takes 32 columns: eight groups of 32 threads sum
// the partials k = g mod 8 (batch_col_sum), then the eight sums are added
// in order g = 0..7; the first workgroup of a problem also sums the scalar
// partials (64 threads a scalar, k = q mod 64, added in order q = 0..63).
__global__ void __launch_bounds__(256)
batch_reduce_kernel(const BatchItem *__restrict__ it, const int *__restrict__ off, int n) {
    __shared__ double red[B_RED_GROUPS][B_RED_COLS];
    __shared__ double sred[64][4];
    const int p = find_item(off, n, (int)blockIdx.x);
    const BatchItem &b = it[p];
    if (b.sw.st->done) return;
    const int chunk = (int)blockIdx.x - off[p];
    const int c = threadIdx.x % B_RED_COLS, g = threadIdx.x / B_RED_COLS;
    const int col = chunk * B_RED_COLS + c;
    const int nb = b.sw.nblocks;
    red[g][c] = col < b.L ? batch_col_sum(b.sw.zpart, b.L, col, nb, g) : 0.0;
    if (chunk == 0) {
        const int a = threadIdx.x & 3, q = threadIdx.x >> 2;
        double u = 0.0;
        for (int k = q; k < nb; k += 64) u += b.sw.spart[k * 4 + a];
        sred[q][a] = u;
    }
    __syncthreads();
    if (g == 0 && col < b.L) {
        double t = red[0][c];
        for (int q = 1; q < B_RED_GROUPS; ++q) t += red[q][c];
        b.z[col] = t;
    }
    if (chunk == 0 && threadIdx.x < 4) {
        double u = 0.0;
        for (int q = 0; q < 64; ++q) u += sred[q][threadIdx.x];
        b.sw.st->acc[threadIdx.x] = u;
    }
}

// which 0: wN = P v; 1: t = P^T z; 2: x = P y; refinement: 3: c = P^T h;
// 4: wN = P p (the CG direction); 5: x += P z (the CG solution).  2, 3 and
// 5 run after the loops, whatever the done flags say.
__global__ void __launch_bounds__(256)
batch_gemv_kernel(const BatchItem *__restrict__ it, const int *__restrict__ off, int n, int which,
                  int step = 0) {
    const int p = find_item(off, n, (int)blockIdx.x);
    const BatchItem &b = it[p];
    if ((which == 0 || which == 1 || which == 4) && b.sw.st->done) return;
    if ((which == 3 || which == 5) && step >= b.refine) return;  // no refinement step `step` here
    const int64_t row = (int64_t)((int)blockIdx.x - off[p]) * 4 + (threadIdx.x >> 6);
    const double *M;
    int64_t ld, nrows, ncols;
    const double *x;
    double *y;
    if (which == 1 || which == 3) {
        M = b.Pt; ld = b.L; nrows = b.r; ncols = b.L;
        x = which == 1 ? b.z : b.h;
        y = which == 1 ? b.t : b.c;
    } else {
        M = b.P; ld = b.ldp; nrows = b.L; ncols = b.r;
        x = which == 0 ? b.v : which == 2 ? b.yv : which == 4 ? b.pc : b.zc;
        y = (which == 0 || which == 4) ? const_cast<double *>(b.sw.w) : b.x;
    }
    if (row >= nrows) return;
    const int lane = threadIdx.x & 63;
    // the row and x through buffer resources of ncols entries: eight loads
    // of each in flight per lane, zeros past the end, and lane l still sums
    // its columns l, l + 64, ... in ascending order
    const int nbytes = (int)(ncols * (int64_t)sizeof(double));
    const __amdgpu_buffer_rsrc_t rm = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double *>(M + row * ld), (short)0, nbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double *>(x), (short)0, nbytes, 0x00020000);
    double t = 0.0;
    for (int64_t c0 = 0; c0 < ncols; c0 += 512) {
        double a[8], b[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int off = (int)(c0 + lane + 64 * k) * 8;
            a[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rm, off, 0, 0));
            b[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rx, off, 0, 0));
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) t += a[k] * b[k];
    }
    t = wave_sum(t);
    if (lane == 0) {
        if (which == 5) y[row] += t;
        else y[row] = t;
    }
}

// h partials of the refinement: per row block of each problem, in double-
// double (the single-problem kernel's body, the row blocks of the sweeps).
__global__ void __launch_bounds__(NT)
batch_resid_kernel(const BatchItem *__restrict__ it, const int *__restrict__ off, int n, int step) {
    const int p = find_item(off, n, (int)blockIdx.x);
    const BatchItem &b = it[p];
    if (step >= b.refine) return;
    const int blk = (int)blockIdx.x - off[p];
    const SweepArgs &a = b.sw;
    __shared__ double rh[NT / 64][8 * 64], rl[NT / 64][8 * 64];  // the narrow bodies' wave sums
    switch (b.lpr) {
        case 2: resid_dd_narrow_body<2>(a.T, a.ldt, a.rows, a.L, a.rows_per_block, b.bvec, b.x, b.hhi, b.hlo, blk, rh, rl); break;
        case 4: resid_dd_narrow_body<4>(a.T, a.ldt, a.rows, a.L, a.rows_per_block, b.bvec, b.x, b.hhi, b.hlo, blk, rh, rl); break;
        case 8: resid_dd_narrow_body<8>(a.T, a.ldt, a.rows, a.L, a.rows_per_block, b.bvec, b.x, b.hhi, b.hlo, blk, rh, rl); break;
        case 16: resid_dd_narrow_body<16>(a.T, a.ldt, a.rows, a.L, a.rows_per_block, b.bvec, b.x, b.hhi, b.hlo, blk, rh, rl); break;
        case 32: resid_dd_narrow_body<32>(a.T, a.ldt, a.rows, a.L, a.rows_per_block, b.bvec, b.x, b.hhi, b.hlo, blk, rh, rl); break;
        case 64: resid_dd_narrow_body<64>(a.T, a.ldt, a.rows, a.L, a.rows_per_block, b.bvec, b.x, b.hhi, b.hlo, blk, rh, rl); break;
        default:
            resid_dd_tall_body<BCPT, double>(a.T, a.ldt, a.rows, a.L, a.nblocks, a.rows_per_block, b.bvec, b.x, 0.0,
                                             b.hhi, b.hlo, blk);
            break;
    }
}

// h = the double-double sum of the row-block partials, rounded.
__global__ void __launch_bounds__(256)
batch_reduce_dd_kernel(const BatchItem *__restrict__ it, const int *__restrict__ off, int n, int step) {
    const int p = find_item(off, n, (int)blockIdx.x);
    __shared__ double rhi[B_RED_GROUPS][B_RED_COLS], rlo[B_RED_GROUPS][B_RED_COLS];
    const BatchItem &b = it[p];
    if (step >= b.refine) return;
    const int c = threadIdx.x % B_RED_COLS, g = threadIdx.x / B_RED_COLS;
    const int col = ((int)blockIdx.x - off[p]) * B_RED_COLS + c;
    dd t = {0.0, 0.0};
    if (col < b.L)
        for (int k = g; k < b.sw.nblocks; k += B_RED_GROUPS)
            t = dd_add(t, dd{b.hhi[(int64_t)k * b.L + col], b.hlo[(int64_t)k * b.L + col]});
    rhi[g][c] = t.hi;
    rlo[g][c] = t.lo;
    __syncthreads();
    if (g == 0 && col < b.L) {
        dd u = {rhi[0][c], rlo[0][c]};
        for (int q = 1; q < B_RED_GROUPS; ++q) u = dd_add(u, dd{rhi[q][c], rlo[q][c]});
        b.h[col] = u.hi;
    }
}

__global__ void __launch_bounds__(SNT) batch_cg_init_kernel(const BatchItem *__restrict__ it, int maxiter,
                                                             int step) {
    const BatchItem &b = it[blockIdx.x];
    if (step >= b.refine) {  // done: the CG launches of this step skip the problem
        if (threadIdx.x == 0) {
            State s0 = {};
            s0.done = 1;
            s0.converged = 1;
            *b.sw.st = s0;
        }
        return;
    }
    cg_init_body(b.c, b.r, b.zc, b.rc, b.pc, b.rtol, maxiter, b.sw.st);
}

__global__ void __launch_bounds__(SNT) batch_cg_step_kernel(const BatchItem *__restrict__ it) {
    const BatchItem &b = it[blockIdx.x];
    cg_step_body(b.t, b.r, b.zc, b.rc, b.pc, b.sw.st);
}

__global__ void __launch_bounds__(SNT) batch_init_kernel(const BatchItem *__restrict__ it) {
    const BatchItem &b = it[blockIdx.x];
    if (b.sw.st->done) return;  // parked: a Chebyshev run that passed its check
    lsqr_tall_init_body(b.t, b.r, b.v, b.wdir, b.yv, b.sw.st);
}

// Start of the Chebyshev phase (t = N^T A^T b already formed): for a
// Chebyshev problem v = y = 0, csn[0] = |t|, csn[2] = |b|; an LSQR problem
// is parked (done) until the LSQR phase.
__global__ void __launch_bounds__(SNT) batch_cs_begin_kernel(const BatchItem *__restrict__ it) {
    __shared__ double scratch[SNT / 64];
    const BatchItem &b = it[blockIdx.x];
    if (!b.cs) {
        if (threadIdx.x == 0) b.sw.st->done = 1;
        return;
    }
    double g = 0.0, q = 0.0;
    for (int64_t i = threadIdx.x; i < b.r; i += SNT) {
        b.v[i] = 0.0;
        b.yv[i] = 0.0;
        g += b.t[i] * b.t[i];
    }
    for (int64_t j = threadIdx.x; j < b.sw.rows; j += SNT) q += b.sw.y[j] * b.sw.y[j];
    g = block_sum<SNT>(g, scratch);
    q = block_sum<SNT>(q, scratch);
    if (threadIdx.x == 0) {
        b.csn[0] = sqrt(g);
        b.csn[2] = sqrt(q);
        b.sw.st->iters = 0;
        b.sw.st->done = 0;
    }
}

// Step k of a Chebyshev run (k = the steps done, from its state): v =
// beta_k v + t, y += alpha_k v, and alpha_k handed to this step's sweep.
__global__ void __launch_bounds__(SNT) batch_cs_short_kernel(const BatchItem *__restrict__ it) {
    const BatchItem &b = it[blockIdx.x];
    if (b.sw.st->done) return;
    const int k = b.sw.st->iters;
    const double al = b.sched[k], be = b.sched[b.ncs + k];
    for (int64_t i = threadIdx.x; i < b.r; i += SNT) {
        const double vi = be * b.v[i] + b.t[i];
        b.v[i] = vi;
        b.yv[i] += al * vi;
    }
    if (threadIdx.x == 0) const_cast<BatchItem *>(it)[blockIdx.x].sw.alpha = al;
}

// After a Chebyshev step's products: one more step done; the last one ends
// the run (t then holds N^T A^T r for the check).
__global__ void batch_cs_step_kernel(const BatchItem *__restrict__ it) {
    const BatchItem &b = it[blockIdx.x];
    State *s = b.sw.st;
    if (s->done) return;
    const int k = s->iters + 1;
    s->iters = k;
    if (k >= b.ncs) {
        s->done = 1;
        s->converged = 1;
    }
}

// csn[1] = |t| = |N^T A^T r| after a Chebyshev run.
__global__ void __launch_bounds__(SNT) batch_cs_norm_kernel(const BatchItem *__restrict__ it) {
    __shared__ double scratch[SNT / 64];
    const BatchItem &b = it[blockIdx.x];
    if (!b.cs) return;
    double g = 0.0;
    for (int64_t i = threadIdx.x; i < b.r; i += SNT) g += b.t[i] * b.t[i];
    g = block_sum<SNT>(g, scratch);
    if (threadIdx.x == 0) b.csn[1] = sqrt(g);
}

// The LSQR phase's start for each problem, by mode: 0 parks it (a
// Chebyshev run that passed its check), 1 starts LSQR on b (an LSQR
// problem), 2 on the Chebyshev residual r (the long vector) after keeping
// y, 3 on b again with the Chebyshev iterate dropped (a divergent run).
__global__ void __launch_bounds__(SNT) batch_lsqr_phase_kernel(const BatchItem *__restrict__ it,
                                                               const int *__restrict__ maxit,
                                                               const int *__restrict__ mode) {
    const BatchItem &b = it[blockIdx.x];
    const int md = mode[blockIdx.x];
    if (md == 0) return;
    if (md == 2)
        for (int64_t i = threadIdx.x; i < b.r; i += SNT) b.ycs[i] = b.yv[i];
    if (md == 3) {
        for (int64_t i = threadIdx.x; i < b.r; i += SNT) b.ycs[i] = 0.0;
        for (int64_t j = threadIdx.x; j < b.sw.rows; j += SNT) b.sw.y[j] = b.bvec[j];
    }
    if (threadIdx.x == 0) {
        State z = {};
        z.maxiter = maxit[blockIdx.x];
        *b.sw.st = z;
    }
}

// y += the kept Chebyshev iterate, for the restarted problems (mode 2, 3).
__global__ void __launch_bounds__(SNT) batch_cs_finish_kernel(const BatchItem *__restrict__ it,
                                                              const int *__restrict__ mode) {
    const BatchItem &b = it[blockIdx.x];
    if (mode[blockIdx.x] < 2) return;
    for (int64_t i = threadIdx.x; i < b.r; i += SNT) b.yv[i] += b.ycs[i];
}

__global__ void __launch_bounds__(SNT) batch_step_kernel(const BatchItem *__restrict__ it) {
    const BatchItem &b = it[blockIdx.x];
    lsqr_tall_step_body(b.t, b.r, b.v, b.wdir, b.yv, b.tol, b.sw.st);
}

__global__ void batch_set_state_kernel(const BatchItem *__restrict__ it, const int *__restrict__ maxit) {
    State z = {};
    z.maxiter = maxit[blockIdx.x];
    *it[blockIdx.x].sw.st = z;
}

}  // namespace

std::vector<IterResult> iterate_batch_tall(const std::vector<IterProblem> &pbs,
                                           const std::vector<const double *> &bs,
                                           const std::vector<double *> &xs,
                                           const std::vector<lsrn_options> &opts, hipStream_t st) {
    const int n = (int)pbs.size();
    LSRN_REQUIRE(opts.size() == pbs.size(), "batched iterations: one option set per problem");
    int nref = 0;  // refinement steps of the batch (the most any problem takes)
    for (const lsrn_options &o : opts) nref = std::max(nref, (int)o.refine);
    std::vector<IterResult> res((size_t)n);
    if (n == 0) return res;
    for (const IterProblem &pb : pbs)
        LSRN_REQUIRE(pb.tall && !pb.sp && !pb.T32 && pb.lambda == 0.0 && pb.cols <= 512,
                     "batched iterations: tall dense FP64 problems with n <= 512");
    // per-problem buffers carved from one allocation (32-double alignment)
    std::vector<BatchItem> items((size_t)n);
    std::vector<int> off_sw(n + 1), off_red(n + 1), off_gP(n + 1), off_gPt(n + 1), maxit(n);
    auto carve = [](size_t elems) { return (std::max<size_t>(elems, 1) + 31) & ~(size_t)31; };
    size_t pool_elems = 0;
    for (int p = 0; p < n; ++p) {
        const IterProblem &pb = pbs[(size_t)p];
        const size_t L = (size_t)pb.cols, r = (size_t)pb.r;
        const size_t nb = (size_t)std::max<int64_t>(1, ceil_div(pb.rows, batch_rows_per_block(pb.rows)));
        pool_elems += carve(nb * L) + carve(nb * 4) + carve((size_t)pb.rows) + carve(L) + carve(r * L) +
                      4 * carve(r) + carve(L);
        if (opts[(size_t)p].refine > 0) pool_elems += 2 * carve(nb * L) + carve(L) + 4 * carve(r);
        if (opts[(size_t)p].method == LSRN_CHEBYSHEV) pool_elems += carve(r) + carve(3);
    }
    // Chebyshev schedules (Alg. 3 from each problem's bounds, Theorem 3)
    std::vector<double> sched_h;
    std::vector<size_t> sched_off((size_t)n, 0);
    std::vector<int> ncs((size_t)n, 0);
    bool any_cs = false;
    for (int p = 0; p < n; ++p) {
        if (opts[(size_t)p].method != LSRN_CHEBYSHEV) continue;
        double sl = 0.0, su = 0.0;
        (void)default_maxiter(pbs[(size_t)p], opts[(size_t)p], sl, su);
        if (su <= 0.0) fail(LSRN_E_UNSUPPORTED, "Chebyshev bounds need sqrt(s) - sqrt(r) - t > 0");
        std::vector<double> al, be;
        cs_schedule(sl, su, opts[(size_t)p].tol, al, be);
        sched_off[(size_t)p] = sched_h.size();
        ncs[(size_t)p] = (int)al.size();
        sched_h.insert(sched_h.end(), al.begin(), al.end());
        sched_h.insert(sched_h.end(), be.begin(), be.end());
        any_cs = true;
    }
    DevBuf dsched(sched_h.size() * sizeof(double));
    if (!sched_h.empty())
        LSRN_HIP(hipMemcpyAsync(dsched.as<double>(), sched_h.data(), sched_h.size() * sizeof(double),
                                hipMemcpyHostToDevice, st));
    DevBuf pool(pool_elems * sizeof(double));
    size_t pool_used = 0;
    auto buf = [&](size_t elems) {
        double *q = pool.as<double>() + pool_used;
        pool_used += carve(elems);
        return q;
    };
    DevBuf states((size_t)n * sizeof(State));
    for (int p = 0; p < n; ++p) {
        const IterProblem &pb = pbs[(size_t)p];
        const lsrn_options &opt = opts[(size_t)p];
        BatchItem &b = items[(size_t)p];
        const int64_t L = pb.cols, r = pb.r;
        const int64_t rpb = batch_rows_per_block(pb.rows);
        const int nblocks = (int)std::max<int64_t>(1, ceil_div(pb.rows, rpb));
        std::memset(&b, 0, sizeof(b));
        b.sw.T = pb.T; b.sw.T32 = nullptr; b.sw.ldt = pb.ldt; b.sw.rows = pb.rows; b.sw.L = (int)L;
        b.sw.nblocks = nblocks; b.sw.rows_per_block = rpb;
        b.sw.zpart = buf((size_t)nblocks * L);
        b.sw.spart = buf((size_t)nblocks * 4);
        b.sw.y = buf((size_t)pb.rows);
        b.sw.st = states.as<State>() + p;
        b.sw.lambda = 0.0;
        double *wN = buf((size_t)L);
        b.sw.w = wN;
        b.P = pb.P; b.ldp = pb.ldp; b.r = r; b.L = L;
        double *Pt = buf((size_t)r * L);
        transpose(L, r, pb.P, pb.ldp, Pt, st);
        b.Pt = Pt;
        b.v = buf((size_t)r); b.wdir = buf((size_t)r); b.yv = buf((size_t)r); b.t = buf((size_t)r);
        b.z = buf((size_t)L); b.x = xs[(size_t)p];
        b.tol = opt.tol;
        b.bvec = bs[(size_t)p];
        b.rtol = opt.refine_tol;
        b.refine = (int)opt.refine;
        if (opt.refine > 0) {
            b.hhi = buf((size_t)nblocks * L); b.hlo = buf((size_t)nblocks * L);
            b.h = buf((size_t)L);
            b.c = buf((size_t)r); b.zc = buf((size_t)r); b.rc = buf((size_t)r); b.pc = buf((size_t)r);
        }
        b.lpr = 0;
        if ((pb.rows + 512) * pb.ldt < ((int64_t)1 << 28))  // offsets stay in 31 bits
            for (int l = 2; l <= 64 && !b.lpr; l *= 2)
                if (L <= 8 * l) b.lpr = l;
        LSRN_HIP(hipMemcpyAsync(b.sw.y, bs[(size_t)p], (size_t)pb.rows * sizeof(double),
                                hipMemcpyDeviceToDevice, st));
        double sl = 0.0, su = 0.0;
        maxit[(size_t)p] = (int)default_maxiter(pb, opt, sl, su);
        res[(size_t)p].sigma_l = sl;
        res[(size_t)p].sigma_u = su;
        if (opt.method == LSRN_CHEBYSHEV) {
            // an LSQR restart after a failed check gets a cap not taken from
            // the bounds the check found wrong (as in the one-problem solve)
            maxit[(size_t)p] = (int)(opt.max_iter > 0 ? opt.max_iter : 4 * (int64_t)maxit[(size_t)p]);
            b.cs = 1;
            b.ncs = ncs[(size_t)p];
            b.sched = dsched.as<double>() + sched_off[(size_t)p];
            b.ycs = buf((size_t)r);
            b.csn = buf(3);
        }
        off_sw[(size_t)p + 1] = off_sw[(size_t)p] + nblocks;
        off_red[(size_t)p + 1] = off_red[(size_t)p] + (int)ceil_div(L, (int64_t)B_RED_COLS);
        off_gP[(size_t)p + 1] = off_gP[(size_t)p] + (int)ceil_div(L, 4);
        off_gPt[(size_t)p + 1] = off_gPt[(size_t)p] + (int)ceil_div(r, 4);
    }
    LSRN_REQUIRE(pool_used <= pool_elems, "batched iterations: buffer pool overrun");
    DevBuf ditems((size_t)n * sizeof(BatchItem)), doffs((size_t)(4 * (n + 1) + n) * sizeof(int));
    int *o_sw = doffs.as<int>(), *o_red = o_sw + (n + 1), *o_gP = o_red + (n + 1),
        *o_gPt = o_gP + (n + 1), *o_max = o_gPt + (n + 1);
    std::vector<int> packed;
    packed.insert(packed.end(), off_sw.begin(), off_sw.end());
    packed.insert(packed.end(), off_red.begin(), off_red.end());
    packed.insert(packed.end(), off_gP.begin(), off_gP.end());
    packed.insert(packed.end(), off_gPt.begin(), off_gPt.end());
    packed.insert(packed.end(), maxit.begin(), maxit.end());
    LSRN_HIP(hipMemcpyAsync(ditems.as<BatchItem>(), items.data(), (size_t)n * sizeof(BatchItem),
                            hipMemcpyHostToDevice, st));
    LSRN_HIP(hipMemcpyAsync(o_sw, packed.data(), packed.size() * sizeof(int), hipMemcpyHostToDevice, st));
    const BatchItem *di = ditems.as<BatchItem>();
    hipEvent_t e0, e1;
    LSRN_HIP(hipEventCreate(&e0));
    LSRN_HIP(hipEventCreate(&e1));
    LSRN_HIP(hipEventRecord(e0, st));
    // start: t = N^T A^T b, ||b||
    batch_set_state_kernel<<<n, 1, 0, st>>>(di, o_max);
    batch_sweep_kernel<OP_ATB><<<off_sw[(size_t)n], NT, 0, st>>>(di, o_sw, n);
    batch_reduce_kernel<<<off_red[(size_t)n], 256, 0, st>>>(di, o_red, n);
    batch_gemv_kernel<<<off_gPt[(size_t)n], 256, 0, st>>>(di, o_gPt, n, 1);
    LSRN_HIP(hipGetLastError());
    std::vector<State> hs((size_t)n);
    auto all_done = [&] {
        LSRN_HIP(hipMemcpyAsync(hs.data(), states.as<State>(), (size_t)n * sizeof(State),
                                hipMemcpyDeviceToHost, st));
        LSRN_HIP(hipStreamSynchronize(st));
        for (const State &h : hs)
            if (!h.done) return false;
        return true;
    };
    hipGraphExec_t exec = nullptr, exec_cg = nullptr, exec_cs = nullptr;
    // Chebyshev steps (Alg. 3) for every Chebyshev problem, the LSQR ones
    // parked; each problem's step index is its state's count
    auto chunk_cs = [&] {
        for (int k = 0; k < B_CHUNK; ++k) {
            batch_cs_short_kernel<<<n, SNT, 0, st>>>(di);
            batch_gemv_kernel<<<off_gP[(size_t)n], 256, 0, st>>>(di, o_gP, n, 0);
            batch_sweep_kernel<OP_CS_TALL><<<off_sw[(size_t)n], NT, 0, st>>>(di, o_sw, n);
            batch_reduce_kernel<<<off_red[(size_t)n], 256, 0, st>>>(di, o_red, n);
            batch_gemv_kernel<<<off_gPt[(size_t)n], 256, 0, st>>>(di, o_gPt, n, 1);
            batch_cs_step_kernel<<<n, 1, 0, st>>>(di);
        }
        LSRN_HIP(hipGetLastError());
    };
    auto chunk = [&] {
        for (int k = 0; k < B_CHUNK; ++k) {
            batch_gemv_kernel<<<off_gP[(size_t)n], 256, 0, st>>>(di, o_gP, n, 0);
            batch_sweep_kernel<OP_LSQR_TALL><<<off_sw[(size_t)n], NT, 0, st>>>(di, o_sw, n);
            batch_reduce_kernel<<<off_red[(size_t)n], 256, 0, st>>>(di, o_red, n);
            batch_gemv_kernel<<<off_gPt[(size_t)n], 256, 0, st>>>(di, o_gPt, n, 1);
            batch_step_kernel<<<n, SNT, 0, st>>>(di);
        }
        LSRN_HIP(hipGetLastError());
    };
    // CG on (A N)^T (A N) z = c for every problem (the refinement's inner solve)
    auto chunk_cg = [&] {
        for (int k = 0; k < B_CHUNK; ++k) {
            batch_gemv_kernel<<<off_gP[(size_t)n], 256, 0, st>>>(di, o_gP, n, 4);
            batch_sweep_kernel<OP_NORMAL><<<off_sw[(size_t)n], NT, 0, st>>>(di, o_sw, n);
            batch_reduce_kernel<<<off_red[(size_t)n], 256, 0, st>>>(di, o_red, n);
            batch_gemv_kernel<<<off_gPt[(size_t)n], 256, 0, st>>>(di, o_gPt, n, 1);
            batch_cg_step_kernel<<<n, SNT, 0, st>>>(di);
        }
        LSRN_HIP(hipGetLastError());
    };
    // chunks until every problem's done flag is set, each chunk replayed
    // from a captured graph where graphs are allowed
    auto run_until_done = [&](hipGraphExec_t &ex, auto &&body) {
        while (!all_done()) {
            if (st && graphs_allowed()) {
                if (!ex) {
                    hipGraph_t g = nullptr;
                    LSRN_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                    try {
                        body();
                    } catch (...) {
                        (void)hipStreamEndCapture(st, &g);
                        if (g) (void)hipGraphDestroy(g);
                        throw;
                    }
                    LSRN_HIP(hipStreamEndCapture(st, &g));
                    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                    LSRN_HIP(e);
                }
                LSRN_HIP(hipGraphLaunch(ex, st));
            } else {
                body();
            }
        }
    };
    std::vector<int64_t> iters_main((size_t)n), refine_iters((size_t)n, 0), cs_iters((size_t)n, 0);
    std::vector<bool> conv_main((size_t)n);
    // LSQR phase per problem: 0 parked (Chebyshev run passed its check), 1
    // LSQR, 2 LSQR restart on the Chebyshev residual, 3 restart on b
    std::vector<int> mode((size_t)n, 1);
    DevBuf dmode((size_t)n * sizeof(int));
    bool restarts = false;
    try {
        if (any_cs) {
            batch_cs_begin_kernel<<<n, SNT, 0, st>>>(di);
            LSRN_HIP(hipGetLastError());
            run_until_done(exec_cs, chunk_cs);
            batch_cs_norm_kernel<<<n, SNT, 0, st>>>(di);
            LSRN_HIP(hipGetLastError());
            // the check of each run (as in the one-problem solve): |N^T A^T r|
            // against |N^T A^T b|; a failed run restarts LSQR from its
            // iterate, or from zero if its residual grew beyond |b|
            std::vector<double> csn((size_t)3 * n, 0.0);
            for (int p = 0; p < n; ++p)
                if (items[(size_t)p].cs)
                    LSRN_HIP(hipMemcpyAsync(csn.data() + 3 * p, items[(size_t)p].csn, 3 * sizeof(double),
                                            hipMemcpyDeviceToHost, st));
            LSRN_HIP(hipStreamSynchronize(st));
            bool lsqr_left = false;
            for (int p = 0; p < n; ++p) {
                if (!items[(size_t)p].cs) {
                    lsqr_left = true;
                    continue;
                }
                cs_iters[(size_t)p] = hs[(size_t)p].iters;
                const double g0 = csn[(size_t)3 * p], gn = csn[(size_t)3 * p + 1], bn = csn[(size_t)3 * p + 2];
                if (cs_passes(gn, g0, opts[(size_t)p].tol)) {
                    mode[(size_t)p] = 0;
                    continue;
                }
                const double rn = std::sqrt(std::max(0.0, hs[(size_t)p].acc[0]));
                mode[(size_t)p] = (std::isfinite(rn) && rn <= bn) ? 2 : 3;
                res[(size_t)p].cs_fallbacks = 1;
                restarts = lsqr_left = true;
            }
            LSRN_HIP(hipMemcpyAsync(dmode.as<int>(), mode.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice,
                                    st));
            batch_lsqr_phase_kernel<<<n, SNT, 0, st>>>(di, o_max, dmode.as<int>());
            if (lsqr_left) {
                // t = N^T A^T (the right-hand side) again for the problems
                // that run LSQR (the same bits for an LSQR problem: its b is
                // untouched), then their LSQR start
                batch_sweep_kernel<OP_ATB><<<off_sw[(size_t)n], NT, 0, st>>>(di, o_sw, n);
                batch_reduce_kernel<<<off_red[(size_t)n], 256, 0, st>>>(di, o_red, n);
                batch_gemv_kernel<<<off_gPt[(size_t)n], 256, 0, st>>>(di, o_gPt, n, 1);
                batch_init_kernel<<<n, SNT, 0, st>>>(di);
            }
            LSRN_HIP(hipGetLastError());
        } else {
            batch_init_kernel<<<n, SNT, 0, st>>>(di);
            LSRN_HIP(hipGetLastError());
        }
        run_until_done(exec, chunk);
        for (int p = 0; p < n; ++p) {
            const bool passed = mode[(size_t)p] == 0;
            iters_main[(size_t)p] = cs_iters[(size_t)p] + (passed ? 0 : hs[(size_t)p].iters);
            conv_main[(size_t)p] = passed || hs[(size_t)p].converged != 0;
        }
        if (restarts) {
            batch_cs_finish_kernel<<<n, SNT, 0, st>>>(di, dmode.as<int>());
            LSRN_HIP(hipGetLastError());
        }
        batch_gemv_kernel<<<off_gP[(size_t)n], 256, 0, st>>>(di, o_gP, n, 2);
        LSRN_HIP(hipGetLastError());
        // refinement steps (as for one problem): h = A^T (b - A x) in
        // double-double, CG on (A N)^T (A N) z = N^T h to refine_tol, x += N z
        for (int step = 0; step < nref; ++step) {
            batch_resid_kernel<<<off_sw[(size_t)n], NT, 0, st>>>(di, o_sw, n, step);
            batch_reduce_dd_kernel<<<off_red[(size_t)n], 256, 0, st>>>(di, o_red, n, step);
            batch_gemv_kernel<<<off_gPt[(size_t)n], 256, 0, st>>>(di, o_gPt, n, 3, step);
            batch_cg_init_kernel<<<n, SNT, 0, st>>>(di, 200, step);
            LSRN_HIP(hipGetLastError());
            run_until_done(exec_cg, chunk_cg);
            for (int p = 0; p < n; ++p) refine_iters[(size_t)p] += hs[(size_t)p].iters;
            batch_gemv_kernel<<<off_gP[(size_t)n], 256, 0, st>>>(di, o_gP, n, 5, step);
            LSRN_HIP(hipGetLastError());
        }
    } catch (...) {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (exec_cg) (void)hipGraphExecDestroy(exec_cg);
        if (exec_cs) (void)hipGraphExecDestroy(exec_cs);
        (void)hipStreamSynchronize(st);
        throw;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (exec_cg) (void)hipGraphExecDestroy(exec_cg);
    if (exec_cs) (void)hipGraphExecDestroy(exec_cs);
    LSRN_HIP(hipEventRecord(e1, st));
    LSRN_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    LSRN_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int p = 0; p < n; ++p) {
        res[(size_t)p].iters = iters_main[(size_t)p];
        res[(size_t)p].converged = conv_main[(size_t)p];
        res[(size_t)p].refine_steps = opts[(size_t)p].refine;
        res[(size_t)p].refine_iters = refine_iters[(size_t)p];
        res[(size_t)p].t_iter_ms = ms;
    }
    LSRN_HIP(hipStreamSynchronize(st));  // before the buffers are freed
    return res;
}

}  // namespace lsrn
