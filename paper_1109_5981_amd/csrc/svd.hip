// svd.hip -- economy SVD of the sketch and the preconditioner (Alg. 1/2
// steps 4-5).
//
// X (s x d, column-major) = Q R by Householder reflections; then one-sided
// (Hestenes) Jacobi orthogonalises the columns of Y = R^T: Y J = W.  Since
// R^T = W J^T, the columns of W are V_i sigma_i with V the right singular
// vectors of X, so N = V_r Sigma_r^{-1} = W_r Sigma_r^{-2} needs no
// accumulated rotations.  r counts sigma_i > rcond sigma_1.
#include <algorithm>
#include <mutex>
#include <cfloat>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace lsrn {

namespace {

constexpr int QNB = 32;  // Householder panel width

// ------------------------------------------------------------------ QR

// Factor columns p0 .. p0+nb-1 of X (rows >= column index) in place with
// one workgroup.  Reflector j is H_j = I - beta_j v_j v_j^T with v_j stored
// in V[:, j] (zero above row p0 + j); R's entries overwrite X.
__global__ void __launch_bounds__(1024)
qr_panel_kernel(double *__restrict__ X, int64_t s, int64_t p0, int nb, double *__restrict__ V,
                double *__restrict__ beta) {
    __shared__ double red[16][QNB + 1];
    __shared__ double wvec[QNB];
    __shared__ double scratch[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int j = 0; j < nb; ++j) {
        const int64_t c = p0 + j;
        double *xc = X + c * s;
        double acc = 0.0;
        for (int64_t i = c + tid; i < s; i += 1024) acc += xc[i] * xc[i];
        const double nrm2 = block_sum<1024>(acc, scratch);
        const double x0 = xc[c];
        const double normx = sqrt(nrm2);
        // sign of alpha opposite to x0 so that v0 = x0 - alpha does not cancel
        const double alpha = x0 >= 0.0 ? -normx : normx;
        const double v0 = x0 - alpha;
        const double vtv = nrm2 - x0 * x0 + v0 * v0;
        const double bet = normx == 0.0 ? 0.0 : 2.0 / vtv;
        double *vj = V + (int64_t)j * s;
        for (int64_t i = tid; i < s; i += 1024) vj[i] = i < c ? 0.0 : (i == c ? v0 : xc[i]);
        if (tid == 0) beta[j] = bet;

        const int ncols = nb - j - 1;
        double part[QNB];
#pragma unroll
        for (int k = 0; k < QNB; ++k) part[k] = 0.0;
        for (int64_t i = c + tid; i < s; i += 1024) {
            const double vi = i == c ? v0 : xc[i];
#pragma unroll
            for (int k = 0; k < QNB - 1; ++k)
                if (k < ncols) part[k] += vi * X[(c + 1 + k) * s + i];
        }
#pragma unroll
        for (int k = 0; k < QNB - 1; ++k)
            if (k < ncols) {
                const double t = wave_sum(part[k]);
                if (lane == 0) red[wid][k] = t;
            }
        __syncthreads();
        if (tid < ncols) {
            double t = 0.0;
            for (int w = 0; w < 16; ++w) t += red[w][tid];
            wvec[tid] = bet * t;
        }
        __syncthreads();
        for (int64_t i = c + tid; i < s; i += 1024) {
            const double vi = i == c ? v0 : xc[i];
#pragma unroll
            for (int k = 0; k < QNB - 1; ++k)
                if (k < ncols) X[(c + 1 + k) * s + i] -= wvec[k] * vi;
        }
        __syncthreads();
        for (int64_t i = c + tid; i < s; i += 1024) xc[i] = i == c ? alpha : 0.0;
        __syncthreads();
    }
}

// The same panel factorisation with the panel (rows >= p0, NB columns) held
// in registers: thread t owns rows p0 + t + 1024 e, e < EPT, so each column
// step costs three block reductions and no global traffic.
template <int NB, int EPT>
__device__ __forceinline__ void qr_panel_reg(double *__restrict__ X, int64_t s, int64_t p0, int nb,
                                             double *__restrict__ V, double *__restrict__ beta) {
    __shared__ double red[16][NB];
    __shared__ double bc[NB + 1];
    __shared__ double scratch[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double pr[NB][EPT];
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t i = p0 + tid + 1024 * e;
            pr[k][e] = (k < nb && i < s) ? X[(p0 + k) * s + i] : 0.0;
        }
    for (int k = 0; k < nb; ++k)
        for (int64_t i = tid; i < p0; i += 1024) V[(int64_t)k * s + i] = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j < nb) {
            const int64_t c = p0 + j;
            double acc = 0.0;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int64_t i = p0 + tid + 1024 * e;
                if (i >= c && i < s) acc += pr[j][e] * pr[j][e];
            }
            const double nrm2 = block_sum<1024>(acc, scratch);
            if (tid == j) bc[NB] = pr[j][0];  // row c = p0 + j sits in thread j, e = 0
            __syncthreads();
            const double x0 = bc[NB];
            const double normx = sqrt(nrm2);
            const double alpha = x0 >= 0.0 ? -normx : normx;
            const double v0 = x0 - alpha;
            const double vtv = nrm2 - x0 * x0 + v0 * v0;
            const double bet = normx == 0.0 ? 0.0 : 2.0 / vtv;
            double vr[EPT];
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int64_t i = p0 + tid + 1024 * e;
                vr[e] = (i < c || i >= s) ? 0.0 : (i == c ? v0 : pr[j][e]);
            }
#pragma unroll
            for (int k = j + 1; k < NB; ++k) {
                if (k < nb) {
                    double t = 0.0;
#pragma unroll
                    for (int e = 0; e < EPT; ++e) t += vr[e] * pr[k][e];
                    t = wave_sum(t);
                    if (lane == 0) red[wid][k] = t;
                }
            }
            __syncthreads();
            if (tid > j && tid < nb) {
                double t = 0.0;
                for (int w = 0; w < 16; ++w) t += red[w][tid];
                bc[tid] = bet * t;
            }
            __syncthreads();
#pragma unroll
            for (int k = j + 1; k < NB; ++k) {
                if (k < nb) {
                    const double f = bc[k];
#pragma unroll
                    for (int e = 0; e < EPT; ++e) pr[k][e] -= f * vr[e];
                }
            }
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int64_t i = p0 + tid + 1024 * e;
                if (i < s) {
                    V[(int64_t)j * s + i] = vr[e];
                    if (i >= c) pr[j][e] = i == c ? alpha : 0.0;
                }
            }
            if (tid == 0) beta[j] = bet;
            __syncthreads();
        }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t i = p0 + tid + 1024 * e;
            if (k < nb && i < s) X[(p0 + k) * s + i] = pr[k][e];
        }
}

template <int NB, int EPT>
__global__ void __launch_bounds__(1024)
qr_panel_reg_kernel(double *__restrict__ X, int64_t s, int64_t p0, int nb, double *__restrict__ V,
                    double *__restrict__ beta) {
    qr_panel_reg<NB, EPT>(X, s, p0, nb, V, beta);
}

// One problem of a batched QR: the sketch and its panel buffers.
struct QrItem {
    double *X;
    int64_t s, d;
    double *V, *beta;  // s x QNB and QNB entries
};

// The panel at column p0 of every problem with d > p0, workgroup p for
// problem p.
template <int NB, int EPT>
__global__ void __launch_bounds__(1024)
qr_panel_reg_batch_kernel(const QrItem *__restrict__ items, int64_t p0, int pw) {
    const QrItem it = items[blockIdx.x];
    if (it.d <= p0) return;
    const int nb = (int)min((int64_t)pw, it.d - p0);
    qr_panel_reg<NB, EPT>(it.X, it.s, p0, nb, it.V, it.beta);
}

// Apply the nb reflectors of a panel, in order, to the trailing columns
// c >= p0 + nb: one column per workgroup, held in registers.
template <int NT, int EPT>
__device__ __forceinline__ void qr_apply(double *__restrict__ X, int64_t s, int64_t p0, int nb,
                                         const double *__restrict__ V,
                                         const double *__restrict__ beta, int64_t col) {
    __shared__ double scratch[NT / 64];
    const int64_t c = p0 + nb + col;
    double *xc = X + c * s;
    double reg[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t i = p0 + threadIdx.x + (int64_t)NT * e;
        reg[e] = i < s ? xc[i] : 0.0;
    }
    for (int j = 0; j < nb; ++j) {
        const double *vj = V + (int64_t)j * s;
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t i = p0 + threadIdx.x + (int64_t)NT * e;
            if (i < s) acc += vj[i] * reg[e];
        }
        const double f = beta[j] * block_sum<NT>(acc, scratch);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t i = p0 + threadIdx.x + (int64_t)NT * e;
            if (i < s) reg[e] -= f * vj[i];
        }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t i = p0 + threadIdx.x + (int64_t)NT * e;
        if (i < s) xc[i] = reg[e];
    }
}

template <int NT, int EPT>
__global__ void __launch_bounds__(NT)
qr_apply_kernel(double *__restrict__ X, int64_t s, int64_t p0, int nb, const double *__restrict__ V,
                const double *__restrict__ beta) {
    qr_apply<NT, EPT>(X, s, p0, nb, V, beta, blockIdx.x);
}

// The trailing update of the panel at p0 for every problem: workgroup
// (p, y) updates trailing column y of problem p, if it has one.
template <int NT, int EPT>
__global__ void __launch_bounds__(NT)
qr_apply_batch_kernel(const QrItem *__restrict__ items, int64_t p0, int pw) {
    const QrItem it = items[blockIdx.x];
    if (it.d <= p0) return;
    const int nb = (int)min((int64_t)pw, it.d - p0);
    if ((int64_t)blockIdx.y >= it.d - p0 - nb) return;
    qr_apply<NT, EPT>(it.X, it.s, p0, nb, it.V, it.beta, blockIdx.y);
}

// Y (d x dcols, column-major, ld d): column p = row p of R (R upper
// triangle of X); columns p >= d are zero padding.
__global__ void __launch_bounds__(256)
r_to_y_kernel(const double *__restrict__ X, int64_t s, int64_t d, int64_t dcols,
              double *__restrict__ Y) {
    const int64_t total = d * dcols;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = t / d, i = t % d;
        Y[t] = (p < d && i >= p) ? X[i * s + p] : 0.0;
    }
}

// -------------------------------------------------------------- Jacobi

// Pair k of round t of the circle-method round robin on n (even) players.
__device__ __forceinline__ void rr_pair(int n, int t, int k, int &a, int &b) {
    if (k == 0) {
        a = n - 1;
        b = t;
    } else {
        a = (t + k) % (n - 1);
        b = (t - k + (n - 1)) % (n - 1);
    }
}

// Compile-time round-robin pair (same schedule as rr_pair).
template <int N, int T, int K>
struct RR {
    static constexpr int a = K == 0 ? N - 1 : (T + K) % (N - 1);
    static constexpr int b = K == 0 ? T : (T - K + (N - 1)) % (N - 1);
    static constexpr int p = a < b ? a : b;
    static constexpr int q = a < b ? b : a;
};

// Sum each of the 32 values v[0..31] over the 64 lanes of a wavefront by a
// halving butterfly (reduce-scatter): at each step a lane keeps half of its
// values and adds its partner's copy of that half.  Afterwards lanes 2j and
// 2j+1 both hold the total of value j (32 shuffles instead of 192).
template <int N, int H>
__device__ __forceinline__ void butterfly_steps(double (&v)[N], int lane) {
    if constexpr (H >= 1) {
        const bool upper = (lane & (2 * H)) != 0;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const double send = upper ? v[j] : v[j + H];
            const double keep = upper ? v[j + H] : v[j];
            v[j] = keep + __shfl_xor(send, 2 * H, 64);
        }
        butterfly_steps<N, H / 2>(v, lane);
    }
}

// N (a power of two <= 32) values reduced over the wavefront: the halving
// steps consume lane bits 1 .. log2 N, plain butterflies the rest; lane l
// then holds the total of value (l >> 1) & (N - 1).
template <int N>
__device__ __forceinline__ double wave_reduce_n(double (&v)[N]) {
    const int lane = threadIdx.x & 63;
    butterfly_steps<N, N / 2>(v, lane);
    double t = v[0] + __shfl_xor(v[0], 1, 64);
#pragma unroll
    for (int m = 2 * N; m <= 32; m <<= 1) t += __shfl_xor(t, m, 64);
    return t;
}

template <int X>
constexpr int pow2_at_least() {
    int p = 1;
    while (p < X) p <<= 1;
    return p;
}

// Packed index of Gram entry (p, q), p <= q, row by row.
template <int NL>
__host__ __device__ constexpr int gram_index(int p, int q) {
    return p * NL - p * (p - 1) / 2 + (q - p);
}

// 1 / sqrt(x) and 1 / x for normal x > 0 from the hardware estimates; each
// Newton step roughly squares the relative error.
template <int STEPS = 1>
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int k = 0; k < STEPS; ++k) y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return y * fma(-x, y, 2.0);
}

// Rotation of the pair (p, q) from its Gram entries a = |x_p|^2,
// b = |x_q|^2, g = x_p . x_q (Golub & Van Loan Sec. 8.6): x_p <- c x_p - s x_q,
// x_q <- s x_p + c x_q makes the pair orthogonal.  False (c = 1, s = 0) when
// |g| <= tol sqrt(a b).  Only c^2 + s^2 = 1 has to hold to rounding (c from
// t by a refined reciprocal square root); the threshold test and the angle
// itself may carry a few ulp.
__device__ __forceinline__ bool jacobi_angle(double a, double b, double g, double tol,
                                             double tiny2, double &c, double &s) {
    c = 1.0;
    s = 0.0;
    if (!(fmax(a, b) > tiny2 && g != 0.0 && fabs(g) * rsqrt_nr(a) * rsqrt_nr(b) > tol)) return false;
    const double zeta = (b - a) * rcp_nr(2.0 * g);
    const double az = fabs(zeta);
    // 1 / (|zeta| + sqrt(1 + zeta^2)), without overflow for huge |zeta|
    const double den = az < 1e150 ? az + (1.0 + az * az) * rsqrt_nr(1.0 + az * az) : 2.0 * az;
    const double t = copysign(rcp_nr(den), zeta);
    c = rsqrt_nr<2>(fma(t, t, 1.0));
    s = c * t;
    return true;
}

// Whole matrix in LDS (d <= 128), all sweeps in one workgroup of 1024
// threads.  In each round of the circle-method round robin every pair is
// rotated at once by its own group of 16 lanes (lane j holds rows j, j + 16,
// ... in registers); the group's three inner products reduce by xor
// butterflies inside the group, so a round costs one barrier.
__device__ __forceinline__ void jacobi_small(double *__restrict__ Y, int d, int max_sweeps,
                                             double tol, double tiny2, int *__restrict__ sweeps_out) {
    extern __shared__ double W[];  // d * d, column p at W + p*d
    __shared__ int rot;
    constexpr int GS = 16, RPL = 128 / GS;  // lanes per pair, rows per lane
    const int tid = threadIdx.x, grp = tid / GS, j = tid % GS;
    for (int t = tid; t < d * d; t += blockDim.x) W[t] = Y[t];
    const int n = d + (d & 1);
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if (tid == 0) rot = 0;
        __syncthreads();
        int mine = 0;
        for (int round = 0; round < n - 1; ++round) {
            int p = 0, q = 0;
            if (grp < n / 2) {
                rr_pair(n, round, grp, p, q);
                if (p > q) { const int t = p; p = q; q = t; }
            }
            const bool live = grp < n / 2 && q < d;
            double xr[RPL], yr[RPL], a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int i = j + GS * k;
                const bool in = live && i < d;
                xr[k] = in ? W[p * d + i] : 0.0;
                yr[k] = in ? W[q * d + i] : 0.0;
                a += xr[k] * xr[k];
                b += yr[k] * yr[k];
                g += xr[k] * yr[k];
            }
#pragma unroll
            for (int o = 1; o < GS; o <<= 1) {
                a += __shfl_xor(a, o, 64);
                b += __shfl_xor(b, o, 64);
                g += __shfl_xor(g, o, 64);
            }
            double c, sn;
            if (live && jacobi_angle(a, b, g, tol, tiny2, c, sn)) {
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    const int i = j + GS * k;
                    if (i < d) {
                        W[p * d + i] = c * xr[k] - sn * yr[k];
                        W[q * d + i] = sn * xr[k] + c * yr[k];
                    }
                }
                if (j == 0) ++mine;
            }
            __syncthreads();
        }
        if (mine) atomicAdd(&rot, mine);
        __syncthreads();
        const int total = rot;
        __syncthreads();
        if (total == 0) break;
    }
    for (int t = tid; t < d * d; t += blockDim.x) Y[t] = W[t];
    if (tid == 0) *sweeps_out = sweep + 1;
}

__global__ void __launch_bounds__(1024)
jacobi_small_kernel(double *__restrict__ Y, int d, int max_sweeps, double tol, double tiny2,
                    int *__restrict__ sweeps_out) {
    jacobi_small(Y, d, max_sweeps, tol, tiny2, sweeps_out);
}

// Raw buffer resource over the n doubles of one column at p: the hardware
// range check returns 0 for loads past the end and drops stores past the
// end, so the padding rows of a thread's share need no branches.  Word 3
// is the gfx9 buffer format word (32-bit data format).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t column_rsrc(double *p, int n) {
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, n * (int)sizeof(double), 0x00020000);
}
__device__ __forceinline__ double column_load(__amdgpu_buffer_rsrc_t rs, int i) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, i * 8, 0, 0));
}
__device__ __forceinline__ void column_store(__amdgpu_buffer_rsrc_t rs, int i, double v) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, i * 8, 0, 0);
}

// ------------------------------------------- QR, compact WY trailing updates

// Buffer resource over the rows p0 .. s-1 of column `col` of X (s rows,
// column-major); empty when `live` is false, so loads return 0 and stores
// are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t panel_rsrc(double *X, int64_t s, int64_t p0,
                                                             int64_t col, bool live) {
    return __builtin_amdgcn_make_buffer_rsrc(X + col * s + p0, (short)0,
                                             live ? (int)((s - p0) * (int64_t)sizeof(double)) : 0,
                                             0x00020000);
}

// Householder factorisation of the panel of nb <= NB columns at p0 (rows
// >= p0 in registers: thread t owns rows p0 + t + 1024 e, e < EPT) with a
// single block reduction per column.  For column j (diagonal row c) the
// reduction carries |x_j|^2 and x_j . x_k for the later columns k, all over
// rows >= c; with v = x_j - alpha e_c (alpha = -sign(x_jc) |x_j|) the
// products the update needs follow as v . x_k = x_j . x_k - alpha x_kc, and
// x_kc comes from the thread that owns row c.  The reflector
// H_j = I - beta_j v_j v_j^T is stored in V[:, j] (rows >= p0, zero above
// row c).  At the end the upper-triangular T of the compact WY form
// H_1 ... H_nb = I - V T V^T (Schreiber & Van Loan 1989) is formed from
// V^T V and the betas and written row-major to T (NB x NB).
template <int NB, int EPT>
__global__ void __launch_bounds__(1024)
qr_panel_wy_kernel(double *__restrict__ X, int64_t s, int64_t p0, int nb, double *__restrict__ V,
                   double *__restrict__ T) {
    constexpr int NW = 16;
    constexpr int NG = NB * (NB - 1) / 2;  // strictly upper entries of V^T V
    constexpr int NGP = NG <= 1 ? 2 : pow2_at_least<NG>();
    static_assert(NB <= 32 && NGP <= 32, "one butterfly chunk");
    __shared__ double red[NW][NGP > NB ? NGP : NB];
    __shared__ double tot[NGP > NB ? NGP : NB];
    __shared__ double rowc[2][NB];
    __shared__ double betas[NB];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double pr[NB][EPT];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const __amdgpu_buffer_rsrc_t rs = panel_rsrc(X, s, p0, p0 + k, k < nb);
#pragma unroll
        for (int e = 0; e < EPT; ++e) pr[k][e] = column_load(rs, tid + 1024 * e);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j >= nb) break;
        const int64_t c = p0 + j;
        const int buf = j & 1;
        double part[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) part[k] = 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const bool act = p0 + tid + 1024 * e >= c;
            const double xj = act ? pr[j][e] : 0.0;
            part[j] += xj * xj;
#pragma unroll
            for (int k = j + 1; k < NB; ++k) part[k] += xj * pr[k][e];
        }
        if (tid == j) {  // row c: thread j, e = 0
#pragma unroll
            for (int k = j; k < NB; ++k) rowc[buf][k] = pr[k][0];
        }
        const double wt = wave_reduce_n<NB>(part);
        if ((lane & 1) == 0 && (lane >> 1) < NB) red[wid][lane >> 1] = wt;
        __syncthreads();
        if (tid < NB) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) t += red[w][tid];
            tot[tid] = t;
        }
        __syncthreads();
        const double nrm2 = tot[j], x0 = rowc[buf][j];
        const double normx = sqrt(nrm2);
        const double alpha = x0 >= 0.0 ? -normx : normx;
        const double v0 = x0 - alpha;
        const double vtv = nrm2 - x0 * x0 + v0 * v0;
        const double bet = normx == 0.0 ? 0.0 : 2.0 / vtv;
        double v[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t i = p0 + tid + 1024 * e;
            v[e] = i > c ? pr[j][e] : (i == c ? v0 : 0.0);
        }
#pragma unroll
        for (int k = j + 1; k < NB; ++k) {
            if (k < nb) {
                const double f = bet * (tot[k] - alpha * rowc[buf][k]);
#pragma unroll
                for (int e = 0; e < EPT; ++e) pr[k][e] -= f * v[e];
            }
        }
        const __amdgpu_buffer_rsrc_t rv = panel_rsrc(V, s, p0, j, true);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t i = p0 + tid + 1024 * e;
            column_store(rv, tid + 1024 * e, v[e]);
            pr[j][e] = i == c ? alpha : (i > c ? 0.0 : pr[j][e]);
        }
        if (tid == 0) betas[j] = bet;
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const __amdgpu_buffer_rsrc_t rs = panel_rsrc(X, s, p0, p0 + k, k < nb);
#pragma unroll
        for (int e = 0; e < EPT; ++e) column_store(rs, tid + 1024 * e, pr[k][e]);
    }
    // T from G = V^T V: T_jj = beta_j, T(0:j, j) = -beta_j T(0:j, 0:j) G(0:j, j).
    // Each thread reads back the reflector rows it wrote itself.
    double vv[NB][EPT];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const __amdgpu_buffer_rsrc_t rv = panel_rsrc(V, s, p0, k, k < nb);
#pragma unroll
        for (int e = 0; e < EPT; ++e) vv[k][e] = column_load(rv, tid + 1024 * e);
    }
    double g[NGP];
#pragma unroll
    for (int q = 0; q < NGP; ++q) g[q] = 0.0;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = a + 1; b < NB; ++b) {
            const int q = b * (b - 1) / 2 + a;
#pragma unroll
            for (int e = 0; e < EPT; ++e) g[q] += vv[a][e] * vv[b][e];
        }
    const double gt = wave_reduce_n<NGP>(g);
    if ((lane & 1) == 0 && (lane >> 1) < NGP) red[wid][lane >> 1] = gt;
    __syncthreads();
    if (tid < NGP) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += red[w][tid];
        tot[tid] = t;
    }
    __syncthreads();
    if (tid == 0) {
        double Tl[NB][NB];
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) Tl[a][b] = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b >= nb) break;
            const double bb = betas[b];
            Tl[b][b] = bb;
#pragma unroll
            for (int a = 0; a < b; ++a) {
                double t = 0.0;
#pragma unroll
                for (int l = a; l < b; ++l) t += Tl[a][l] * tot[b * (b - 1) / 2 + l];
                Tl[a][b] = -bb * t;
            }
        }
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) T[a * NB + b] = Tl[a][b];
    }
}

// Trailing update by the panel's reflectors in compact WY form,
// x <- (I - V T^T V^T) x = H_nb ... H_1 x, for CPW trailing columns per
// workgroup (rows >= p0 in registers, thread t owns rows p0 + t + 1024 e):
// w = V^T x in one block reduction for all columns, u = T^T w, x -= V u.
template <int NB, int EPT, int CPW>
__global__ void __launch_bounds__(1024)
qr_apply_wy_kernel(double *__restrict__ X, int64_t s, int64_t p0, int nb, int64_t ncols,
                   double *__restrict__ V, const double *__restrict__ T) {
    constexpr int NW = 16, NV = CPW * NB;
    static_assert(NV <= 32 && (NV & (NV - 1)) == 0, "one butterfly chunk");
    __shared__ double red[NW][NV];
    __shared__ double wt[NV], ut[NV];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t c0 = p0 + nb + (int64_t)blockIdx.x * CPW;
    double x[CPW][EPT];
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
        const __amdgpu_buffer_rsrc_t rs = panel_rsrc(X, s, p0, c0 + q, c0 + q < p0 + nb + ncols);
#pragma unroll
        for (int e = 0; e < EPT; ++e) x[q][e] = column_load(rs, tid + 1024 * e);
    }
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const __amdgpu_buffer_rsrc_t rv = panel_rsrc(V, s, p0, j, j < nb);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const double vj = column_load(rv, tid + 1024 * e);
#pragma unroll
            for (int q = 0; q < CPW; ++q) acc[q * NB + j] += vj * x[q][e];
        }
    }
    const double wsum = wave_reduce_n<NV>(acc);
    if ((lane & 1) == 0 && (lane >> 1) < NV) red[wid][lane >> 1] = wsum;
    __syncthreads();
    if (tid < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += red[w][tid];
        wt[tid] = t;
    }
    __syncthreads();
    if (tid < NV) {
        const int q = tid / NB, j = tid % NB;
        double u = 0.0;
        if (j < nb)
            for (int i = 0; i <= j; ++i) u += T[i * NB + j] * wt[q * NB + i];
        ut[tid] = u;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const __amdgpu_buffer_rsrc_t rv = panel_rsrc(V, s, p0, j, j < nb);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const double vj = column_load(rv, tid + 1024 * e);
#pragma unroll
            for (int q = 0; q < CPW; ++q) x[q][e] -= vj * ut[q * NB + j];
        }
    }
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
        const __amdgpu_buffer_rsrc_t rs = panel_rsrc(X, s, p0, c0 + q, c0 + q < p0 + nb + ncols);
#pragma unroll
        for (int e = 0; e < EPT; ++e) column_store(rs, tid + 1024 * e, x[q][e]);
    }
}

// Partner of player i (i < NL, NL even) in sub-round TS of the circle-
// method round robin, and the index of their pair (as in rr_pair), without
// branches: the sub-round loop is unrolled, so these run once per thread
// and sub-round on the update's critical path.
template <int NL, int TS>
__device__ __forceinline__ int rr_partner(int i) {
    constexpr int M = NL - 1;
    int p = 2 * TS - i;
    p += p < 0 ? M : 0;
    p -= p >= M ? M : 0;
    p = i == TS ? M : p;
    return i == M ? TS : p;
}
template <int NL, int TS>
__device__ __forceinline__ int rr_pair_index(int i) {
    constexpr int M = NL - 1;
    int u = i - TS;
    u += u < 0 ? M : 0;
    const int k = u < M - u ? u : M - u;
    return i == M ? 0 : k;
}

// One round of the block round robin, Gram form.  The 2 BW columns of the
// block pair stay in registers (thread t owns rows t + 512 u, u < EPU).
// Their 2 BW x 2 BW Gram matrix G is reduced once; the 2 BW - 1 sub-rounds
// of rotations are then carried out on G itself, every thread owning one
// entry of G and of the accumulated rotation J (G <- R^T G R, J <- J R per
// sub-round, through LDS), and the columns are replaced by x J in a single
// pass.  Each angle follows the one-sided (Hestenes) formula from the
// current Gram entries.  The first sub-round tests exact inner products of
// the columns and a sub-round without rotations leaves G and J bit for bit
// unchanged (c = 1, s = 0), so "no rotation in the round" is the same exact
// convergence test as rotating column by column.
//
// last_mod[b] is the global round index (sweep * (nblocks - 1) + round) at
// which a column of block b was last rotated.  Two blocks meet once per
// sweep; if neither changed since their previous meeting (period rounds
// ago) then no rotation happened there and none can happen now, so the
// workgroup returns at once -- an exact shortcut for the converging sweeps.
// d <= 512 EPU.
template <int BW, int EPU>
__device__ __forceinline__ void
jacobi_gram_round(double *__restrict__ Y, int d, int nblocks, int round, int pair, double tol,
                  double tiny2,
                  int *__restrict__ rot_count, int *__restrict__ last_mod, int rnow) {
    constexpr int NL = 2 * BW;
    constexpr int NG = NL * (NL + 1) / 2;
    constexpr int NFULL = NG / 32;                        // 32-value reduction chunks
    constexpr int NREST = NG - 32 * NFULL;                // values of the last chunk
    constexpr int NVREST = NREST ? pow2_at_least<NREST>() : 1;
    static_assert(NL * NL <= 512, "one thread per Gram entry");
    __shared__ double part[8][32 * NFULL + NVREST];
    __shared__ double Gs[2][NL][NL + 1], Js[2][NL][NL + 1], CSs[BW][2];
    __shared__ int nrot_s, any_s[NL];
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    int bi, bj;
    rr_pair(nblocks, round, pair, bi, bj);
    const int prev = rnow - (nblocks - 1);
    if (prev >= 0 && last_mod[bi] < prev && last_mod[bj] < prev) return;
    // local column order follows the global one: block min(bi, bj) first
    const int blo = bi < bj ? bi : bj, bhi = bi < bj ? bj : bi;
    double x[NL][EPU];
#pragma unroll
    for (int cl = 0; cl < NL; ++cl) {
        const int64_t col = (int64_t)(cl < BW ? blo : bhi) * BW + (cl % BW);
        const __amdgpu_buffer_rsrc_t rs = column_rsrc(Y + col * d, d);
#pragma unroll
        for (int u = 0; u < EPU; ++u) x[cl][u] = column_load(rs, tid + 512 * u);
    }
    if (tid == 0) nrot_s = 0;
    if (tid < NL) any_s[tid] = 0;
    // ---- Gram matrix: per-thread partial sums, reduced in chunks of <= 32
    // values per butterfly, then across the 8 wavefronts
    auto chunk = [&](auto cidx, auto nv) {
        constexpr int C = decltype(cidx)::value, NV = decltype(nv)::value;
        double v[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = 0.0;
#pragma unroll
        for (int p = 0; p < NL; ++p)
#pragma unroll
            for (int q = p; q < NL; ++q) {
                const int k = gram_index<NL>(p, q) - 32 * C;
                if (k >= 0 && k < NV) {
                    double t = 0.0;
#pragma unroll
                    for (int u = 0; u < EPU; ++u) t += x[p][u] * x[q][u];
                    v[k] = t;
                }
            }
        const double tot = wave_reduce_n<NV>(v);
        if ((lane & 1) == 0 && (lane >> 1) < NV) part[wid][32 * C + (lane >> 1)] = tot;
    };
    [&]<int... C>(std::integer_sequence<int, C...>) {
        (chunk(std::integral_constant<int, C>{}, std::integral_constant<int, 32>{}), ...);
    }(std::make_integer_sequence<int, NFULL>{});
    if constexpr (NREST > 0)
        chunk(std::integral_constant<int, NFULL>{}, std::integral_constant<int, NVREST>{});
    __syncthreads();
    // thread t < NL^2 owns entry (r, c) of G and J
    const bool owner = tid < NL * NL;
    const int r = owner ? tid / NL : 0, c = owner ? tid % NL : 0;
    double gv = 0.0, jv = 0.0;
    if (owner) {
        const int k = r <= c ? gram_index<NL>(r, c) : gram_index<NL>(c, r);
#pragma unroll
        for (int w = 0; w < 8; ++w) gv += part[w][k];
        jv = r == c ? 1.0 : 0.0;
        Gs[0][r][c] = gv;
        Js[0][r][c] = jv;
    }
    __syncthreads();
    int mine = 0, cur = 0;
    auto sub_round = [&](auto tsub) {
        constexpr int TS = decltype(tsub)::value;
        // (a) the angle of pair k, once, by thread k
        if (tid < BW) {
            const int k = tid;
            int a = TS + k, b = TS - k;
            a -= a >= NL - 1 ? NL - 1 : 0;
            b += b < 0 ? NL - 1 : 0;
            a = k == 0 ? NL - 1 : a;
            const int pp = a < b ? a : b, qq = a < b ? b : a;
            double cs, sn;
            if (jacobi_angle(Gs[cur][pp][pp], Gs[cur][qq][qq], Gs[cur][pp][qq], tol, tiny2, cs, sn)) {
                ++mine;
                any_s[TS] = 1;
            }
            CSs[k][0] = cs;
            CSs[k][1] = sn;
        }
        __syncthreads();
        if (!any_s[TS]) return;  // uniform: G and J stay as they are
        // (b) G <- R^T G R and J <- J R entry by entry
        if (owner) {
            // partners of r and c in this sub-round and the indices of their pairs
            const int r2 = rr_partner<NL, TS>(r), c2 = rr_partner<NL, TS>(c);
            const int kr = rr_pair_index<NL, TS>(r), kc = rr_pair_index<NL, TS>(c);
            // new column x = alpha x_own + beta x_partner
            const double ar = CSs[kr][0], br = r < r2 ? -CSs[kr][1] : CSs[kr][1];
            const double ac = CSs[kc][0], bc = c < c2 ? -CSs[kc][1] : CSs[kc][1];
            const double g_rc2 = Gs[cur][r][c2], g_r2c = Gs[cur][r2][c], g_r2c2 = Gs[cur][r2][c2];
            const double j_rc2 = Js[cur][r][c2];
            gv = ar * (ac * gv + bc * g_rc2) + br * (ac * g_r2c + bc * g_r2c2);
            jv = ac * jv + bc * j_rc2;
            Gs[cur ^ 1][r][c] = gv;
            Js[cur ^ 1][r][c] = jv;
        }
        cur ^= 1;
        __syncthreads();
    };
    [&]<int... TS>(std::integer_sequence<int, TS...>) {
        (sub_round(std::integral_constant<int, TS>{}), ...);
    }(std::make_integer_sequence<int, NL - 1>{});
    if (mine) atomicAdd(&nrot_s, mine);
    __syncthreads();
    const int nrot = nrot_s;
    if (nrot == 0) return;
    // ---- columns <- x J, written straight back
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        double acc[EPU];
#pragma unroll
        for (int u = 0; u < EPU; ++u) acc[u] = 0.0;
#pragma unroll
        for (int p = 0; p < NL; ++p) {
            const double jpq = Js[cur][p][q];
#pragma unroll
            for (int u = 0; u < EPU; ++u) acc[u] += x[p][u] * jpq;
        }
        const int64_t col = (int64_t)(q < BW ? blo : bhi) * BW + (q % BW);
        const __amdgpu_buffer_rsrc_t rs = column_rsrc(Y + col * d, d);
#pragma unroll
        for (int u = 0; u < EPU; ++u) column_store(rs, tid + 512 * u, acc[u]);
    }
    if (tid == 0) {
        atomicAdd(rot_count, nrot);
        last_mod[bi] = rnow;
        last_mod[bj] = rnow;
    }
}

template <int BW, int EPU>
__global__ void __launch_bounds__(512)
jacobi_gram_round_kernel(double *__restrict__ Y, int d, int nblocks, int round, double tol, double tiny2,
                         int *__restrict__ rot_count, int *__restrict__ last_mod, int rnow) {
    jacobi_gram_round<BW, EPU>(Y, d, nblocks, round, blockIdx.x, tol, tiny2, rot_count, last_mod, rnow);
}

// One problem of a batch for the batched Jacobi rounds.
struct JacobiItem {
    double *Y;
    int d, nblocks;
    double tol;
    double tiny2;   // pairs whose columns both have |y|^2 <= tiny2 are not rotated
    int *rot;       // rotations of the current sweep
    int *last_mod;  // nblocks entries
};

// Round `round` of sweep `sweep` for every active problem of a batch: work
// item g is pair g - pair_off[p] of problem p (pair_off: prefix sums of
// nblocks / 2).  Problems whose own round count is smaller, or that have
// converged (active[p] == 0), leave their work items empty.
template <int BW, int EPU>
__global__ void __launch_bounds__(512)
jacobi_gram_round_batch_kernel(const JacobiItem *__restrict__ items, const int *__restrict__ pair_off,
                               const int *__restrict__ active, int count, int round, int sweep) {
    const int g = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pair_off[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    const JacobiItem it = items[lo];
    const int period = it.nblocks - 1;
    if (!active[lo] || round >= period) return;
    jacobi_gram_round<BW, EPU>(it.Y, it.d, it.nblocks, round, g - pair_off[lo], it.tol, it.tiny2, it.rot,
                               it.last_mod, sweep * period + round);
}

// Whole sweeps of many small problems (d <= 128, the matrix in LDS), one
// workgroup per problem: item p is problem p.
__global__ void __launch_bounds__(1024)
jacobi_small_batch_kernel(const JacobiItem *__restrict__ items, int max_sweeps,
                          int *__restrict__ sweeps_out) {
    const JacobiItem it = items[blockIdx.x];
    jacobi_small(it.Y, it.d, max_sweeps, it.tol, it.tiny2, sweeps_out + blockIdx.x);
}

// sigma_p = ||Y[:, p]||, one wavefront per column.
__global__ void __launch_bounds__(256)
col_norms_kernel(const double *__restrict__ Y, int64_t d, double *__restrict__ nrm) {
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= d) return;
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    for (int64_t i = lane; i < d; i += 64) {
        const double v = Y[p * d + i];
        acc += v * v;
    }
    acc = wave_sum(acc);
    if (lane == 0) nrm[p] = sqrt(acc);
}

// Descending order, ties by index: order[rank(p)] = p.
__global__ void __launch_bounds__(256)
rank_sort_kernel(const double *__restrict__ nrm, int64_t d, int64_t *__restrict__ order,
                 double *__restrict__ sigma) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d) return;
    const double v = nrm[p];
    int64_t rank = 0;
    for (int64_t q = 0; q < d; ++q) {
        const double u = nrm[q];
        rank += (u > v) || (u == v && q < p);
    }
    order[rank] = p;
    sigma[rank] = v;
}

// P[i][c] = Y[:, order[c]][i] / sigma_c^2 for c < r (row-major, ld d).
__global__ void __launch_bounds__(256)
form_p_kernel(const double *__restrict__ Y, int64_t d, int64_t r, const int64_t *__restrict__ order,
              const double *__restrict__ sigma, double *__restrict__ P) {
    const int64_t total = d * r;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / r, c = t % r;
        const double sg = sigma[c];
        P[i * d + c] = Y[order[c] * d + i] / (sg * sg);
    }
}

// out[i] = |R(i, i)| (R the upper triangle of X, column-major, ld s).
__global__ void __launch_bounds__(256)
diag_abs_kernel(const double *__restrict__ X, int64_t s, int64_t d, double *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = fabs(X[i * s + i]);
}

int grid1d(int64_t total) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(total, 256), 16384)); }

template <int NT, int EPT>
void launch_apply(double *X, int64_t s, int64_t p0, int nb, int64_t ncols, const double *V,
                  const double *beta, hipStream_t st) {
    qr_apply_kernel<NT, EPT><<<(unsigned)ncols, NT, 0, st>>>(X, s, p0, nb, V, beta);
}

size_t lds_limit() {
    static const size_t lim = [] {  // queried once (a thread-safe static)
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
            (void)hipGetLastError();
            v = 65536;
        }
        return (size_t)v;
    }();
    return lim;
}

}  // namespace

size_t precond_workspace_bytes(int64_t s, int64_t d) {
    const int64_t dcols = round_up(d, 64) + 64;
    // after the QR: the Jacobi path's Y, or the certified path's R^-1, the
    // triangular inverse's product buffer and the power steps' vectors
    const size_t after = std::max((size_t)d * dcols, (size_t)d * d + (size_t)trtri_work_elems(d) + 4 * (size_t)d + 1);
    return sizeof(double) * ((size_t)s * QNB + QNB + after + 2 * (size_t)d) + sizeof(int64_t) * (size_t)d + 64;
}

void householder_qr(int64_t s, int64_t d, double *X, hipStream_t st) {
    LSRN_REQUIRE(s >= d && d > 0, "qr: need s >= d > 0");
    if (s > 1024 * 40) fail(LSRN_E_UNSUPPORTED, "precond: the QR kernels support sketches of up to 40960 rows");
    DevBuf Vb((size_t)s * QNB * sizeof(double)), betab(QNB * sizeof(double));
    if (s <= 8192) {
        // register panels of 8 columns (4 while more than 4096 rows remain)
        // with one block reduction per column; trailing updates in compact
        // WY form, one block reduction per trailing column and panel
        DevBuf Tb(8 * 8 * sizeof(double));
        double *Vp = Vb.as<double>(), *Tp = Tb.as<double>();
        for (int64_t p0 = 0; p0 < d;) {
            const int64_t rows = s - p0;
            const int pw = rows <= 4096 ? 8 : 4;
            const int nb = (int)std::min<int64_t>(pw, d - p0);
            if (rows <= 1024) qr_panel_wy_kernel<8, 1><<<1, 1024, 0, st>>>(X, s, p0, nb, Vp, Tp);
            else if (rows <= 2048) qr_panel_wy_kernel<8, 2><<<1, 1024, 0, st>>>(X, s, p0, nb, Vp, Tp);
            else if (rows <= 4096) qr_panel_wy_kernel<8, 4><<<1, 1024, 0, st>>>(X, s, p0, nb, Vp, Tp);
            else qr_panel_wy_kernel<4, 8><<<1, 1024, 0, st>>>(X, s, p0, nb, Vp, Tp);
            LSRN_HIP(hipGetLastError());
            const int64_t ncols = d - p0 - nb;
            if (ncols > 0) {
                const dim3 g4((unsigned)ceil_div(ncols, 4)), g2((unsigned)ceil_div(ncols, 2));
                if (rows <= 1024) qr_apply_wy_kernel<8, 1, 4><<<g4, 1024, 0, st>>>(X, s, p0, nb, ncols, Vp, Tp);
                else if (rows <= 2048) qr_apply_wy_kernel<8, 2, 4><<<g4, 1024, 0, st>>>(X, s, p0, nb, ncols, Vp, Tp);
                else if (rows <= 4096) qr_apply_wy_kernel<8, 4, 4><<<g4, 1024, 0, st>>>(X, s, p0, nb, ncols, Vp, Tp);
                else qr_apply_wy_kernel<4, 8, 2><<<g2, 1024, 0, st>>>(X, s, p0, nb, ncols, Vp, Tp);
                LSRN_HIP(hipGetLastError());
            }
            p0 += nb;
        }
        LSRN_HIP(hipStreamSynchronize(st));  // before the panel buffers are freed
        return;
    }
    // taller sketches: panels of 32 columns in global memory
    const int pw = QNB;
    for (int64_t p0 = 0; p0 < d; p0 += pw) {
        const int nb = (int)std::min<int64_t>(pw, d - p0);
        double *Vp = Vb.as<double>(), *bp = betab.as<double>();
        if (s <= 1024) qr_panel_reg_kernel<8, 1><<<1, 1024, 0, st>>>(X, s, p0, nb, Vp, bp);
        else if (s <= 2048) qr_panel_reg_kernel<8, 2><<<1, 1024, 0, st>>>(X, s, p0, nb, Vp, bp);
        else if (s <= 4096) qr_panel_reg_kernel<8, 4><<<1, 1024, 0, st>>>(X, s, p0, nb, Vp, bp);
        else if (s <= 8192) qr_panel_reg_kernel<4, 8><<<1, 1024, 0, st>>>(X, s, p0, nb, Vp, bp);
        else qr_panel_kernel<<<1, 1024, 0, st>>>(X, s, p0, nb, Vp, bp);
        LSRN_HIP(hipGetLastError());
        const int64_t ncols = d - p0 - nb;
        if (ncols > 0) {
            const int64_t rows = s - p0;
            if (rows <= 256 * 4) launch_apply<256, 4>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            else if (rows <= 256 * 8) launch_apply<256, 8>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            else if (rows <= 256 * 16) launch_apply<256, 16>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            else if (rows <= 256 * 32) launch_apply<256, 32>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            else if (rows <= 1024 * 16) launch_apply<1024, 16>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            else launch_apply<1024, 40>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            LSRN_HIP(hipGetLastError());
        }
    }

    LSRN_HIP(hipStreamSynchronize(st));  // before the panel buffers are freed
}

namespace {

constexpr int kJacobiMaxSweeps = 60;

// Which Jacobi kernel a d x d matrix Y = R^T uses, and its padded width:
// the whole matrix in LDS for d <= 128, else the Gram round kernel with the
// widest column block whose 2 BW register columns fit next to the
// reduction.
struct JacobiPlan {
    bool small = false;
    int variant = -1;  // index into the round-kernel tables
    int64_t nblocks = 0, dcols = 0;
};

JacobiPlan jacobi_plan(int64_t d) {
    static const int kBW[] = {8, 8, 8, 4, 2}, kDMAX[] = {512, 1024, 2048, 4096, 8192};
    JacobiPlan pl;
    for (int v = 0; v < 5 && pl.variant < 0; ++v)
        if (d <= kDMAX[v]) pl.variant = v;
    pl.small = (size_t)d * (size_t)d * sizeof(double) <= lds_limit() && d <= 128;
    if (!pl.small && pl.variant < 0)
        fail(LSRN_E_UNSUPPORTED, "precond: the Jacobi kernels support min(m, n) <= 8192");
    const int bw = pl.variant >= 0 ? kBW[pl.variant] : 1;
    pl.nblocks = ceil_div(d, bw);
    pl.nblocks += pl.nblocks & 1;
    pl.dcols = pl.small ? d : pl.nblocks * bw;
    return pl;
}

// The small-matrix Jacobi kernels use d^2 doubles of dynamic LDS, at most
// 128 KiB (d <= 128); the attribute is raised once per process, not per
// call, which solves on several host threads would do concurrently.
void set_small_lds(size_t bytes) {
    static std::once_flag once;
    if (bytes <= 65536) return;
    std::call_once(once, [] {
        const int lim = 128 * 1024;
        LSRN_HIP(hipFuncSetAttribute((const void *)jacobi_small_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        LSRN_HIP(hipFuncSetAttribute((const void *)jacobi_small_batch_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    });
}

// Squared threshold below which two columns are not rotated against each
// other, per problem: tau = rcond max_j |y_j| / (2 sqrt d).  A rotation
// leaves the smaller column of its pair no larger, and pairs of columns
// both within tau are skipped, so the columns that end within tau have a
// Frobenius norm of at most sqrt(d) tau <= rcond sigma_1 / 2 (max_j |y_j|
// <= sigma_1): their singular values stay below the rank cutoff, while
// every column above tau is orthogonalised against all others as usual.
// The kept part of the SVD is therefore unchanged; the rounding-level
// columns of a rank-deficient sketch stop costing sweeps.
std::vector<double> tiny_thresholds2(int count, const double *const *Y, const int64_t *s,
                                     const int64_t *d, double rcond, hipStream_t st) {
    std::vector<size_t> off((size_t)count + 1, 0);
    for (int p = 0; p < count; ++p) off[(size_t)p + 1] = off[(size_t)p] + (size_t)d[p];
    DevBuf nrm(std::max<size_t>(off[(size_t)count], 1) * sizeof(double));
    for (int p = 0; p < count; ++p)
        col_norms_kernel<<<(unsigned)ceil_div(d[p], 4), 256, 0, st>>>(Y[p], d[p], nrm.as<double>() + off[(size_t)p]);
    LSRN_HIP(hipGetLastError());
    std::vector<double> h(off[(size_t)count]);
    LSRN_HIP(hipMemcpyAsync(h.data(), nrm.as<double>(), h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LSRN_HIP(hipStreamSynchronize(st));
    std::vector<double> t2((size_t)count);
    for (int p = 0; p < count; ++p) {
        double mx = 0.0;
        for (size_t j = off[(size_t)p]; j < off[(size_t)p + 1]; ++j) mx = std::max(mx, h[j]);
        const double rc = rcond > 0.0 ? rcond : (double)std::max(s[p], d[p]) * DBL_EPSILON;
        const double tau = rc * mx / (2.0 * std::sqrt((double)d[p]));
        t2[(size_t)p] = tau * tau;
    }
    return t2;
}

// All sweeps of one problem; returns the sweep count.
int64_t jacobi_single(double *Y, int64_t d, const JacobiPlan &pl, hipStream_t st, bool profile,
                      PrecondResult &res, double tiny2) {
    const double tol = (double)d * DBL_EPSILON;
    DevBuf cnt(2 * sizeof(int));
    int *dcnt = cnt.as<int>();
    if (pl.small) {
        const size_t bytes = (size_t)d * d * sizeof(double);
        set_small_lds(bytes);
        jacobi_small_kernel<<<1, 1024, bytes, st>>>(Y, (int)d, kJacobiMaxSweeps, tol, tiny2, dcnt);
        LSRN_HIP(hipGetLastError());
        int sw = 0;
        LSRN_HIP(hipMemcpyAsync(&sw, dcnt, sizeof(int), hipMemcpyDeviceToHost, st));
        LSRN_HIP(hipStreamSynchronize(st));
        return sw;
    }
    typedef void (*RoundFn)(double *, int, int, int, double, double, int *, int *, int);
    static const RoundFn kFn[] = {jacobi_gram_round_kernel<8, 1>, jacobi_gram_round_kernel<8, 2>,
                                  jacobi_gram_round_kernel<8, 4>, jacobi_gram_round_kernel<4, 8>,
                                  jacobi_gram_round_kernel<2, 16>};
    const RoundFn fn = kFn[pl.variant];
    const int64_t nblocks = pl.nblocks;
    DevBuf lastb((size_t)nblocks * sizeof(int));
    int *last_mod = lastb.as<int>();
    LSRN_HIP(hipMemsetAsync(last_mod, 0, (size_t)nblocks * sizeof(int), st));
    const int period = (int)nblocks - 1;
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (profile) {
        LSRN_HIP(hipEventCreate(&ev[0]));
        LSRN_HIP(hipEventCreate(&ev[1]));
    }
    int sweep = 0;
    for (; sweep < kJacobiMaxSweeps; ++sweep) {
        LSRN_HIP(hipMemsetAsync(dcnt, 0, sizeof(int), st));
        if (profile) LSRN_HIP(hipEventRecord(ev[0], st));
        for (int round = 0; round < period; ++round) {
            hipLaunchKernelGGL(fn, dim3((unsigned)(nblocks / 2)), dim3(512), 0, st, Y, (int)d,
                               (int)nblocks, round, tol, tiny2, dcnt, last_mod, sweep * period + round);
        }
        LSRN_HIP(hipGetLastError());
        if (profile) LSRN_HIP(hipEventRecord(ev[1], st));
        int rot = 0;
        LSRN_HIP(hipMemcpyAsync(&rot, dcnt, sizeof(int), hipMemcpyDeviceToHost, st));
        LSRN_HIP(hipStreamSynchronize(st));
        if (profile) {
            float ms = 0.f;
            LSRN_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
            res.t_jacobi_kernel_ms += ms;
            res.jacobi_kernels += period;
        }
        if (rot == 0) break;
    }
    if (profile) {
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
    }
    return std::min(sweep + 1, kJacobiMaxSweeps);
}

// Singular values (column norms of the converged Y), their order, the rank
// cutoff and P = Y(:, order) Sigma^-2 for the kept columns.
void precond_finish(int64_t s, int64_t d, const double *Y, double rcond, double *sigma, double *P,
                    PrecondResult &res, hipStream_t st) {
    DevBuf nrmb((size_t)d * sizeof(double)), ordb((size_t)d * sizeof(int64_t));
    col_norms_kernel<<<(unsigned)ceil_div(d, 4), 256, 0, st>>>(Y, d, nrmb.as<double>());
    rank_sort_kernel<<<(unsigned)ceil_div(d, 256), 256, 0, st>>>(nrmb.as<double>(), d,
                                                                  ordb.as<int64_t>(), sigma);
    LSRN_HIP(hipGetLastError());
    std::vector<double> hs((size_t)d);
    LSRN_HIP(hipMemcpyAsync(hs.data(), sigma, (size_t)d * sizeof(double), hipMemcpyDeviceToHost, st));
    LSRN_HIP(hipStreamSynchronize(st));
    if (rcond <= 0.0) rcond = (double)std::max(s, d) * DBL_EPSILON;
    int64_t r = 0;
    while (r < d && hs[0] > 0.0 && hs[(size_t)r] > rcond * hs[0]) ++r;
    res.rank = r;
    res.sigma_max = hs[0];
    res.sigma_min_kept = r > 0 ? hs[(size_t)r - 1] : 0.0;
    if (r > 0) {
        form_p_kernel<<<grid1d(d * r), 256, 0, st>>>(Y, d, r, ordb.as<int64_t>(), sigma, P);
        LSRN_HIP(hipGetLastError());
    }
    LSRN_HIP(hipStreamSynchronize(st));
}

// Sums of squares of the upper triangle of R (column j: rows 0 .. j, leading
// dimension ldr) and of all of Ri (d x d, leading dimension d), one
// workgroup per column: part[j] and part[d + j].
__global__ void __launch_bounds__(256)
col_sumsq_kernel(const double *__restrict__ R, int64_t ldr, const double *__restrict__ Ri, int64_t d,
                 double *__restrict__ part) {
    __shared__ double red[2][4];
    const int64_t j = blockIdx.x;
    const int tid = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t i = tid; i <= j; i += 256) {
        const double v = R[j * ldr + i];
        a += v * v;
    }
    for (int64_t i = tid; i < d; i += 256) {
        const double v = Ri[j * d + i];
        b += v * v;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = a;
        red[1][tid >> 6] = b;
    }
    __syncthreads();
    if (tid < 2) part[tid * d + j] = red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
}

// y = M x for a row-major d x d M (leading dimension ld): one wavefront per
// row, lanes over the columns, the wavefront's fixed butterfly.
__global__ void __launch_bounds__(256)
gemv_sq_kernel(const double *__restrict__ M, int64_t ld, int64_t d, const double *__restrict__ x,
               double *__restrict__ y) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= d) return;
    const int lane = threadIdx.x & 63;
    double t = 0.0;
    for (int64_t j = lane; j < d; j += 64) t += M[row * ld + j] * x[j];
    t = wave_sum(t);
    if (lane == 0) y[row] = t;
}

// v <- v / |v| (one workgroup); out[0] = |v|.
__global__ void __launch_bounds__(1024) normalize_kernel(double *__restrict__ v, int64_t d,
                                                         double *__restrict__ out) {
    __shared__ double red[16];
    const int tid = threadIdx.x;
    double t = 0.0;
    for (int64_t i = tid; i < d; i += 1024) t += v[i] * v[i];
    t = wave_sum(t);
    if ((tid & 63) == 0) red[tid >> 6] = t;
    __syncthreads();
    if (tid == 0) {
        double a = 0.0;
        for (int w = 0; w < 16; ++w) a += red[w];
        red[0] = sqrt(a);
        out[0] = red[0];
    }
    __syncthreads();
    const double nv = red[0];
    if (nv > 0.0)
        for (int64_t i = tid; i < d; i += 1024) v[i] /= nv;
}

// |R^-1|_2^2 estimated by eight power steps on R^-T R^-1 from a uniform
// start (P is R^-1 row-major, Ri, column-major, is R^-T row-major): a lower
// bound, within a small factor for such sketches.  Synchronises.
double inv_norm2_sq(int64_t d, const double *P, const double *Ri, hipStream_t st) {
    DevBuf vb((size_t)2 * d * sizeof(double)), nb(sizeof(double));
    std::vector<double> v0((size_t)d, 1.0 / std::sqrt((double)d));
    LSRN_HIP(hipMemcpyAsync(vb.as<double>(), v0.data(), (size_t)d * sizeof(double), hipMemcpyHostToDevice, st));
    double *v = vb.as<double>(), *u = vb.as<double>() + d;
    for (int it = 0; it < 8; ++it) {
        gemv_sq_kernel<<<(unsigned)ceil_div(d, 4), 256, 0, st>>>(P, d, d, v, u);
        gemv_sq_kernel<<<(unsigned)ceil_div(d, 4), 256, 0, st>>>(Ri, d, d, u, v);
        normalize_kernel<<<1, 1024, 0, st>>>(v, d, nb.as<double>());
    }
    LSRN_HIP(hipGetLastError());
    double lam = 0.0;
    LSRN_HIP(hipMemcpyAsync(&lam, nb.as<double>(), sizeof(double), hipMemcpyDeviceToHost, st));
    LSRN_HIP(hipStreamSynchronize(st));  // before v0 and the buffers go
    return lam;
}

// The full-rank case of steps 4-5 without the Jacobi sweeps.  With X = Q R,
// N = R^-1 gives T N the singular values of T V Sigma^-1 (R^-1 = V Sigma^-1
// times an orthogonal factor), so it preconditions as well (reading of
// Sec. 4 on the range and spectrum of N).  It is taken only when the SVD
// would keep every singular value: kappa_2(R) <= |R|_F |R^-1|_F, so
// |R|_F |R^-1|_F <= 1 / (2 rc) certifies sigma_min > rc sigma_1, the
// cutoff of the SVD path.  sigma receives |diag R| in descending order;
// sigma_max / sigma_min_kept are estimates of sigma_1 and sigma_d (below).
// False (nothing written to P) otherwise.
bool full_rank_inverse(int64_t s, int64_t d, const double *R, double rcond, double *sigma, double *P,
                       PrecondResult &res, hipStream_t st) {
    const double rc = rcond > 0.0 ? rcond : (double)std::max(s, d) * DBL_EPSILON;
    DevBuf Ri((size_t)d * (size_t)d * sizeof(double)), part((size_t)2 * d * sizeof(double));
    trtri_upper(d, R, s, Ri.as<double>(), d, st);
    col_sumsq_kernel<<<(unsigned)d, 256, 0, st>>>(R, s, Ri.as<double>(), d, part.as<double>());
    LSRN_HIP(hipGetLastError());
    std::vector<double> h((size_t)2 * d);
    LSRN_HIP(hipMemcpyAsync(h.data(), part.as<double>(), h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LSRN_HIP(hipStreamSynchronize(st));
    double sr = 0.0, si = 0.0;
    for (int64_t j = 0; j < d; ++j) {
        sr += h[(size_t)j];
        si += h[(size_t)(d + j)];
    }
    const double nr = std::sqrt(sr), ni = std::sqrt(si);
    if (!(nr > 0.0 && nr * ni <= 0.5 / rc)) return false;  // NaN / inf fail too
    transpose(d, d, Ri.as<double>(), d, P, st);  // P row-major = R^-1
    diag_abs_kernel<<<grid1d(d), 256, 0, st>>>(R, s, d, sigma);
    LSRN_HIP(hipGetLastError());
    std::vector<double> g((size_t)d);
    LSRN_HIP(hipMemcpyAsync(g.data(), sigma, (size_t)d * sizeof(double), hipMemcpyDeviceToHost, st));
    LSRN_HIP(hipStreamSynchronize(st));
    std::sort(g.begin(), g.end(), [](double a, double b) { return a > b; });
    LSRN_HIP(hipMemcpyAsync(sigma, g.data(), (size_t)d * sizeof(double), hipMemcpyHostToDevice, st));
    // estimates of the extreme singular values of R (the precision form
    // chooses FP32 or FP64 sweeps from their ratio): the largest column norm
    // of R for sigma_1, and 1 / |R^-1|_2 for sigma_d with |R^-1|_2 from eight
    // power steps on R^-T R^-1 (P is R^-1 row-major; Ri, column-major, is
    // R^-T row-major).  Both are lower bounds on the true values, each within
    // a small factor for such sketches.
    double cmax = 0.0;
    for (int64_t j = 0; j < d; ++j) cmax = std::max(cmax, h[(size_t)j]);
    const double lam = inv_norm2_sq(d, P, Ri.as<double>(), st);
    res.rank = d;
    res.sweeps = 0;
    res.sigma_max = std::sqrt(cmax);
    res.sigma_min_kept = lam > 0.0 ? 1.0 / std::sqrt(lam) : g[(size_t)d - 1];
    res.full_rank_inverse = true;
    return true;
}

}  // namespace

PrecondResult precond(int64_t s, int64_t d, double *X, double rcond, double *sigma, double *P,
                      hipStream_t st, bool profile, bool try_full_rank) {
    LSRN_REQUIRE(s >= d && d > 0, "precond: need s >= d > 0");
    PrecondResult res;
    householder_qr(s, d, X, st);
    if (try_full_rank && full_rank_inverse(s, d, X, rcond, sigma, P, res, st)) return res;
    // ---- Jacobi on Y = R^T
    const JacobiPlan pl = jacobi_plan(d);
    DevBuf Yb((size_t)d * (size_t)pl.dcols * sizeof(double));
    double *Y = Yb.as<double>();
    r_to_y_kernel<<<grid1d(d * pl.dcols), 256, 0, st>>>(X, s, d, pl.dcols, Y);
    LSRN_HIP(hipGetLastError());
    const double *Yc = Y;
    const double tiny2 = tiny_thresholds2(1, &Yc, &s, &d, rcond, st)[0];
    res.sweeps = jacobi_single(Y, d, pl, st, profile, res, tiny2);
    precond_finish(s, d, Y, rcond, sigma, P, res, st);
    return res;
}

namespace {

// One problem of a batched triangular inverse (d <= 512).
struct TriInvItem {
    const double *R;  // upper triangle, column-major, leading dimension ldr
    int64_t ldr;
    int d;
    double *P;     // R^-1, row-major d x d
    double *part;  // [0, d): |R(:, j)|^2; [d, 2d): |R^-1(:, j)|^2; [2d, 3d): |r_jj|
};

// Column j of R^-1 for every problem of a batch (workgroup g: column
// g - off[p] of problem p): back substitution on R y = e_j, the right-hand
// side in LDS, one row a step from j down to 0 (step k reads only x_k and
// updates only x_i, i < k, so one barrier a step suffices).
__global__ void __launch_bounds__(256)
trinv_col_batch_kernel(const TriInvItem *__restrict__ items, const int *__restrict__ off, int n) {
    __shared__ double xs[512], ys[512];
    __shared__ double red[2][4];
    const int g = (int)blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    const TriInvItem it = items[lo];
    const int j = g - off[lo], d = it.d, tid = (int)threadIdx.x;
    const double *__restrict__ R = it.R;
    for (int i = tid; i <= j; i += 256) xs[i] = i == j ? 1.0 : 0.0;
    __syncthreads();
    for (int k = j; k >= 0; --k) {
        const double *__restrict__ rk = R + (int64_t)k * it.ldr;
        const double yk = xs[k] / rk[k];
        if (tid == 0) ys[k] = yk;
        for (int i = tid; i < k; i += 256) xs[i] -= rk[i] * yk;
        __syncthreads();
    }
    double sy = 0.0, sr = 0.0;
    const double *__restrict__ rj = R + (int64_t)j * it.ldr;
    for (int i = tid; i < d; i += 256) {
        const double y = i <= j ? ys[i] : 0.0;
        it.P[(int64_t)i * d + j] = y;
        sy += y * y;
        if (i <= j) sr += rj[i] * rj[i];
    }
    sy = wave_sum(sy);
    sr = wave_sum(sr);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = sr;
        red[1][tid >> 6] = sy;
    }
    __syncthreads();
    if (tid == 0) {
        it.part[j] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        it.part[d + j] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
        it.part[2 * d + j] = fabs(rj[j]);
    }
}

// The full-rank case of full_rank_inverse for the problems of a batch that
// try it, in one launch and one read-back: P = R^-1 where |R|_F |R^-1|_F
// <= 1 / (2 rc) certifies that the SVD would keep every singular value
// (done[p] = 1; sigma = |diag R| descending; sigma_min_kept = 1 / |R^-1|_F,
// a lower bound on sigma_d).  The others are left to the SVD.
void certified_inverse_batch(int count, const int64_t *s, const int64_t *d, double *const *X, double rcond,
                             double *const *sigma, double *const *P, PrecondResult *res,
                             const char *try_fr, std::vector<char> &done, hipStream_t st) {
    std::vector<TriInvItem> items;
    std::vector<int> off(1, 0), ids;
    std::vector<size_t> po;
    size_t ptot = 0;
    for (int p = 0; p < count; ++p) {
        if (!try_fr[p]) continue;
        LSRN_REQUIRE(d[p] <= 512, "batched certified inverse: d <= 512");
        ids.push_back(p);
        po.push_back(ptot);
        ptot += (size_t)3 * (size_t)d[p];
        off.push_back(off.back() + (int)d[p]);
    }
    if (ids.empty()) return;
    const int n = (int)ids.size();
    DevBuf part(ptot * sizeof(double));
    for (int k = 0; k < n; ++k) {
        const int p = ids[(size_t)k];
        items.push_back(TriInvItem{X[p], s[p], (int)d[p], P[p], part.as<double>() + po[(size_t)k]});
    }
    DevBuf ditems((size_t)n * sizeof(TriInvItem)), doff(off.size() * sizeof(int));
    LSRN_HIP(hipMemcpyAsync(ditems.as<TriInvItem>(), items.data(), (size_t)n * sizeof(TriInvItem),
                            hipMemcpyHostToDevice, st));
    LSRN_HIP(hipMemcpyAsync(doff.as<int>(), off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, st));
    trinv_col_batch_kernel<<<(unsigned)off.back(), 256, 0, st>>>(ditems.as<TriInvItem>(), doff.as<int>(), n);
    LSRN_HIP(hipGetLastError());
    std::vector<double> h(ptot);
    LSRN_HIP(hipMemcpyAsync(h.data(), part.as<double>(), ptot * sizeof(double), hipMemcpyDeviceToHost, st));
    LSRN_HIP(hipStreamSynchronize(st));
    std::vector<double> sig(ptot);  // sorted |diag R| of each certified problem
    for (int k = 0; k < n; ++k) {
        const int p = ids[(size_t)k];
        const int64_t dp = d[p];
        const double *hp = h.data() + po[(size_t)k];
        double sr = 0.0, si = 0.0, cmax = 0.0;
        for (int64_t j = 0; j < dp; ++j) {
            sr += hp[j];
            si += hp[dp + j];
            cmax = std::max(cmax, hp[j]);
        }
        const double rc = rcond > 0.0 ? rcond : (double)std::max(s[p], dp) * DBL_EPSILON;
        const double nr = std::sqrt(sr), ni = std::sqrt(si);
        if (!(nr > 0.0 && nr * ni <= 0.5 / rc)) continue;  // NaN / inf fail too
        double *g = sig.data() + po[(size_t)k];
        std::copy(hp + 2 * dp, hp + 3 * dp, g);
        std::sort(g, g + dp, [](double a, double b) { return a > b; });
        LSRN_HIP(hipMemcpyAsync(sigma[p], g, (size_t)dp * sizeof(double), hipMemcpyHostToDevice, st));
        res[p] = PrecondResult();
        res[p].rank = dp;
        res[p].sweeps = 0;
        res[p].sigma_max = std::sqrt(cmax);
        res[p].sigma_min_kept = 1.0 / ni;
        res[p].full_rank_inverse = true;
        done[(size_t)p] = 1;
    }
    LSRN_HIP(hipStreamSynchronize(st));  // before sig and the buffers go
}

// Steps 4-5 after the QR for a batch: Jacobi on Y = R^T, sigma, rank, P.
void svd_batch(int count, const int64_t *s, const int64_t *d, double *const *X, double rcond,
               double *const *sigma, double *const *P, PrecondResult *res, hipStream_t st);

}  // namespace

void precond_batch(int count, const int64_t *s, const int64_t *d, double *const *X, double rcond,
                   double *const *sigma, double *const *P, PrecondResult *res, hipStream_t st,
                   const char *try_fr) {
    // ---- QR: sketches of up to 1024 rows factor together, one launch per
    // panel step for all of them; taller ones one at a time
    {
        std::vector<QrItem> qi;
        int64_t vtotal = 0, dmax = 0;
        for (int p = 0; p < count; ++p) {
            LSRN_REQUIRE(s[p] >= d[p] && d[p] > 0, "precond: need s >= d > 0");
            if (s[p] <= 1024) {
                qi.push_back(QrItem{X[p], s[p], d[p], nullptr, nullptr});
                vtotal += s[p] * QNB;
                dmax = std::max(dmax, d[p]);
            } else {
                householder_qr(s[p], d[p], X[p], st);
            }
        }
        if (!qi.empty()) {
            const int n = (int)qi.size();
            DevBuf Vb((size_t)vtotal * sizeof(double)), bb((size_t)n * QNB * sizeof(double));
            int64_t vo = 0;
            for (int k = 0; k < n; ++k) {
                qi[(size_t)k].V = Vb.as<double>() + vo;
                qi[(size_t)k].beta = bb.as<double>() + (size_t)k * QNB;
                vo += qi[(size_t)k].s * QNB;
            }
            DevBuf ditems((size_t)n * sizeof(QrItem));
            LSRN_HIP(hipMemcpyAsync(ditems.as<QrItem>(), qi.data(), (size_t)n * sizeof(QrItem),
                                    hipMemcpyHostToDevice, st));
            const int pw = 8;
            for (int64_t p0 = 0; p0 < dmax; p0 += pw) {
                qr_panel_reg_batch_kernel<8, 1><<<(unsigned)n, 1024, 0, st>>>(ditems.as<QrItem>(), p0, pw);
                const int64_t ncols = dmax - p0 - std::min<int64_t>(pw, dmax - p0);
                if (ncols > 0)
                    qr_apply_batch_kernel<256, 4><<<dim3((unsigned)n, (unsigned)ncols), 256, 0, st>>>(
                        ditems.as<QrItem>(), p0, pw);
                LSRN_HIP(hipGetLastError());
            }
            LSRN_HIP(hipStreamSynchronize(st));  // before the panel buffers are freed
        }
    }
    std::vector<char> done((size_t)count, 0);
    if (try_fr) certified_inverse_batch(count, s, d, X, rcond, sigma, P, res, try_fr, done, st);
    std::vector<int> rest;
    for (int p = 0; p < count; ++p)
        if (!done[(size_t)p]) rest.push_back(p);
    if (rest.empty()) return;
    if ((int)rest.size() == count) {
        svd_batch(count, s, d, X, rcond, sigma, P, res, st);
        return;
    }
    const size_t nr = rest.size();
    std::vector<int64_t> s2(nr), d2(nr);
    std::vector<double *> X2(nr), sig2(nr), P2(nr);
    std::vector<PrecondResult> r2(nr);
    for (size_t k = 0; k < nr; ++k) {
        const int p = rest[k];
        s2[k] = s[p]; d2[k] = d[p]; X2[k] = X[p]; sig2[k] = sigma[p]; P2[k] = P[p];
    }
    svd_batch((int)nr, s2.data(), d2.data(), X2.data(), rcond, sig2.data(), P2.data(), r2.data(), st);
    for (size_t k = 0; k < nr; ++k) res[rest[k]] = r2[k];
}

namespace {

void svd_batch(int count, const int64_t *s, const int64_t *d, double *const *X, double rcond,
               double *const *sigma, double *const *P, PrecondResult *res, hipStream_t st) {
    std::vector<JacobiPlan> pl((size_t)count);
    std::vector<double *> Yb((size_t)count);  // carved from one allocation
    std::vector<int> small_ids, gram_ids, other_ids;
    size_t ytotal = 0;
    for (int p = 0; p < count; ++p) {
        pl[(size_t)p] = jacobi_plan(d[p]);
        ytotal += ((size_t)d[p] * (size_t)pl[(size_t)p].dcols + 31) & ~(size_t)31;
    }
    DevBuf Ypool(std::max<size_t>(ytotal, 1) * sizeof(double));
    size_t yused = 0;
    for (int p = 0; p < count; ++p) {
        res[p] = PrecondResult();
        Yb[(size_t)p] = Ypool.as<double>() + yused;
        yused += ((size_t)d[p] * (size_t)pl[(size_t)p].dcols + 31) & ~(size_t)31;
        r_to_y_kernel<<<grid1d(d[p] * pl[(size_t)p].dcols), 256, 0, st>>>(
            X[p], s[p], d[p], pl[(size_t)p].dcols, Yb[(size_t)p]);
        LSRN_HIP(hipGetLastError());
        if (pl[(size_t)p].small) small_ids.push_back(p);
        else if (pl[(size_t)p].variant == 0) gram_ids.push_back(p);
        else other_ids.push_back(p);
    }
    std::vector<const double *> Ycs(Yb.begin(), Yb.end());
    const std::vector<double> tiny2 = tiny_thresholds2(count, Ycs.data(), s, d, rcond, st);
    // ---- d <= 128: one workgroup per problem, all sweeps, one launch
    if (!small_ids.empty()) {
        const int n = (int)small_ids.size();
        std::vector<JacobiItem> it((size_t)n);
        size_t bytes = 0;
        for (int k = 0; k < n; ++k) {
            const int p = small_ids[(size_t)k];
            it[(size_t)k] = JacobiItem{Yb[(size_t)p], (int)d[p], 0,
                                       (double)d[p] * DBL_EPSILON, tiny2[(size_t)p], nullptr, nullptr};
            bytes = std::max(bytes, (size_t)d[p] * (size_t)d[p] * sizeof(double));
        }
        DevBuf ditems((size_t)n * sizeof(JacobiItem)), dsw((size_t)n * sizeof(int));
        LSRN_HIP(hipMemcpyAsync(ditems.as<JacobiItem>(), it.data(), (size_t)n * sizeof(JacobiItem),
                                hipMemcpyHostToDevice, st));
        set_small_lds(bytes);
        jacobi_small_batch_kernel<<<(unsigned)n, 1024, bytes, st>>>(ditems.as<JacobiItem>(),
                                                                     kJacobiMaxSweeps, dsw.as<int>());
        LSRN_HIP(hipGetLastError());
        std::vector<int> sw((size_t)n);
        LSRN_HIP(hipMemcpyAsync(sw.data(), dsw.as<int>(), (size_t)n * sizeof(int), hipMemcpyDeviceToHost, st));
        LSRN_HIP(hipStreamSynchronize(st));
        for (int k = 0; k < n; ++k) res[small_ids[(size_t)k]].sweeps = sw[(size_t)k];
    }
    // ---- 128 < d <= 512: every problem's round r in one launch, one host
    // check per sweep for the whole batch
    if (!gram_ids.empty()) {
        const int n = (int)gram_ids.size();
        std::vector<JacobiItem> it((size_t)n);
        std::vector<int> off((size_t)n + 1, 0), lastoff((size_t)n + 1, 0), active((size_t)n, 1);
        int max_period = 0;
        for (int k = 0; k < n; ++k) {
            const int64_t nb = pl[(size_t)gram_ids[(size_t)k]].nblocks;
            off[(size_t)k + 1] = off[(size_t)k] + (int)(nb / 2);
            lastoff[(size_t)k + 1] = lastoff[(size_t)k] + (int)nb;
            max_period = std::max(max_period, (int)nb - 1);
        }
        DevBuf ditems((size_t)n * sizeof(JacobiItem)), doff(((size_t)n + 1) * sizeof(int));
        DevBuf dact((size_t)n * sizeof(int)), drot((size_t)n * sizeof(int));
        DevBuf dlast((size_t)lastoff[(size_t)n] * sizeof(int));
        for (int k = 0; k < n; ++k) {
            const int p = gram_ids[(size_t)k];
            it[(size_t)k] = JacobiItem{Yb[(size_t)p], (int)d[p], (int)pl[(size_t)p].nblocks,
                                       (double)d[p] * DBL_EPSILON, tiny2[(size_t)p], drot.as<int>() + k,
                                       dlast.as<int>() + lastoff[(size_t)k]};
        }
        LSRN_HIP(hipMemcpyAsync(ditems.as<JacobiItem>(), it.data(), (size_t)n * sizeof(JacobiItem),
                                hipMemcpyHostToDevice, st));
        LSRN_HIP(hipMemcpyAsync(doff.as<int>(), off.data(), ((size_t)n + 1) * sizeof(int),
                                hipMemcpyHostToDevice, st));
        LSRN_HIP(hipMemsetAsync(dlast.as<int>(), 0, (size_t)lastoff[(size_t)n] * sizeof(int), st));
        std::vector<int> rot((size_t)n);
        int left = n;
        for (int sweep = 0; sweep < kJacobiMaxSweeps && left > 0; ++sweep) {
            LSRN_HIP(hipMemsetAsync(drot.as<int>(), 0, (size_t)n * sizeof(int), st));
            LSRN_HIP(hipMemcpyAsync(dact.as<int>(), active.data(), (size_t)n * sizeof(int),
                                    hipMemcpyHostToDevice, st));
            for (int round = 0; round < max_period; ++round)
                jacobi_gram_round_batch_kernel<8, 1><<<(unsigned)off[(size_t)n], 512, 0, st>>>(
                    ditems.as<JacobiItem>(), doff.as<int>(), dact.as<int>(), n, round, sweep);
            LSRN_HIP(hipGetLastError());
            LSRN_HIP(hipMemcpyAsync(rot.data(), drot.as<int>(), (size_t)n * sizeof(int),
                                    hipMemcpyDeviceToHost, st));
            LSRN_HIP(hipStreamSynchronize(st));
            for (int k = 0; k < n; ++k) {
                if (!active[(size_t)k]) continue;
                res[gram_ids[(size_t)k]].sweeps = sweep + 1;
                if (rot[(size_t)k] == 0) {
                    active[(size_t)k] = 0;
                    --left;
                }
            }
        }
    }
    // ---- wider problems: one at a time
    for (int p : other_ids)
        res[p].sweeps = jacobi_single(Yb[(size_t)p], d[p], pl[(size_t)p], st, false, res[p], tiny2[(size_t)p]);
    // sigma, order and P of every problem: the norms and sorts in one pass
    // of launches, one read-back of all sigmas, then the P of each
    std::vector<size_t> so((size_t)count + 1, 0);
    for (int p = 0; p < count; ++p) so[(size_t)p + 1] = so[(size_t)p] + (size_t)d[p];
    DevBuf nrmb(so[(size_t)count] * sizeof(double)), ordb(so[(size_t)count] * sizeof(int64_t));
    std::vector<double> hs(so[(size_t)count]);
    for (int p = 0; p < count; ++p) {
        double *nrm = nrmb.as<double>() + so[(size_t)p];
        int64_t *ord = ordb.as<int64_t>() + so[(size_t)p];
        col_norms_kernel<<<(unsigned)ceil_div(d[p], 4), 256, 0, st>>>(Yb[(size_t)p], d[p], nrm);
        rank_sort_kernel<<<(unsigned)ceil_div(d[p], 256), 256, 0, st>>>(nrm, d[p], ord, sigma[p]);
        LSRN_HIP(hipGetLastError());
        LSRN_HIP(hipMemcpyAsync(hs.data() + so[(size_t)p], sigma[p], (size_t)d[p] * sizeof(double),
                                hipMemcpyDeviceToHost, st));
    }
    LSRN_HIP(hipStreamSynchronize(st));
    for (int p = 0; p < count; ++p) {
        const double *h = hs.data() + so[(size_t)p];
        const double rc = rcond > 0.0 ? rcond : (double)std::max(s[p], d[p]) * DBL_EPSILON;
        int64_t r = 0;
        while (r < d[p] && h[0] > 0.0 && h[r] > rc * h[0]) ++r;
        res[p].rank = r;
        res[p].sigma_max = h[0];
        res[p].sigma_min_kept = r > 0 ? h[r - 1] : 0.0;
        if (r > 0) {
            form_p_kernel<<<grid1d(d[p] * r), 256, 0, st>>>(Yb[(size_t)p], d[p], r,
                                                            ordb.as<int64_t>() + so[(size_t)p], sigma[p], P[p]);
            LSRN_HIP(hipGetLastError());
        }
    }
    LSRN_HIP(hipStreamSynchronize(st));
}

}  // namespace

PrecondResult precond_qr_inverse(int64_t s, int64_t d, double *X, double rcond, double *sigma,
                                 double *P, hipStream_t st) {
    LSRN_REQUIRE(s >= d && d > 0, "precond: need s >= d > 0");
    PrecondResult res;
    const double rc = rcond > 0.0 ? rcond : (double)std::max(s, d) * DBL_EPSILON;
    std::vector<double> h((size_t)d);
    auto sorted_diag = [&](const double *R, int64_t ldr) {
        diag_abs_kernel<<<grid1d(d), 256, 0, st>>>(R, ldr, d, sigma);
        LSRN_HIP(hipGetLastError());
        LSRN_HIP(hipMemcpyAsync(h.data(), sigma, (size_t)d * sizeof(double), hipMemcpyDeviceToHost, st));
        LSRN_HIP(hipStreamSynchronize(st));
        std::sort(h.begin(), h.end(), [](double a, double b) { return a > b; });
    };
    // Cholesky QR: R^T R = X^T X from the upper triangle of the Gram matrix
    // (one FP64 MFMA product, then a blocked Cholesky).  X R^-1 is then
    // orthonormal to about d eps kappa(X)^2, so it is kept only while an
    // estimate of kappa(R) (largest column norm of R times |R^-1|_2 from
    // power steps, both from below, hence the margin) keeps d eps kappa^2
    // below 1e-5; max r_ii / min r_ii, a cheaper lower bound, screens first.
    // Otherwise, or when a pivot is not positive, Householder QR of X (for
    // up to 40960 sketch rows; beyond that the call fails).
    DevBuf gram((size_t)d * (size_t)d * sizeof(double));
    gemm(true, true, d, d, s, 1.0, X, s, X, s, 0.0, gram.as<double>(), d, st);
    const double *R = gram.as<double>();
    int64_t ldr = d;
    DevBuf Rinv((size_t)d * (size_t)d * sizeof(double));
    // P (row-major d x d) = R^-1: invert column-major, then transpose
    auto invert = [&] {
        trtri_upper(d, R, ldr, Rinv.as<double>(), d, st);
        transpose(d, d, Rinv.as<double>(), d, P, st);
        LSRN_HIP(hipStreamSynchronize(st));
    };
    bool ok = cholesky_upper(d, gram.as<double>(), d, st);
    if (ok) {
        sorted_diag(R, ldr);
        const double ratio = h[0] / h[(size_t)d - 1];
        ok = h[(size_t)d - 1] > 0.0 && ratio * ratio * (double)d * DBL_EPSILON <= 1e-5;
    }
    if (ok) {
        invert();
        DevBuf part((size_t)2 * d * sizeof(double));
        col_sumsq_kernel<<<(unsigned)d, 256, 0, st>>>(R, ldr, Rinv.as<double>(), d, part.as<double>());
        LSRN_HIP(hipGetLastError());
        std::vector<double> cs((size_t)d);
        LSRN_HIP(hipMemcpyAsync(cs.data(), part.as<double>(), (size_t)d * sizeof(double), hipMemcpyDeviceToHost, st));
        LSRN_HIP(hipStreamSynchronize(st));
        double cmax = 0.0;
        for (int64_t j = 0; j < d; ++j) cmax = std::max(cmax, cs[(size_t)j]);
        const double k2 = cmax * inv_norm2_sq(d, P, Rinv.as<double>(), st);  // kappa^2 estimate
        ok = std::isfinite(k2) && k2 * (double)d * DBL_EPSILON <= 1e-5;
    }
    if (!ok) {
        gram.release();
        householder_qr(s, d, X, st);
        R = X;
        ldr = s;
        sorted_diag(R, ldr);
    }
    if (!(h[(size_t)d - 1] > rc * h[0]))
        fail(LSRN_E_UNSUPPORTED, "precond: the QR-inverse preconditioner needs a full-rank sketch");
    LSRN_HIP(hipMemcpyAsync(sigma, h.data(), (size_t)d * sizeof(double), hipMemcpyHostToDevice, st));
    if (!ok) invert();
    res.rank = d;
    res.sigma_max = h[0];
    res.sigma_min_kept = h[(size_t)d - 1];
    res.full_rank_inverse = true;
    return res;
}

}  // namespace lsrn
