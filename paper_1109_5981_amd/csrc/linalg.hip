// linalg.hip -- dense FP64 building blocks on the matrix cores: a general
// column-major GEMM and the inverse of an upper-triangular matrix (used for
// the preconditioner N = R^-1 of a full-rank sketch).
#include <algorithm>

#include "internal.hpp"

namespace lsrn {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int GBM = 128, GBN = 128, GKT = 16, GLDP = 144, GNT = 256;

__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A (M x K, column-major, lda): stage kk rows of k, 128 consecutive i.
__device__ __forceinline__ void load_a(const double *__restrict__ A, int64_t lda, int64_t M,
                                       int64_t K, int64_t m0, int64_t k0, double (&reg)[8]) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int idx = it * GNT + threadIdx.x;  // 0 .. 2047
        const int kk = idx >> 7, i = idx & 127;
        const int64_t k = k0 + kk, row = m0 + i;
        reg[it] = (k < K && row < M) ? A[k * lda + row] : 0.0;
    }
}

__device__ __forceinline__ void store_a(double (*As)[GLDP], const double (&reg)[8]) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int idx = it * GNT + threadIdx.x;
        As[idx >> 7][idx & 127] = reg[it];
    }
}

// A^T where A is K x M column-major (lda): 16 consecutive k of row i of
// op(A) per 16 lanes.
__device__ __forceinline__ void load_at(const double *__restrict__ A, int64_t lda, int64_t M,
                                        int64_t K, int64_t m0, int64_t k0, double (&reg)[8]) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int idx = it * GNT + threadIdx.x;
        const int kk = idx & 15, i = idx >> 4;
        const int64_t k = k0 + kk, row = m0 + i;
        reg[it] = (k < K && row < M) ? A[row * lda + k] : 0.0;
    }
}

__device__ __forceinline__ void store_at(double (*As)[GLDP], const double (&reg)[8]) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int idx = it * GNT + threadIdx.x;
        As[idx & 15][idx >> 4] = reg[it];
    }
}

// B (K x N, column-major, ldb): 16 consecutive k of column j per 16 lanes.
__device__ __forceinline__ void load_b(const double *__restrict__ B, int64_t ldb, int64_t K,
                                       int64_t N, int64_t k0, int64_t n0, double (&reg)[8]) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int idx = it * GNT + threadIdx.x;
        const int kk = idx & 15, j = idx >> 4;  // j 0 .. 127
        const int64_t k = k0 + kk, col = n0 + j;
        reg[it] = (k < K && col < N) ? B[col * ldb + k] : 0.0;
    }
}

__device__ __forceinline__ void store_b(double (*Bs)[GLDP], const double (&reg)[8]) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int idx = it * GNT + threadIdx.x;
        Bs[idx & 15][idx >> 4] = reg[it];
    }
}

// C = alpha op(A) B + beta C, op(A) = A (TA false) or A^T (TA true); each
// workgroup one 128 x 128 tile of C (2 x 2 wavefronts of 64 x 64, 4 x 4
// blocks of v_mfma_f64_16x16x4f64).  UPPER: tiles entirely below the
// diagonal are skipped (the lower triangle of C is left unspecified).
template <bool TA, bool UPPER>
__global__ void __launch_bounds__(GNT, 2)
gemm_kernel(int64_t M, int64_t N, int64_t K, double alpha, const double *__restrict__ A,
            int64_t lda, const double *__restrict__ B, int64_t ldb, double beta,
            double *__restrict__ C, int64_t ldc, int tiles_m) {
    __shared__ double As[2][GKT][GLDP];
    __shared__ double Bs[2][GKT][GLDP];
    const int64_t m0 = (int64_t)(blockIdx.x % tiles_m) * GBM;
    const int64_t n0 = (int64_t)(blockIdx.x / tiles_m) * GBN;
    if (UPPER && m0 >= n0 + GBN) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1, lr = lane & 15, lk = lane >> 4;
    f64x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int64_t nstage = ceil_div(K, GKT);
    double ra[8], rb[8];
    if (nstage > 0) {
        if (TA) load_at(A, lda, M, K, m0, 0, ra);
        else load_a(A, lda, M, K, m0, 0, ra);
        load_b(B, ldb, K, N, 0, n0, rb);
        if (TA) store_at(As[0], ra);
        else store_a(As[0], ra);
        store_b(Bs[0], rb);
    }
    __syncthreads();
    for (int64_t st = 0; st < nstage; ++st) {
        const int buf = (int)(st & 1);
        const bool more = st + 1 < nstage;
        if (more) {
            if (TA) load_at(A, lda, M, K, m0, (st + 1) * GKT, ra);
            else load_a(A, lda, M, K, m0, (st + 1) * GKT, ra);
            load_b(B, ldb, K, N, (st + 1) * GKT, n0, rb);
        }
#pragma unroll
        for (int kk = 0; kk < GKT / 4; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[buf][kk * 4 + lk][wm * 64 + i * 16 + lr];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[buf][kk * 4 + lk][wn * 64 + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
        }
        if (more) {
            if (TA) store_at(As[buf ^ 1], ra);
            else store_a(As[buf ^ 1], ra);
            store_b(Bs[buf ^ 1], rb);
        }
        __syncthreads();
    }
    // accumulator element v of lane (lr, lk) is row lk + 4 v, column lr of
    // its 16 x 16 block
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t col = n0 + wn * 64 + j * 16 + lr;
            const int64_t rbase = m0 + wm * 64 + i * 16 + lk;
            if (col < N) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = rbase + 4 * v;
                    if (row < M) {
                        double *c = C + col * ldc + row;
                        *c = beta == 0.0 ? alpha * acc[i][j][v] : alpha * acc[i][j][v] + beta * *c;
                    }
                }
            }
        }
}

constexpr int TB = 64;  // diagonal block of the triangular inverse

// Inverse of each 64 x 64 diagonal block of upper-triangular R (column-
// major, ldr) into Rinv (column-major, ldi): thread j back-substitutes
// column j of the block's inverse.
__global__ void __launch_bounds__(TB)
trtri_diag_kernel(int64_t d, const double *__restrict__ R, int64_t ldr, double *__restrict__ Rinv,
                  int64_t ldi) {
    __shared__ double Rs[TB][TB + 1];  // Rs[i][k] = R(o + i, o + k)
    __shared__ double Xs[TB][TB + 1];  // Xs[i][j] = inverse (i, j)
    const int64_t o = (int64_t)blockIdx.x * TB;
    const int nb = (int)min<int64_t>(TB, d - o);
    const int j = threadIdx.x;
    for (int k = 0; k < nb; ++k)
        if (j < nb) Rs[j][k] = R[(o + k) * ldr + o + j];
    __syncthreads();
    if (j < nb) {
        for (int i = nb - 1; i >= 0; --i) {
            double v;
            if (i > j) {
                v = 0.0;
            } else {
                double t = i == j ? 1.0 : 0.0;
                for (int k = i + 1; k <= j; ++k) t -= Rs[i][k] * Xs[k][j];
                v = t / Rs[i][i];
            }
            Xs[i][j] = v;
        }
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k)
        if (j < nb) Rinv[(o + k) * ldi + o + j] = Xs[j][k];
}

// Cholesky of the jb x jb diagonal block at (j0, j0) of C (upper triangle,
// column-major, ldc): C = R^T R with R upper triangular written over C's
// upper triangle, and Dinv (ld TB) = R^-1.  A pivot <= 0 (or NaN) sets *bad.
__global__ void __launch_bounds__(TB)
chol_diag_kernel(double *__restrict__ C, int64_t ldc, int64_t j0, int jb,
                 double *__restrict__ Dinv, int *__restrict__ bad) {
    __shared__ double A[TB][TB + 1];   // A[i][k] = C(j0 + i, j0 + k), i <= k
    __shared__ double Xs[TB][TB + 1];
    __shared__ int flag;
    const int k = threadIdx.x;
    if (k == 0) flag = 0;
    for (int i = 0; i < jb; ++i)
        if (k < jb) A[i][k] = i <= k ? C[(j0 + k) * ldc + j0 + i] : 0.0;
    __syncthreads();
    for (int p = 0; p < jb; ++p) {
        if (k == 0) {
            double piv = A[p][p];
            if (!(piv > 0.0)) {
                flag = 1;
                piv = 1.0;
            }
            A[p][p] = sqrt(piv);
        }
        __syncthreads();
        if (k > p && k < jb) A[p][k] /= A[p][p];
        __syncthreads();
        if (k > p && k < jb)
            for (int i = p + 1; i <= k; ++i) A[i][k] -= A[p][i] * A[p][k];
        __syncthreads();
    }
    // inverse of the block: thread j back-substitutes column j
    if (k < jb) {
        for (int i = jb - 1; i >= 0; --i) {
            double v = 0.0;
            if (i <= k) {
                double t = i == k ? 1.0 : 0.0;
                for (int q = i + 1; q <= k; ++q) t -= A[i][q] * Xs[q][k];
                v = t / A[i][i];
            }
            Xs[i][k] = v;
        }
    }
    __syncthreads();
    for (int i = 0; i < jb; ++i) {
        if (k < jb) {
            if (i <= k) C[(j0 + k) * ldc + j0 + i] = A[i][k];
            Dinv[k * TB + i] = Xs[i][k];
        }
    }
    if (k == 0 && flag) atomicOr(bad, 1);
}

// dst (rows x cols, ld ldd) = src (ld lds), column-major.
__global__ void __launch_bounds__(256)
copy_block_kernel(int64_t rows, int64_t cols, const double *__restrict__ src, int64_t lds,
                  double *__restrict__ dst, int64_t ldd) {
    const int64_t total = rows * cols;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = t / rows, r = t % rows;
        dst[c * ldd + r] = src[c * lds + r];
    }
}

}  // namespace

void gemm(bool ta, bool upper, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
          int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
          hipStream_t st) {
    if (M <= 0 || N <= 0) return;
    const int64_t tm = ceil_div(M, GBM), tn = ceil_div(N, GBN);
    LSRN_REQUIRE(tm * tn < ((int64_t)1 << 31), "gemm: too many tiles");
    const dim3 grid((unsigned)(tm * tn));
    if (ta && upper)
        gemm_kernel<true, true><<<grid, GNT, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, (int)tm);
    else if (ta)
        gemm_kernel<true, false><<<grid, GNT, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, (int)tm);
    else if (upper)
        gemm_kernel<false, true><<<grid, GNT, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, (int)tm);
    else
        gemm_kernel<false, false><<<grid, GNT, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, (int)tm);
    LSRN_HIP(hipGetLastError());
}

void gemm_nn(int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t lda,
             const double *B, int64_t ldb, double beta, double *C, int64_t ldc, hipStream_t st) {
    gemm(false, false, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, st);
}

namespace {

// Split of a diagonal block of n > TB rows: n1 (a multiple of TB, about
// n / 2) and n - n1.
int64_t trtri_split(int64_t n) { return TB * ceil_div(ceil_div(n, 2), TB); }

// Elements of the product buffer W that the halving tree of a block of n
// rows needs: the largest n1 (n - n1) over all its levels.  (A sub-block can
// need more than the top split: n = 130 splits 128 + 2, and the 128 block
// then 64 + 64.)
int64_t trtri_work(int64_t n) {
    if (n <= TB) return 0;
    const int64_t n1 = trtri_split(n), n2 = n - n1;
    return std::max(n1 * n2, std::max(trtri_work(n1), trtri_work(n2)));
}

// Off-diagonal blocks of the inverse, bottom-up over the halving tree: for
// the diagonal block [off, off + n) split as [A B; 0 C] with both diagonal
// inverses already in Rinv, Rinv(top-right) = -A^-1 B C^-1.  W holds wcap
// elements.
void trtri_rec(int64_t off, int64_t n, const double *R, int64_t ldr, double *Rinv, int64_t ldi,
               double *W, int64_t wcap, hipStream_t st) {
    if (n <= TB) return;
    const int64_t n1 = trtri_split(n), n2 = n - n1;
    LSRN_REQUIRE(n1 * n2 <= wcap, "trtri: product buffer too small");
    trtri_rec(off, n1, R, ldr, Rinv, ldi, W, wcap, st);
    trtri_rec(off + n1, n2, R, ldr, Rinv, ldi, W, wcap, st);
    // W (n1 x n2, ld n1) = A^-1 B
    gemm_nn(n1, n2, n1, 1.0, Rinv + off * ldi + off, ldi, R + (off + n1) * ldr + off, ldr, 0.0, W, n1,
            st);
    // top-right = -W C^-1
    gemm_nn(n1, n2, n2, -1.0, W, n1, Rinv + (off + n1) * ldi + off + n1, ldi, 0.0,
            Rinv + (off + n1) * ldi + off, ldi, st);
}

}  // namespace

int64_t trtri_work_elems(int64_t d) { return trtri_work(d); }

void trtri_upper(int64_t d, const double *R, int64_t ldr, double *Rinv, int64_t ldi, hipStream_t st) {
    LSRN_HIP(hipMemsetAsync(Rinv, 0, (size_t)ldi * (size_t)d * sizeof(double), st));
    trtri_diag_kernel<<<(unsigned)ceil_div(d, TB), TB, 0, st>>>(d, R, ldr, Rinv, ldi);
    LSRN_HIP(hipGetLastError());
    if (d > TB) {
        const int64_t wn = trtri_work(d);
        DevBuf W((size_t)wn * sizeof(double));
        trtri_rec(0, d, R, ldr, Rinv, ldi, W.as<double>(), wn, st);
        LSRN_HIP(hipStreamSynchronize(st));  // before W is freed
    }
}

bool cholesky_upper(int64_t d, double *C, int64_t ldc, hipStream_t st) {
    DevBuf Dinv((size_t)TB * TB * sizeof(double)), flag(sizeof(int));
    const int64_t wmax = std::max<int64_t>(0, d - TB);
    DevBuf W((size_t)TB * (size_t)std::max<int64_t>(wmax, 1) * sizeof(double));
    LSRN_HIP(hipMemsetAsync(flag.as<int>(), 0, sizeof(int), st));
    for (int64_t j0 = 0; j0 < d; j0 += TB) {
        const int jb = (int)std::min<int64_t>(TB, d - j0);
        chol_diag_kernel<<<1, TB, 0, st>>>(C, ldc, j0, jb, Dinv.as<double>(), flag.as<int>());
        LSRN_HIP(hipGetLastError());
        const int64_t nr = d - j0 - jb;
        if (nr <= 0) break;
        double *Crow = C + (j0 + jb) * ldc + j0;  // C(j0 : j0 + jb, j0 + jb : d)
        // W = R_jj^-T C(j, rest): the block row of R
        gemm(true, false, jb, nr, jb, 1.0, Dinv.as<double>(), TB, Crow, ldc, 0.0, W.as<double>(), jb, st);
        // trailing update of the upper triangle: C(rest, rest) -= W^T W
        double *Ct = C + (j0 + jb) * ldc + j0 + jb;
        gemm(true, true, nr, nr, jb, -1.0, W.as<double>(), jb, W.as<double>(), jb, 1.0, Ct, ldc, st);
        copy_block_kernel<<<(unsigned)std::min<int64_t>(ceil_div(jb * nr, 256), 8192), 256, 0, st>>>(
            jb, nr, W.as<double>(), jb, Crow, ldc);
        LSRN_HIP(hipGetLastError());
    }
    int bad = 0;
    LSRN_HIP(hipMemcpyAsync(&bad, flag.as<int>(), sizeof(int), hipMemcpyDeviceToHost, st));
    LSRN_HIP(hipStreamSynchronize(st));  // before the buffers are freed
    return bad == 0;
}

}  // namespace lsrn
