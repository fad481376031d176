// internal.hpp -- host-side interfaces between the translation units of liblsrn.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "common.hpp"

namespace lsrn {

// ------------------------------------------------------------ rng.hip
void launch_philox_words(uint64_t seed, int64_t row0, int64_t nrows, int64_t q0, int64_t nq,
                         uint32_t *out, hipStream_t s);
void launch_gauss_fill(uint64_t seed, int64_t row0, int64_t nrows, int64_t col0, int64_t ncols,
                       double *out, hipStream_t s);

// ---------------------------------------------------------- sketch.hip
// X (s x d, column-major, ld = s) = G T, T row-major K x d with leading
// dimension ldt (T = A for tall row-major A, T = A^T for fat column-major
// A).  When lambda > 0, adds lambda * G(i, K + c) to X(i, c) (the rows
// lambda I of the augmented tall matrix, Sec. 5).
// With kernel_ms != NULL the GEMM kernel is timed with HIP events on st.
void sketch_rows(int64_t K, int64_t d, const double *T, int64_t ldt, double lambda, int64_t s,
                 uint64_t seed, double *X, hipStream_t st, double *kernel_ms = nullptr);
// The same for T stored in FP32 (each entry exact in FP64).
void sketch_rows(int64_t K, int64_t d, const float *T, int64_t ldt, double lambda, int64_t s,
                 uint64_t seed, double *X, hipStream_t st, double *kernel_ms = nullptr);
size_t sketch_workspace_bytes(int64_t K, int64_t d, int64_t s);
// Bytes of split-K partial sums sketch_rows takes for FP64 T (0: none).
size_t sketch_slices_bytes(int64_t K, int64_t d, int64_t s);
// sketch_rows for FP64 T with the partial sums in the library's static
// scratch (LSRN_NOALLOC_SCRATCH_BYTES): allocates nothing and does not
// synchronise; LSRN_E_NOMEM when the partial sums would not fit.
void sketch_rows_noalloc(int64_t K, int64_t d, const double *T, int64_t ldt, double lambda,
                         int64_t s, uint64_t seed, double *X, hipStream_t st);
// The sketches of `count` tall problems (T[p] row-major K[p] x d[p], G[p]
// from key seeds[p]) in one launch per alignment class, no split of K.
// Synchronises.
void sketch_rows_batch(int count, const int64_t *K, const int64_t *d, const double *const *T,
                       const int64_t *ldt, const int64_t *s, const uint64_t *seeds, double *const *X,
                       hipStream_t st);

// The precision form's sketch: X = bf16(G) fl32(T) on the BF16 matrix
// cores (FP32 accumulation flushed to FP64), plus the FP64 rows lambda G of
// the Tikhonov block.  Synchronises.
// device bytes of the precision-form sketch's pre-generated bf16(G) and split
// terms of T (0: generated and split in the kernel)
size_t sketch_bf16_g_bytes(int64_t K, int64_t d, int64_t s);
void sketch_rows_bf16(int64_t K, int64_t d, const double *T, int64_t ldt, double lambda, int64_t s,
                      uint64_t seed, double *X, hipStream_t st, double *kernel_ms = nullptr);
// T32 (rows x cols, leading dimension ldt) = T rounded to FP32.
void to_f32(int64_t rows, int64_t cols, const double *T, int64_t ldt, float *T32, hipStream_t st);

// X(i, c) += lambda G(i, K + c): the rows lambda I of the augmented tall
// matrix (Sec. 5).
void add_identity_rows(int64_t K, int64_t d, int64_t s, double lambda, uint64_t seed, double *X,
                       hipStream_t st);

// Out-of-place transpose: out (cols x rows, leading dim rows) = in^T, in
// row-major rows x cols with leading dim ldin.
void transpose(int64_t rows, int64_t cols, const double *in, int64_t ldin, double *out,
               hipStream_t st);
void transpose(int64_t rows, int64_t cols, const float *in, int64_t ldin, float *out,
               hipStream_t st);

// ------------------------------------------------------------- csr.hip
// Row-compressed structure of a sparse matrix (device arrays).
struct CsrMat {
    int64_t nrows = 0, ncols = 0, nnz = 0;
    const int64_t *ptr = nullptr;  // nrows + 1 offsets
    const int32_t *idx = nullptr;  // column index of each entry
    const double *val = nullptr;
};

// The tall view T (K x d) of a CSR matrix A (m x n): T = A when m >= n,
// T = A^T otherwise, held row-compressed (rows = CSR of T) and column-
// compressed (cols = CSR of T^T).  One of the two is the caller's A; the
// other is the transposed copy the library builds (stable, so entries of a
// column keep the row order and every sum runs in a fixed order).
struct SparseView {
    bool tall = true;
    int64_t K = 0, d = 0, nnz = 0;
    CsrMat rows, cols;
    DevBuf tptr, tidx, tval;
    // the rows of `cols` cut into segments of at most kColSeg entries, so a
    // few long columns of T do not serialise the column pass: segment g
    // belongs to row seg_row[g] of `cols`, whose segments start at
    // row_seg[row] (d + 1 offsets)
    static constexpr int64_t kColSeg = 512;
    int64_t nseg = 0;
    DevBuf seg_row, row_seg;
};
// Validates the structure (LSRN_E_INVALID on bad offsets or indices) and
// builds the transposed copy.  Synchronises.
void make_sparse_view(SparseView &v, int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                      const int32_t *colind, const double *val, hipStream_t st);
size_t sparse_view_bytes(int64_t m, int64_t n, int64_t nnz);
// X (s x d, column-major) = G T (+ lambda G(:, K + c) when tall and
// lambda > 0).  Synchronises.
// device bytes the sparse sketch allocates besides its nnz-sized arrays
size_t sketch_csr_tile_bytes(int64_t K, int64_t d, int64_t nnz, int64_t s);
void sketch_csr(const SparseView &v, double lambda, int64_t s, uint64_t seed, double *X,
                hipStream_t st, double *kernel_ms = nullptr);

// ------------------------------------------------------------- svd.hip
struct PrecondResult {
    int64_t rank = 0;
    int64_t sweeps = 0;
    double sigma_max = 0.0;
    double sigma_min_kept = 0.0;
    double t_jacobi_kernel_ms = 0.0;  // with profile: summed per-sweep spans
    int64_t jacobi_kernels = 0;
    bool full_rank_inverse = false;   // P = R^-1 (certified full rank), no sweeps
};
// X: s x d column-major (overwritten).  P: d x d row-major (first r columns
// hold V_r Sigma_r^{-1}); sigma: d values, descending.  With try_full_rank,
// a sketch whose R is certified to keep every singular value under the
// cutoff gets P = R^-1 instead (no Jacobi sweeps; sigma = |diag R|
// descending).  Synchronises.
PrecondResult precond(int64_t s, int64_t d, double *X, double rcond, double *sigma, double *P,
                      hipStream_t st, bool profile = false, bool try_full_rank = false);
// precond for `count` sketches at once: the QR of each; for the problems
// with try_fr[p] (d <= 512; try_fr may be NULL) the certified P = R^-1 of
// all of them in one launch; then the Jacobi sweeps of the rest with
// d <= 512 in shared launches (wider ones one at a time).  X[p] is
// overwritten.
void precond_batch(int count, const int64_t *s, const int64_t *d, double *const *X, double rcond,
                   double *const *sigma, double *const *P, PrecondResult *res, hipStream_t st,
                   const char *try_fr = nullptr);
size_t precond_workspace_bytes(int64_t s, int64_t d);
// Householder QR of X (s x d, column-major, in place; R in the upper
// triangle).  Synchronises.
void householder_qr(int64_t s, int64_t d, double *X, hipStream_t st);
// Full-rank alternative to steps 4-5: QR of the sketch and P = R^-1
// (row-major d x d); sigma receives |diag R| in descending order.
// LSRN_E_UNSUPPORTED when min |r_ii| <= rcond max |r_ii|.  Synchronises.
PrecondResult precond_qr_inverse(int64_t s, int64_t d, double *X, double rcond, double *sigma,
                                 double *P, hipStream_t st);

// ---------------------------------------------------------- linalg.hip
// C = alpha op(A) B + beta C, column-major (FP64 MFMA); op(A) = A^T when
// ta (A then K x M); upper: only tiles touching the upper triangle.
void gemm(bool ta, bool upper, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
          int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
          hipStream_t st);
// In-place Cholesky C = R^T R of the upper triangle of C (d x d, column-
// major, ldc), R written over the upper triangle; false on a pivot <= 0.
// Synchronises.
bool cholesky_upper(int64_t d, double *C, int64_t ldc, hipStream_t st);
// C = alpha A B + beta C, all column-major (FP64 MFMA).
void gemm_nn(int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t lda,
             const double *B, int64_t ldb, double beta, double *C, int64_t ldc, hipStream_t st);
// Rinv (column-major, ldi) = R^-1 for upper-triangular R (column-major, ldr;
// entries below the diagonal are ignored).
void trtri_upper(int64_t d, const double *R, int64_t ldr, double *Rinv, int64_t ldi, hipStream_t st);
// Elements of the temporary product buffer trtri_upper allocates for order d.
int64_t trtri_work_elems(int64_t d);

// --------------------------------------------------------- iterate.hip
// The operator of the iteration phase.  Tall: T = A row-major (rows = m,
// cols = n) with optional lambda rows; Fat: T = A^T row-major (rows = n,
// cols = m).  P is d x r row-major (leading dim ldp), d = cols of T.
// ------------------------------------------------------------ tune.hip
enum TunePhase { TUNE_SWEEP = 0 };
struct TuneKey {
    int phase = TUNE_SWEEP;
    int dtype = 0;      // 0: FP64 sweeps, 1: FP32 (precision form)
    int rows_log2 = 0;  // ceil(log2(rows of the tall view))
    int64_t cols = 0;
};
int rows_bucket(int64_t rows);
bool tune_lookup(const TuneKey &k, int &value);
void tune_store(const TuneKey &k, int value);

// A matrix given only through the caller's product routine: out = op(A) in
// for k columns (trans = 0: A, trans = 1: A^T), m x n.
struct OpView {
    lsrn_apply_fn fn = nullptr;
    void *ctx = nullptr;
    int64_t m = 0, n = 0;
    // out (rows of the result) = T in (t = 0) or T^T in (t = 1) for the
    // tall view T: A when m >= n, A^T otherwise.  Throws on a nonzero
    // return of the routine.
    void apply_t(int t, int64_t k, const double *in, int64_t ldin, double *out, int64_t ldout,
                 hipStream_t st) const;
};

struct IterProblem {
    bool tall = true;
    int64_t rows = 0;       // rows of T
    int64_t cols = 0;       // cols of T (= d)
    const double *T = nullptr;
    int64_t ldt = 0;
    double lambda = 0.0;    // tall only
    const double *P = nullptr;
    int64_t ldp = 0;
    int64_t r = 0;
    int64_t s = 0;
    const SparseView *sp = nullptr;  // sparse T (then T and ldt are unused)
    const OpView *op = nullptr;      // T through the caller's products (no refinement)
    // precision form: FP32 copy of T (leading dimension ldt) read by every
    // sweep; refinement residuals still use the FP64 T
    const float *T32 = nullptr;
    // sigma_max / sigma_min_kept of the sketch (0: unknown); the precision
    // form reads the FP64 T from the start when this times 2^-24 exceeds 1/2
    double kappa_sketch = 0.0;
};

struct IterResult {
    int64_t iters = 0;
    int64_t refine_steps = 0;
    int64_t refine_iters = 0;
    int64_t fp64_refine_steps = 0;  // precision form: steps whose sweeps read the FP64 A
    int64_t cs_fallbacks = 0;       // Chebyshev runs whose post-check failed (LSQR restarts)
    bool converged = true;
    double sigma_l = 0.0, sigma_u = 0.0;
    double t_iter_ms = 0.0, t_refine_ms = 0.0;
    double t_sweep_kernel_ms = 0.0;  // opt.profile: summed sweep kernel time
    int64_t sweep_kernels = 0;
};

// Runs step 6 (and 7) for b (length m of the original problem) and
// writes x (length n).  Synchronises.
IterResult iterate(const IterProblem &pb, const double *b, double *x, const lsrn_options &opt,
                   hipStream_t st);

// LSQR for many tall dense FP64 problems (cols <= 512, no lambda) at once,
// then opts[p].refine refinement steps of each: each kernel launch covers
// the whole batch.  opts[p] gives problem p's tol, max_iter, refine and
// refine_tol.  Synchronises.
std::vector<IterResult> iterate_batch_tall(const std::vector<IterProblem> &pbs,
                                           const std::vector<const double *> &bs,
                                           const std::vector<double *> &xs,
                                           const std::vector<lsrn_options> &opts, hipStream_t st);

}  // namespace lsrn
