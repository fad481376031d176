/*
 * lsrn.h -- C ABI of the MI355X (gfx950) LSRN library, liblsrn.so.
 *
 * LSRN (Meng, Saunders, Mahoney, arXiv:1109.5981) computes the min-length
 * least-squares solution x = A^+ b of a strongly over- or under-determined,
 * possibly rank-deficient A (Sec. 1, eq. for x*), optionally with Tikhonov
 * regularisation W = lambda I (Sec. 5):
 *   1. s = ceil(gamma * min(m, n))                         (Alg. 1/2 step 1)
 *   2. G: s x m (tall) or n x s (fat) standard normal, generated on the fly
 *      from Philox4x32-10 counters and never stored       (step 2)
 *   3. sketch A~ = G A (tall) or A G (fat)                (step 3)
 *   4. economy SVD of A~, rank r                           (step 4)
 *   5. N = V~ Sigma~^{-1} (tall) or M = U~ Sigma~^{-1} (fat)  (step 5)
 *   6. LSQR or the Chebyshev semi-iteration (Alg. 3) on A N or M^T A
 *   7. x = N y (tall) or x (fat)                          (step 7)
 *
 * Conventions for every entry point below:
 *   - All array arguments are DEVICE pointers (hipMalloc'd or equivalent) on
 *     the current HIP device, owned by the caller.  The library never frees
 *     or keeps caller memory beyond the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is ordered on that stream.  Calls that return sizes or ranks to
 *     the host synchronise the stream before returning.
 *   - Workspace is allocated by the library with hipMalloc and freed before
 *     the call returns.
 *   - No exception crosses the ABI.  On failure the return code says what
 *     went wrong and lsrn_last_error() (per thread) holds a message.
 *   - Dense A is FP64 with leading dimension lda >= (columns of the stored
 *     layout).  LSRN_ROW_MAJOR: A[i][j] = A[i*lda + j];
 *     LSRN_COL_MAJOR: A[i][j] = A[j*lda + i].  Tall problems (m >= n) run
 *     from row-major storage and fat ones (m < n) from column-major storage
 *     without copying A; the other two combinations are transposed once
 *     into workspace.
 */
#ifndef LSRN_H
#define LSRN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LSRN_OK = 0,
    LSRN_E_INVALID = 1,       /* bad size, pointer or option                */
    LSRN_E_NOMEM = 2,         /* device allocation failed                   */
    LSRN_E_HIP = 3,           /* a HIP runtime call failed                  */
    LSRN_E_NOT_CONVERGED = 4, /* LSQR hit max_iter; x holds the last iterate */
    LSRN_E_UNSUPPORTED = 5    /* e.g. Chebyshev with the precision form     */
} lsrn_status;

typedef enum { LSRN_LSQR = 0, LSRN_CHEBYSHEV = 1 } lsrn_method;
typedef enum { LSRN_ROW_MAJOR = 0, LSRN_COL_MAJOR = 1 } lsrn_layout;

/* How steps 4-5 form the preconditioner.
 *   LSRN_PRECOND_SVD: QR + one-sided Jacobi SVD of the sketch, rank cutoff,
 *     N = V_r Sigma_r^-1 (Alg. 1/2 steps 4-5); min(m, n) <= 8192.
 *   LSRN_PRECOND_QR: N = R^-1 from the QR of the sketch.  G A R^-1 = Q has
 *     orthonormal columns, the property the condition-number bound of
 *     Sec. 4.2 rests on, but no rank is revealed: needs a full-rank sketch
 *     (guaranteed when lambda > 0) and returns LSRN_E_UNSUPPORTED otherwise.
 *   LSRN_PRECOND_AUTO: for min(m, n) <= 8192 the SVD, except that the QR
 *     of the sketch is first tested: when |R|_F |R^-1|_F <= 1 / (2 rcond)
 *     (so every singular value lies above the SVD's cutoff) N = R^-1 is
 *     used and the Jacobi sweeps are skipped (same preconditioned
 *     spectrum, same solution; lsrn_info.precond_used reports the choice).
 *     Above 8192: QR when lambda > 0, else LSRN_E_UNSUPPORTED.
 *     lsrn_solve_batch always takes the SVD. */
typedef enum { LSRN_PRECOND_AUTO = 0, LSRN_PRECOND_SVD = 1, LSRN_PRECOND_QR = 2 } lsrn_precond_kind;

/* Arithmetic of the solve (dense A only).
 *   LSRN_PREC_FP64: everything in FP64 (refinement residuals in
 *     double-double).
 *   LSRN_PREC_MIXED: the precision form.  The sketch is bf16(G) fl32(A) on
 *     the BF16 matrix cores (A rounded to FP32 and split exactly into three
 *     BF16 terms, FP32 accumulation flushed to FP64); the library keeps an
 *     FP32 copy of A (4 m n bytes) that every LSQR sweep reads, accumulating
 *     in FP64; the SVD / cutoff / N, the scalar recurrences and the
 *     refinement residuals (double-double, with the FP64 A) stay FP64.  The
 *     main LSQR stops at max(tol, 1e-8) and refinement steps (opt->refine, 10
 *     when 0) bring x to the FP64 solution while kappa(A) * 2^-24 << 1.
 *     When the sketch's sigma_max / sigma_min_kept times 2^-24 exceeds 1/2
 *     (FP32 sweeps could not contract) the sweeps read the FP64 A from the
 *     start and only the sketch is BF16 (info->fp64_refine_steps then counts
 *     every refinement step).
 *     The Chebyshev bounds of Sec. 4.2 hold for the exact sketch only, so
 *     LSRN_CHEBYSHEV is rejected (LSRN_E_UNSUPPORTED), and so are
 *     under-determined A: the FP32 sweeps would leave a component of size
 *     about kappa(A) 2^-24 outside range(A^T) that residual refinement does
 *     not remove.  Refinement stops when a correction is below 1e-15 ||x||
 *     or no longer half the previous one; the solve counts as converged
 *     (info->converged, else LSRN_E_NOT_CONVERGED with x the last iterate)
 *     when the last correction is below max(tol, 1e-12) ||x||. */
typedef enum { LSRN_PREC_FP64 = 0, LSRN_PREC_MIXED = 1 } lsrn_precision;

typedef struct lsrn_options {
    double gamma;      /* oversampling factor gamma > 1 (Alg. 1 step 1); 2     */
    double lambda;     /* Tikhonov weight, W = lambda I (Sec. 5); 0            */
    double tol;        /* LSQR atol = btol, or the epsilon of Alg. 3; 1e-14    */
    double rcond;      /* rank cutoff relative to sigma_1; <= 0 selects
                          max(s, d) * 2^-52 (d = min(m, n))                     */
    double t_margin;   /* margin t of Lemma 3 in the Chebyshev bounds
                          sigma_U = 1/(sqrt s - sqrt r - t),
                          sigma_L = 1/(sqrt s + sqrt r + t) (Theorem 3); 1.
                          A negative t narrows the interval (it then misses
                          part of the spectrum: a way to exercise the check
                          after a Chebyshev run)                              */
    double refine_tol; /* relative accuracy asked of each refinement
                          correction; 1e-6                                      */
    uint64_t seed;     /* Philox key of G; 0                                   */
    int64_t max_iter;  /* LSQR iteration cap; <= 0 selects the Alg. 3 count
                          for the same bounds plus 10                           */
    int32_t method;    /* lsrn_method; LSRN_LSQR                               */
    int32_t refine;    /* number of refinement steps whose residuals are
                          formed in double-double arithmetic; 0                 */
    int32_t profile;   /* nonzero: time every sketch and sweep kernel launch
                          with HIP events on `stream` (lsrn_info fields
                          t_*_kernel_ms); 0                                     */
    int32_t precond;   /* lsrn_precond_kind; LSRN_PRECOND_AUTO                 */
    int32_t precision; /* lsrn_precision; LSRN_PREC_FP64                       */
    int32_t autotune;  /* nonzero: the first solve of a new shape key times
                          the candidate launch shapes of the dense sweep and
                          records the fastest (see lsrn_tune_export); zero:
                          recorded shapes if any, else the built-in ones; 0 */
    int32_t keep_sketch; /* plans: keep the sketch G T of A (s d doubles) so
                          that lsrn_plan_set_lambda re-forms the
                          preconditioner for another lambda without a new
                          sketch; 0                                         */
} lsrn_options;

typedef struct lsrn_info {
    int64_t s;              /* sketch size ceil(gamma d)                         */
    int64_t d;              /* min(m, n) of the (augmented) problem              */
    int64_t rank;           /* r, numerical rank of the sketch                   */
    int64_t iters;          /* LSQR / Chebyshev iterations of the main solve     */
    int64_t refine_steps;   /* refinement steps taken                            */
    int64_t refine_iters;   /* inner iterations summed over refinement steps     */
    int64_t sweeps;         /* Jacobi sweeps of the sketch SVD                   */
    int32_t tall;           /* 1: Alg. 1 (m >= n), 0: Alg. 2                     */
    int32_t converged;      /* LSQR: stopping rule met; Chebyshev: the check
                               after the run passed, or the LSQR restart it
                               triggered met its stopping rule; with
                               refinement (FP64): the last correction's
                               inner solve met its rule                     */
    double sigma_l, sigma_u;/* Chebyshev bounds used (0 when r is too large)     */
    double sigma_max;       /* largest singular value of the sketch (N = R^-1:
                               an estimate, the largest column norm of R)    */
    double sigma_min_kept;  /* sigma_r of the sketch (N = R^-1: an estimate,
                               1 / |R^-1|_2 from eight power steps)          */
    double t_sketch_ms;     /* RNG + sketch GEMM                                 */
    double t_svd_ms;        /* QR + Jacobi + cutoff + N                          */
    double t_iter_ms;       /* iterations incl. x = N y                          */
    double t_refine_ms;     /* refinement                                        */
    double t_total_ms;
    /* with opt->profile: summed durations of the sketch GEMM kernel and of
     * the row-sweep kernels (each sweep = one pass over A), and their
     * counts; sweeps enqueued past the last iteration of a loop (they find
     * the loop finished and read nothing) are not counted */
    double t_sketch_kernel_ms;
    double t_sweep_kernel_ms;
    int64_t sketch_kernels;
    int64_t sweep_kernels;
    /* with opt->profile: span of the Jacobi round kernels (summed per
     * sweep) and the number of round launches */
    double t_jacobi_kernel_ms;
    int64_t jacobi_kernels;
    /* precision form: refinement steps whose sweeps read the FP64 A because
     * the FP32 ones had stopped shrinking the corrections                   */
    int64_t fp64_refine_steps;
    /* Chebyshev runs (main solve and refinement corrections) that failed the
     * check after the run and were continued by LSQR.  Theorem 3's bounds
     * hold with a probability (Lemma 3); inside them the normal-equation
     * gradient after the run is at most tol times the starting one, and a
     * run outside them grows it instead.  The check passes when ||g|| <=
     * 2 max(tol, 2^-27) ||g0|| (tall: g = (A N)^T r, g0 = (A N)^T b; fat:
     * the residual of M^T A x = M^T b against M^T b; the floor 2^-27 stays
     * above the rounding of the products A (N y)); on failure LSQR
     * continues from the Chebyshev iterate (from 0 when the run left a
     * residual above the right-hand side's).                               */
    int64_t cs_fallbacks;
    /* the preconditioner formed: LSRN_PRECOND_SVD (N = V_r Sigma_r^-1 from
     * the Jacobi SVD) or LSRN_PRECOND_QR (N = R^-1: chosen by
     * opt->precond, or by LSRN_PRECOND_AUTO when |R|_F |R^-1|_F
     * <= 1 / (2 rcond) certifies that the SVD would keep every singular
     * value -- the sketch's R^-1 and V Sigma^-1 differ by an orthogonal
     * factor, so the preconditioned spectrum and the solution are the
     * same; sweeps is then 0 and sigma_max / sigma_min_kept are estimates).
     * 0 when no preconditioner was formed (lsrn_iterate_*). */
    int64_t precond_used;
} lsrn_info;

/* Fill *opt with the defaults listed above. */
void lsrn_default_options(lsrn_options *opt);

/* Short text for a status code (static storage). */
const char *lsrn_status_string(lsrn_status st);

/* Message describing the last failure of a call made on this thread. */
const char *lsrn_last_error(void);

/*
 * Min-length solution x (length n) of min ||A x - b||_2 for dense FP64 A
 * (m x n) -- Alg. 1 when m >= n, Alg. 2 when m < n.  With opt->lambda > 0
 * the Tikhonov problem min ||A x - b||^2 + lambda^2 ||x||^2 (Sec. 5,
 * W = lambda I): m >= n runs Alg. 1 on the over-determined [A; lambda I_n]
 * (rhs [b; 0]); m < n runs Alg. 2 on the under-determined [A, lambda I_m]
 * (Sec. 5's form with the scale lambda taken into the unknown), whose
 * min-length solution is [x; (b - A x) / lambda] -- the sketch size is then
 * ceil(gamma m), not ceil(gamma n).
 * b: length m.  x: length n, overwritten.  opt may be NULL (defaults).
 * info may be NULL.  Errors: LSRN_E_INVALID for m, n <= 0, NULL pointers,
 * gamma <= 1, tol <= 0, lambda < 0, lda too small, bad layout or method.
 */
lsrn_status lsrn_solve_dense(int64_t m, int64_t n, const double *A, int64_t lda,
                             int32_t layout, const double *b, double *x,
                             const lsrn_options *opt, lsrn_info *info, void *stream);

/* lsrn_solve_dense for A stored in FP32 (b and x FP64): the least-squares
 * problem of the stored FP32 values, solved in FP64 arithmetic -- the
 * sketch reads the FP32 entries into the FP64 matrix cores, the sweeps load
 * them as FP32 and accumulate in FP64, and refinement residuals are formed
 * from them exactly in double-double, so the FP64 accuracy bar holds while
 * every pass over A moves half the bytes.  Same layouts, options (precision
 * must be FP64; LSRN_E_UNSUPPORTED otherwise) and errors as
 * lsrn_solve_dense. */
lsrn_status lsrn_solve_dense_f32(int64_t m, int64_t n, const float *A, int64_t lda, int32_t layout,
                                 const double *b, double *x, const lsrn_options *opt,
                                 lsrn_info *info, void *stream);

/* Bytes of device workspace lsrn_solve_dense allocates for these sizes
 * (used for HBM admission by callers that batch solves). */
size_t lsrn_workspace_bytes(int64_t m, int64_t n, int32_t layout, const lsrn_options *opt);

/*
 * The same solve for sparse A (m x n) in CSR: rowptr (m + 1 int64, rowptr[0]
 * = 0, rowptr[m] = nnz, nondecreasing), colind (nnz int32 in [0, n)), val
 * (nnz FP64); entries of a row in any order (sums follow the given order).
 * The sketch G T and every iteration read the nonzeros only (Sec. 4.3: the
 * cost follows nnz); the library builds a transposed copy of the structure
 * (12 nnz + 8 (n + 1) bytes) for the products with A^T.  Needs nnz, m, n <
 * 2^31.  Errors as lsrn_solve_dense, plus LSRN_E_INVALID for a malformed
 * structure (checked on the device before use).
 */
lsrn_status lsrn_solve_csr(int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                           const int32_t *colind, const double *val, const double *b, double *x,
                           const lsrn_options *opt, lsrn_info *info, void *stream);

/* Device bytes lsrn_solve_csr allocates for these sizes. */
size_t lsrn_workspace_bytes_csr(int64_t m, int64_t n, int64_t nnz, const lsrn_options *opt);

/* ------------------------------------------------------------------------
 * Step-level entry points.  Each runs one step of the path in the same
 * kernels lsrn_solve_dense uses, so that every step can be checked alone.
 * ---------------------------------------------------------------------- */

/* Philox4x32-10 words (Salmon et al., SC'11) behind G:
 * out[((r * nq) + j) * 4 + w] = word w of the block with counter
 * (q_lo, q_hi, row_lo, row_hi), q = q0 + j, row = row0 + r, and key
 * (seed_lo, seed_hi).  out: nrows * nq * 4 uint32. */
lsrn_status lsrn_philox_words(uint64_t seed, int64_t row0, int64_t nrows, int64_t q0,
                              int64_t nq, uint32_t *out, void *stream);

/* Entries of G: out[r * ncols + c] = G(row0 + r, col0 + c), where block q
 * = col / 4 gives words w0..w3 and Box-Muller maps (w0, w1) to columns
 * 4q, 4q+1 and (w2, w3) to 4q+2, 4q+3 with u = (w + 1/2) 2^-32,
 * g = sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1). */
lsrn_status lsrn_gauss_fill(uint64_t seed, int64_t row0, int64_t nrows, int64_t col0,
                            int64_t ncols, double *out, void *stream);

/* Sketch X = G T (Alg. 1/2 step 3) with T the tall view of A: T = A if
 * m >= n, else T = A^T, followed by the rows lambda I_d when lambda > 0
 * ([A; lambda I_n] or [A^T; lambda I_m], Sec. 5).
 * X is s x d (d = n if tall else m), written COLUMN-MAJOR: X[i][j] at
 * X[j * s + i].  G(i, k) as in lsrn_gauss_fill. */
lsrn_status lsrn_sketch_dense(int64_t m, int64_t n, const double *A, int64_t lda,
                              int32_t layout, double lambda, int64_t s, uint64_t seed,
                              double *X, void *stream);

/* Size of the static device scratch behind lsrn_sketch_dense_noalloc:
 * 64 MiB (the partial sums of every sketch with min(m, n) <= 512 and
 * s = 2 min(m, n) fit), held on every device the library runs on until
 * the process ends. */
#define LSRN_NOALLOC_SCRATCH_BYTES (64ll << 20)

/* lsrn_sketch_dense for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result bit for bit, with the
 * split-K partial sums of small tile grids kept in the library's static
 * scratch (LSRN_NOALLOC_SCRATCH_BYTES) instead of an allocation.  It
 * allocates nothing and does not synchronise: it returns once the work is
 * enqueued on `stream`.  A must be stored so that it is read in place
 * (row-major when m >= n, column-major when m < n;
 * LSRN_E_UNSUPPORTED otherwise).  LSRN_E_NOMEM when the partial sums of
 * this shape would exceed the scratch.  All calls on one device share its
 * scratch: calls whose work overlaps on the device (enqueued on different
 * streams without ordering between them) race; calls on one stream, or
 * ordered by events, do not. */
lsrn_status lsrn_sketch_dense_noalloc(int64_t m, int64_t n, const double *A, int64_t lda,
                                      int32_t layout, double lambda, int64_t s, uint64_t seed,
                                      double *X, void *stream);

/* The precision form's sketch X = bf16(G) fl32(T) (+ lambda G(:, K + c) in
 * FP64), arguments and layout as lsrn_sketch_dense. */
lsrn_status lsrn_sketch_dense_bf16(int64_t m, int64_t n, const double *A, int64_t lda,
                                   int32_t layout, double lambda, int64_t s, uint64_t seed,
                                   double *X, void *stream);

/* lsrn_sketch_dense for CSR A (arguments as in lsrn_solve_csr). */
lsrn_status lsrn_sketch_csr(int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                            const int32_t *colind, const double *val, double lambda, int64_t s,
                            uint64_t seed, double *X, void *stream);

/* Steps 4-5 on a sketch X (s x d, column-major, s >= d): Householder QR,
 * one-sided Jacobi on R^T, rank r = #{sigma_i > rcond sigma_1} (rcond <= 0
 * as in lsrn_options), P = V_r Sigma_r^{-1} written row-major d x r with
 * leading dimension d (P must hold d * d doubles).  sigma (length d)
 * receives the singular values in descending order.  *rank and *sweeps
 * are host pointers (sweeps may be NULL).  Synchronises the stream. */
lsrn_status lsrn_precond(int64_t s, int64_t d, const double *X, double rcond, double *sigma,
                         double *P, int64_t *rank, int64_t *sweeps, void *stream);

/* The full-rank alternative (LSRN_PRECOND_QR): Householder QR of X (s x d,
 * column-major, s >= d) and P = R^-1 (row-major d x d, leading dimension
 * d); sigma receives |r_ii| in descending order.  LSRN_E_UNSUPPORTED when
 * min |r_ii| <= rcond max |r_ii| (rcond <= 0: max(s, d) 2^-52).
 * Synchronises the stream. */
lsrn_status lsrn_precond_qr(int64_t s, int64_t d, const double *X, double rcond, double *sigma,
                            double *P, void *stream);

/* Step 6-7 with a given preconditioner: P (d x r, row-major, leading
 * dimension ldp >= r) is N (tall) or M (fat) for A as in lsrn_solve_dense;
 * s is the sketch size the Chebyshev bounds use.  Runs LSQR or Chebyshev
 * (opt->method), opt->refine refinement steps, and writes x.  info->iters
 * etc. are filled. */
lsrn_status lsrn_iterate_dense(int64_t m, int64_t n, const double *A, int64_t lda,
                               int32_t layout, const double *b, const double *P,
                               int64_t ldp, int64_t r, int64_t s, double *x,
                               const lsrn_options *opt, lsrn_info *info, void *stream);

/* lsrn_iterate_dense for CSR A (arguments as in lsrn_solve_csr). */
lsrn_status lsrn_iterate_csr(int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                             const int32_t *colind, const double *val, const double *b,
                             const double *P, int64_t ldp, int64_t r, int64_t s, double *x,
                             const lsrn_options *opt, lsrn_info *info, void *stream);

/*
 * Many small over-determined solves at once (Alg. 1 for each problem): A[p]
 * dense FP64 row-major, m[p] >= n[p], n[p] <= 512, leading dimension
 * lda[p]; b[p] length m[p]; x[p] length n[p] (arrays of device pointers
 * held on the host).  The sketches of all problems run in one launch; the
 * QR of the sketches (up to 1024 rows) runs for all problems in shared
 * launches; with LSRN_PRECOND_AUTO a problem takes N = R^-1 when
 * |R|_F |R^-1|_F certifies that the SVD would keep every singular value
 * (the rule of lsrn_solve_dense; the inverses of all problems in one
 * launch; precond_used = LSRN_PRECOND_QR), and the other problems (and all
 * with LSRN_PRECOND_SVD) take the Jacobi sweeps (d <= 512) in shared
 * launches; then the LSQR iterations of all
 * problems advance together: every kernel launch covers the whole batch
 * (one work item per problem row block, column chunk or problem) and each
 * chunk of iterations is replayed as a HIP graph, so the number of
 * launches does not grow with the number of problems.  opt->refine
 * refinement steps follow the same way (the double-double residual
 * A^T (b - A x) of every problem, then CG on the preconditioned normal
 * equations to opt->refine_tol for all problems together, x += N z; as in
 * lsrn_solve_dense).  One option set for all problems.  Chebyshev
 * problems (Alg. 3) run their steps for all of them in shared launches
 * first (the LSQR problems waiting), each with its own schedule from its
 * bounds, then the check of lsrn_solve_dense (cs_fallbacks = 1 and an LSQR
 * restart where it fails), then the LSQR problems and the restarts
 * together; LSRN_E_UNSUPPORTED for the whole call if a Chebyshev problem's
 * bounds do not hold (sqrt(s) - sqrt(r) - t_margin <= 0).  lambda = 0,
 * precond AUTO or SVD (LSRN_E_UNSUPPORTED otherwise).  The
 * batched path computes in FP64 only: a problem that asks for
 * LSRN_PREC_MIXED is solved exactly as with LSRN_PREC_FP64 (the precision
 * form's result is the FP64 answer its refinement reaches; for problems
 * this small FP32 sweeps save nothing).  infos (count entries, may be NULL) report per problem; the
 * stage times are those of the whole batch (t_iter_ms includes the
 * refinement).  LSRN_E_NOT_CONVERGED if any problem's LSQR reached
 * max_iter (its x holds the last iterate, refined).
 */
lsrn_status lsrn_solve_batch(int32_t count, const int64_t *m, const int64_t *n,
                             const double *const *A, const int64_t *lda, const double *const *b,
                             double *const *x, const lsrn_options *opt, lsrn_info *infos,
                             void *stream);

/* lsrn_solve_batch with one option set per problem (opts: count entries):
 * each problem has its own seed, gamma, tol, max_iter, refine and
 * refine_tol; every problem must meet the batch's limits above, and all
 * must share rcond (their preconditioners are formed together).  A
 * problem's result does not depend on the other problems of the batch: it
 * equals the same problem batched alone.  The serving runtime solves its
 * qualifying requests together through this call (an addition, not a step
 * of the paper). */
lsrn_status lsrn_solve_batch_opts(int32_t count, const int64_t *m, const int64_t *n,
                                  const double *const *A, const int64_t *lda, const double *const *b,
                                  double *const *x, const lsrn_options *opts, lsrn_info *infos,
                                  void *stream);

/* ------------------------------------------------------------------------
 * Launch-shape tuning table (not a paper passage).  Keys are (phase, dtype,
 * rows bucket, cols): phase "sweep" is the fused pass over dense A, dtype
 * "f64" or "f32" (precision form), rows bucket = ceil(log2(rows of the tall
 * view)), cols = d.  The value is the number of sweep workgroups per
 * compute unit.  Entries are made by solves with opt->autotune set and used
 * by every later solve in the process; the choice changes only the
 * summation order of the sweep's partial sums, so importing a table
 * reproduces results across processes.  The table is process-wide and
 * guarded by a mutex.
 * ---------------------------------------------------------------------- */

/* Write the table as text, one "phase dtype rows_log2 cols value" line per
 * entry, into buf (len bytes, NUL-terminated when it fits); returns the
 * length the text needs including the NUL. */
size_t lsrn_tune_export(char *buf, size_t len);

/* Add the entries of such a text (replacing equal keys); LSRN_E_INVALID on
 * a malformed line (then nothing is added). */
lsrn_status lsrn_tune_import(const char *text);

/* Forget every entry. */
void lsrn_tune_clear(void);

/* ------------------------------------------------------------------------
 * A given only through products (Sec. 1 and 4: LSRN needs A only through
 * A v and A^T u, and the sketch G A).
 *
 * The routine computes out = A in (trans = 0; in: n x k, out: m x k) or
 * out = A^T in (trans = 1; in: m x k, out: n x k), both column-major with
 * leading dimensions ldin and ldout, device pointers.  It must enqueue its
 * work on `stream` (or finish it before returning), must not write `in`,
 * and returns 0 on success; any other value ends the solve with
 * LSRN_E_INVALID.  The library calls it with k up to s (sketch: G^T in
 * column blocks of at most 2^27 / max(m, n) columns, i.e. <= 1 GiB) and with
 * k = 1 (iterations: one product with A and one with A^T per iteration,
 * since the fused pass needs A's rows).
 * ---------------------------------------------------------------------- */
typedef int (*lsrn_apply_fn)(void *ctx, int32_t trans, int64_t k, const double *in, int64_t ldin,
                             double *out, int64_t ldout, void *stream);

/* The whole solve (Alg. 1 / Alg. 2, Sec. 5) for an operator A (m x n):
 * b length m, x length n; options as lsrn_solve_dense except that
 * refinement and the precision form are not provided (refine must be 0,
 * precision FP64; LSRN_E_UNSUPPORTED otherwise).  The sketch is formed
 * from the routine's products with G^T, generated block by block. */
lsrn_status lsrn_solve_op(int64_t m, int64_t n, lsrn_apply_fn apply, void *ctx, const double *b,
                          double *x, const lsrn_options *opt, lsrn_info *info, void *stream);

/* ------------------------------------------------------------------------
 * Plans: steps 1-5 of Alg. 1/2 (sketch, SVD, preconditioner N or M) run
 * once for a matrix; lsrn_plan_solve then runs steps 6-7 (and refinement)
 * for any number of right-hand sides.  By Thm. 2 the preconditioner does
 * not depend on b, so every solve gets the min-length solution; a solve
 * through a plan returns bit for bit what lsrn_solve_dense /
 * lsrn_solve_csr return for the same A, b and options.
 *
 * The plan keeps the caller's pointers to A (it copies only what a layout
 * conversion needs): A must stay valid and unchanged until
 * lsrn_plan_destroy.  The plan owns its preconditioner (d x d FP64), the
 * transposed copy of A when the layout needs one, the CSR transpose, and
 * (precision form) the FP32 copy of A.  Creation synchronises `stream`;
 * afterwards the plan is read-only, so solves on one plan may run
 * concurrently on different streams.
 *
 * `opt` of lsrn_plan_solve may be NULL (the creation options) or carry new
 * per-solve settings: tol, max_iter, method, refine, refine_tol, profile.
 * gamma, lambda, seed, rcond, precond and precision must equal the
 * creation ones (LSRN_E_INVALID otherwise).  Errors as in lsrn_solve_dense.
 * ---------------------------------------------------------------------- */
typedef struct lsrn_plan lsrn_plan;

/* Steps 1-5 for dense A (arguments as lsrn_solve_dense); *out receives the
 * plan; info (may be NULL) reports the sketch and the SVD (s, d, rank,
 * sweeps, sigma_max, sigma_min_kept, t_sketch_ms, t_svd_ms). */
lsrn_status lsrn_plan_create_dense(int64_t m, int64_t n, const double *A, int64_t lda,
                                   int32_t layout, const lsrn_options *opt, lsrn_plan **out,
                                   lsrn_info *info, void *stream);

/* Steps 1-5 for CSR A (arguments as lsrn_solve_csr). */
lsrn_status lsrn_plan_create_csr(int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                                 const int32_t *colind, const double *val,
                                 const lsrn_options *opt, lsrn_plan **out, lsrn_info *info,
                                 void *stream);

/* Steps 6-7 (+ refinement) for b (length m) into x (length n). */
lsrn_status lsrn_plan_solve(const lsrn_plan *plan, const double *b, double *x,
                            const lsrn_options *opt, lsrn_info *info, void *stream);

/* Regularisation path (Sec. 5, closing paragraph: for a new W only the
 * sketch of W is new): re-form the plan's preconditioner for the Tikhonov
 * weight `lambda` (>= 0) from the sketch kept at creation (opt.keep_sketch;
 * LSRN_E_INVALID otherwise) -- X(lambda) = G T + lambda G(:, K .. K+d-1),
 * the same bits as a fresh sketch with that lambda -- then SVD, rank and N
 * (or M) again.  Later lsrn_plan_solve calls solve the problem with this
 * lambda and return bit for bit what lsrn_solve_dense / lsrn_solve_csr
 * return for it.  info (may be NULL) reports s, d, rank, sweeps, sigma and
 * the stage times (t_sketch_ms covers only the added rows).  Must not run
 * while solves on this plan are in flight.  Synchronises `stream`. */
lsrn_status lsrn_plan_set_lambda(lsrn_plan *plan, double lambda, lsrn_info *info, void *stream);

/* The oversampling factor gamma in [gamma_min, gamma_max] that minimises a
 * solve's modelled time, from the stage times and counts of a solve
 * measured with some gamma0 (`measured`: s, d, rank, iters, t_sketch_ms,
 * t_svd_ms, t_iter_ms) -- Sec. 6.3's choice of gamma.  The model (Sec. 4.3's
 * cost terms): the sketch time grows with s; of the SVD, the QR part
 * (2 s d^2 flop) grows with s and the rest (11 d^3) does not; the iteration
 * time scales with the Alg. 3 count for the bounds of (s, r) (Theorem 3,
 * t = 1) at tolerance `tol`.  Host arithmetic only (no device call). */
lsrn_status lsrn_tune_gamma(const lsrn_info *measured, double tol, double gamma_min,
                            double gamma_max, double *gamma_out);

/* Free the plan's device memory (after its solves have finished). */
void lsrn_plan_destroy(lsrn_plan *plan);

/* ------------------------------------------------------------------------
 * Serving runtime: solves of different shapes submitted as they arrive,
 * admitted by device-memory footprint onto a pool of streams (not a paper
 * passage: the serving loop around Alg. 1/2).
 *
 * A request is admitted, in arrival order, when one of `streams` worker
 * streams is free and its footprint (lsrn_workspace_bytes /
 * lsrn_workspace_bytes_csr, plus the FP32 copy of the precision form) fits
 * in `hbm_budget_bytes` next to the solves already running; a request
 * larger than the budget runs alone.  Admitted solves overlap on the device
 * and each runs exactly the kernels of lsrn_solve_dense / lsrn_solve_csr,
 * so its result equals that of the same call made alone.  Requests that
 * lsrn_solve_batch_opts covers (dense row-major, m >= n, n <= 512, valid
 * options, lambda = 0, precond AUTO or SVD, rcond 0; Chebyshev ones only
 * when their bounds hold at full rank) queue apart instead: max(1,
 * streams / 2) batcher threads, each on a stream of its own, take the
 * waiting ones of one method (up to 256, within the budget, without the
 * FP32 copy: the batched path computes in FP64) and solve them in one
 * lsrn_solve_batch_opts call, so each such result equals that of the same
 * request batched alone (lsrn_server_timing.batch_size reports the batch).  Served requests
 * never tune launch shapes (opt.autotune is ignored; recorded shapes are
 * used): timings taken while other solves share the device are noise, and
 * a new table entry would change the summation order of later requests.
 * The caller keeps
 * A, b and x (device memory) alive and unused until lsrn_server_wait
 * returns for the ticket.  Errors of a request are returned by
 * lsrn_server_wait (message in lsrn_server_last_error()).
 * ---------------------------------------------------------------------- */
typedef struct lsrn_server lsrn_server;

typedef struct lsrn_server_timing {
    double queue_ms;          /* submit -> admitted                          */
    double run_ms;            /* admitted -> finished                        */
    double latency_ms;        /* submit -> finished                          */
    int64_t footprint_bytes;  /* memory the admission reserved               */
    int64_t batch_size;       /* requests solved in the same batched call,
                                 0 for a request solved on its own          */
} lsrn_server_timing;

/* Start the worker threads on the current device.  0 < streams <= 64. */
lsrn_status lsrn_server_create(int64_t hbm_budget_bytes, int32_t streams, lsrn_server **out);

/* Queue a dense solve (arguments as lsrn_solve_dense); *ticket identifies it. */
lsrn_status lsrn_server_submit_dense(lsrn_server *srv, int64_t m, int64_t n, const double *A,
                                     int64_t lda, int32_t layout, const double *b, double *x,
                                     const lsrn_options *opt, int64_t *ticket);

/* Queue a CSR solve (arguments as lsrn_solve_csr). */
lsrn_status lsrn_server_submit_csr(lsrn_server *srv, int64_t m, int64_t n, int64_t nnz,
                                   const int64_t *rowptr, const int32_t *colind, const double *val,
                                   const double *b, double *x, const lsrn_options *opt,
                                   int64_t *ticket);

/* Block until the request finishes; returns its status and fills info and
 * timing (either may be NULL).  A ticket can be waited for once. */
lsrn_status lsrn_server_wait(lsrn_server *srv, int64_t ticket, lsrn_info *info,
                             lsrn_server_timing *timing);

/* Requests queued, running, and the footprint admitted right now. */
lsrn_status lsrn_server_stats(lsrn_server *srv, int64_t *pending, int64_t *running,
                              int64_t *bytes_in_use);

const char *lsrn_server_last_error(void);

/* Finish every queued request, then stop the workers and free the server. */
void lsrn_server_destroy(lsrn_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* LSRN_H */
