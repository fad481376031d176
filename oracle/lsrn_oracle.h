/*
 * lsrn_oracle.h -- plain, slow CPU reference implementation of LSRN
 * (Meng, Saunders, Mahoney, "LSRN: A parallel iterative solver for strongly
 * over- or under-determined systems", arXiv:1109.5981).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the GPU path can be
 * checked against an independent, obviously-correct computation.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source, header, table or helper with the HIP
 * library under paper_1109_5981_amd/; neither includes or links the other.
 *
 * Everything is FP64 except the reference-mode residuals, which use
 * long double (x87 80-bit on x86-64).  Matrices are row-major unless a
 * field says otherwise.  All functions are single-process; loops over
 * independent outputs may run under OpenMP, with a fixed summation order per
 * output, so results do not depend on the thread count.
 *
 * Parity status of each function (what pins it, see tests/test_oracle_*.py):
 *   orc_philox4x32_10   pinned: rocRAND's header-only philox4x32_10 engine
 *   orc_gauss           pinned: Box-Muller identity vs libm, moments, KS test
 *   orc_sketch          pinned: exact rational check on integer-valued A,
 *                               brute force via orc_gauss on tiny inputs
 *   orc_sketch_bf16     pinned: torch's BF16 rounding of G times fl32(A)
 *   orc_bf16_round      pinned: torch.bfloat16 conversion, ties to even
 *   orc_qr_r            pinned: R^T R = X^T X, LAPACK |diag R|
 *   orc_jacobi_rt       pinned: LAPACK singular values, W W^T = R^T R
 *   orc_precond         pinned: X N orthonormal, range(N) = range(X^T)
 *   orc_precond_qr      pinned: X P orthonormal, R P = I, P upper triangular
 *   orc_lsqr / orc_cs   pinned: diagonal problems, Chebyshev closed form,
 *                               SciPy LSQR iterates on the same operator
 *   orc_cs_iterations   pinned: Table 3 of the paper (106 iterations)
 *   orc_pinv_solve      pinned: numpy.linalg.pinv / lstsq
 *   orc_lsrn_solve      pinned: brute-force pinv, optimality invariants
 */
#ifndef LSRN_ORACLE_H
#define LSRN_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ RNG */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).
 * ctr: 128-bit counter as 4 words (word 0 least significant);
 * key: 64-bit key as 2 words. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The four words that feed G(row, 4q .. 4q+3):
 * counter = (q_lo, q_hi, row_lo, row_hi), key = (seed_lo, seed_hi). */
void orc_philox_block(uint64_t seed, uint64_t row, uint64_t q, uint32_t out[4]);

/* Box-Muller pair from two 32-bit words: u = (w + 1/2) 2^-32,
 * g0 = sqrt(-2 ln u0) cos(2 pi u1), g1 = sqrt(-2 ln u0) sin(2 pi u1). */
void orc_box_muller(uint32_t w0, uint32_t w1, double *g0, double *g1);

/* Entry (row, col) of the virtual Gaussian matrix of the sketch (Alg. 1/2,
 * step 2).  Words 0,1 of block q = col/4 give cols 4q, 4q+1; words 2,3 give
 * 4q+2, 4q+3. */
double orc_gauss(uint64_t seed, uint64_t row, uint64_t col);

/* out[r*ncols + c] = G(row0 + r, col0 + c). */
void orc_gauss_fill(uint64_t seed, int64_t row0, int64_t nrows, int64_t col0,
                    int64_t ncols, double *out);

/* -------------------------------------------------------------- problem */

enum { ORC_DENSE_ROW = 0, ORC_DENSE_COL = 1, ORC_CSR = 2 };
enum { ORC_LSQR = 0, ORC_CS = 1 };

/* The least-squares matrix A (m x n).  Dense: a with leading dimension lda,
 * row-major (ORC_DENSE_ROW: a[i*lda+j]) or column-major (ORC_DENSE_COL:
 * a[j*lda+i]).  CSR: rowptr[m+1], colind[nnz], val[nnz].
 * lambda > 0 means the Tikhonov problem min ||Ax-b||^2 + lambda^2 ||x||^2
 * (Sec. 5), solved as the over-determined [A; lambda I_n] x ~ [b; 0] when
 * m >= n, and for m < n as the min-length solution x^ = [x; rho] of the
 * under-determined [A, lambda I_m] x^ = b (the paper's form with
 * W = lambda I, scaled by lambda: its minimiser has rho = (b - A x)/lambda,
 * so ||x^||^2 = ||x||^2 + ||b - A x||^2 / lambda^2). */
typedef struct {
    int64_t m, n;
    int32_t kind;
    int32_t pad_;
    const double *a;
    int64_t lda;
    const int64_t *rowptr;
    const int32_t *colind;
    const double *val;
    double lambda;
} orc_matrix;

/* y = A x (length m) and x = A^T y (length n), augmented rows excluded. */
void orc_matvec(const orc_matrix *A, const double *x, double *y);
void orc_matvec_t(const orc_matrix *A, const double *y, double *x);

/* ------------------------------------------------------------ sketch */

/* Tall view: if m >= n, T = A (d = n) and the sketch is X = G T (Alg. 1,
 * step 3).  Otherwise T = A^T (n x m, d = m) and the sketch is
 * X = (A G')^T = G T with G' = G^T (Alg. 2, step 3).  When lambda > 0 the
 * rows lambda I_d follow (T = [A; lambda I_n] or [A^T; lambda I_m]).
 * G(i, k) is orc_gauss(seed, i, k) for i < s, k < rows(T).
 * X is s x d, row-major.  Returns d, or -1 on bad input. */
int64_t orc_sketch(const orc_matrix *A, int64_t s, uint64_t seed, double *X);

/* The precision form's sketch: as orc_sketch with G(i, k) replaced by
 * bf16(fl32(G(i, k))) and A by fl32(A) (exact products summed in FP64);
 * the Tikhonov rows lambda G(i, K + c) stay FP64. */
int64_t orc_sketch_bf16(const orc_matrix *A, int64_t s, uint64_t seed, double *X);

/* Nearest BF16 value of a float (ties to even). */
float orc_bf16_round(float f);

/* ------------------------------------------------------------ SVD */

/* Householder QR of X (s x d, s >= d, row-major); writes the d x d upper
 * triangular factor R (row-major, zeros below the diagonal). */
int orc_qr_r(int64_t s, int64_t d, const double *X, double *R);

/* One-sided (Hestenes) Jacobi on Y = R^T.  On return column c of Y, stored
 * in W[c*d .. c*d+d-1], is orthogonal to the others; W W^T = R^T R.
 * Returns the number of sweeps, or -1 if max_sweeps was reached. */
int orc_jacobi_rt(int64_t d, const double *R, double *W, int max_sweeps);

/* Steps 4-5 of Alg. 1 (and Alg. 2): economy SVD of the sketch X through
 * QR + Jacobi, rank r = #{sigma_i > rcond sigma_1} (rcond <= 0 selects
 * max(s,d) * DBL_EPSILON), and the preconditioner P = V_r Sigma_r^{-1}
 * (tall: N; fat: M = U_r Sigma_r^{-1}).  P is d x r row-major with
 * leading dimension d (room for r = d).  sigma receives all d singular
 * values in descending order.  Returns r. */
int64_t orc_precond(int64_t s, int64_t d, const double *X, double rcond,
                    double *sigma, double *P, int *sweeps);

/* Full-rank alternative to steps 4-5: R from the Householder QR of X
 * (s x d, row-major) and P = R^{-1} (d x d, row-major, upper triangular) by
 * back substitution, so that X P = Q has orthonormal columns.  diag_out
 * (length d, may be NULL) receives |r_ii| in descending order.  Returns d,
 * or -1 when min |r_ii| <= rcond max |r_ii| (rcond <= 0: max(s,d) eps). */
int64_t orc_precond_qr(int64_t s, int64_t d, const double *X, double rcond,
                       double *diag_out, double *P);

/* --------------------------------------------------------- iterations */

/* Linear operator K (rows x cols) given by callbacks. */
typedef struct {
    int64_t rows, cols;
    void (*mv)(void *ctx, const double *x, double *y);   /* y = K x   */
    void (*mvt)(void *ctx, const double *y, double *x);  /* x = K^T y */
    void *ctx;
} orc_linop;

/* LSQR (Paige & Saunders 1982) from x = 0 with atol = btol = tol.
 * Stops when ||K^T r|| <= tol ||K|| ||r|| or ||r|| <= tol ||b|| +
 * tol ||K|| ||x||, with ||K|| the Frobenius estimate of the bidiagonal.
 * Returns the number of iterations, or -(maxiter) if not converged. */
int64_t orc_lsqr(const orc_linop *K, const double *b, double tol, int64_t maxiter,
                 double *x);

/* Chebyshev semi-iteration (Alg. 3): runs k = 0 .. K with
 * K = ceil((ln eps - ln 2) / ln((sU - sL)/(sU + sL))), i.e. K + 1
 * iterations, with the step-1 length 1/(d - c^2/(2d)).  Returns K + 1. */
int64_t orc_cs(const orc_linop *K, const double *b, double sigma_l, double sigma_u,
               double eps, double *x);

/* K + 1 of Alg. 3 for bounds (sigma_l, sigma_u) and tolerance eps. */
int64_t orc_cs_iterations(double sigma_l, double sigma_u, double eps);

/* Singular-value bounds of A N from Theorem 3 with Lemma 3's margin t:
 * sigma_u = 1/(sqrt s - sqrt r - t), sigma_l = 1/(sqrt s + sqrt r + t).
 * Returns 0, or -1 when sqrt s - sqrt r - t <= 0. */
int orc_cs_bounds(int64_t s, int64_t r, double t, double *sigma_l, double *sigma_u);

/* ------------------------------------------------------------ LSRN */

typedef struct {
    double gamma;      /* oversampling factor, > 1 (Alg. 1 step 1)          */
    double tol;        /* LSQR atol = btol, or the CS epsilon               */
    double rcond;      /* rank cutoff relative to sigma_1; <= 0: default    */
    double t_margin;   /* Lemma 3 margin t used for the CS bounds           */
    uint64_t seed;     /* Philox key of the sketch                          */
    int64_t max_iter;  /* LSQR cap; <= 0 selects the CS count + 10          */
    int32_t method;    /* ORC_LSQR or ORC_CS                                */
    int32_t refine;    /* reference-mode refinement steps (0 = none)        */
    int32_t precond;   /* ORC_PRECOND_SVD (0) or ORC_PRECOND_QR (1)         */
    int32_t pad_;
} orc_options;

enum { ORC_PRECOND_SVD = 0, ORC_PRECOND_QR = 1 };

typedef struct {
    int64_t s, d, rank, iters, sweeps, refine_steps;
    double sigma_l, sigma_u;
    double t_sketch, t_svd, t_iter, t_refine;
    int32_t tall;
    int32_t converged;
    int64_t cs_fallbacks;  /* Chebyshev runs that failed the check after the
                              run and were continued by LSQR (see
                              orc_lsrn_iterate)                              */
} orc_info;

/* Min-length least-squares solution x (length n) of min ||Ax - b||
 * (Tikhonov-regularised when A->lambda > 0) by LSRN.  With opt->refine > 0
 * the result is refined: tall problems solve the preconditioned normal
 * equations (A N)^T (A N) dy = N^T A^T (b - A x) with the normal-equation
 * residual in long double; fat problems solve M^T A^ dx^ = M^T (b - A^ x^)
 * (A^ = A, or [A, lambda I_m] with x^ = [x; rho]) with the residual in long
 * double.  Both corrections stay in range(A^T) (range(A^^T)).
 * sigma_out (length d) and P_out (d*d) may be NULL.  Returns 0 on success. */
int orc_lsrn_solve(const orc_matrix *A, const double *b, const orc_options *opt,
                   double *x, orc_info *info, double *sigma_out, double *P_out);

/* Steps 6-7 (and refinement) of the above with a given preconditioner P
 * (d x r, row-major, leading dimension ldp): N for tall problems, M for fat
 * ones; s is the sketch size behind the Chebyshev bounds.  Returns 0, or -3
 * when method = ORC_CS and the bounds do not exist. */
int orc_lsrn_iterate(const orc_matrix *A, const double *b, const double *P, int64_t ldp,
                     int64_t r, int64_t s, const orc_options *opt, double *x, orc_info *info);

/* Brute force x = A^+ b from a one-sided Jacobi SVD of A carried out in long
 * double, singular values below rcond * sigma_1 dropped.  For tiny
 * inputs only (dense A).  Returns the rank. */
int64_t orc_pinv_solve(const orc_matrix *A, const double *b, double rcond, double *x);

/* Number of threads the oracle's OpenMP loops use (1 without OpenMP). */
int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
