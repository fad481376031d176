/*
 * lsrn_oracle.c -- plain CPU reference implementation of LSRN.
 *
 * TEST INFRASTRUCTURE ONLY (see lsrn_oracle.h).  Written for a reader who
 * has the paper (Meng, Saunders, Mahoney, arXiv:1109.5981) beside it: each
 * function follows one step of Algorithms 1-3 in the paper's order, in
 * straight loops, with no blocking, fusion or reordering beyond the step's
 * own definition.  Section / algorithm / equation numbers refer to that
 * paper.  Build:  gcc -O2 -fopenmp -fPIC -shared lsrn_oracle.c -lm
 */
#include "lsrn_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ====================================================================
 * Random normal matrix G (Alg. 1 step 2, Alg. 2 step 2).
 * The paper draws G with a ziggurat sampler (Sec. 6.1); any i.i.d. N(0,1)
 * entries satisfy Theorems 2-4.  Here every entry is a pure function of
 * (seed, row, col): Philox4x32-10 words turned into normals by Box-Muller.
 * ==================================================================== */

/* Philox4x32-10 as defined by Salmon et al. (SC'11): each round multiplies
 * words 0 and 2 by two fixed 32-bit constants, then mixes the high halves
 * with words 1 and 3 and the round key; the key is bumped by the Weyl
 * constants (golden ratio and sqrt(3) - 1, scaled to 32 bits) between
 * rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_philox_block(uint64_t seed, uint64_t row, uint64_t q, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)q, (uint32_t)(q >> 32), (uint32_t)row, (uint32_t)(row >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Box & Muller (1958). */
void orc_box_muller(uint32_t w0, uint32_t w1, double *g0, double *g1)
{
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = ((double)w0 + 0.5) * 0x1p-32;
    double u1 = ((double)w1 + 0.5) * 0x1p-32;
    double rad = sqrt(-2.0 * log(u0));
    *g0 = rad * cos(two_pi * u1);
    *g1 = rad * sin(two_pi * u1);
}

static void gauss_block(uint64_t seed, uint64_t row, uint64_t q, double g[4])
{
    uint32_t w[4];
    orc_philox_block(seed, row, q, w);
    orc_box_muller(w[0], w[1], &g[0], &g[1]);
    orc_box_muller(w[2], w[3], &g[2], &g[3]);
}

double orc_gauss(uint64_t seed, uint64_t row, uint64_t col)
{
    double g[4];
    gauss_block(seed, row, col / 4, g);
    return g[col % 4];
}

void orc_gauss_fill(uint64_t seed, int64_t row0, int64_t nrows, int64_t col0,
                    int64_t ncols, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r)
        for (int64_t c = 0; c < ncols; ++c)
            out[r * ncols + c] = orc_gauss(seed, (uint64_t)(row0 + r), (uint64_t)(col0 + c));
}

/* ====================================================================
 * The matrix A and its products (Sec. 4.1: LSRN touches A only through
 * products with vectors and with G).  Each output is a sum in ascending
 * index order.
 * ==================================================================== */

static double a_at(const orc_matrix *A, int64_t i, int64_t j)
{
    return A->kind == ORC_DENSE_ROW ? A->a[i * A->lda + j] : A->a[j * A->lda + i];
}

void orc_matvec(const orc_matrix *A, const double *x, double *y)
{
    if (A->kind == ORC_CSR) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < A->m; ++i) {
            double acc = 0.0;
            for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
                acc += A->val[p] * x[A->colind[p]];
            y[i] = acc;
        }
        return;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < A->m; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < A->n; ++j)
            acc += a_at(A, i, j) * x[j];
        y[i] = acc;
    }
}

void orc_matvec_t(const orc_matrix *A, const double *y, double *x)
{
    if (A->kind == ORC_CSR) {
        for (int64_t j = 0; j < A->n; ++j)
            x[j] = 0.0;
        for (int64_t i = 0; i < A->m; ++i)
            for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
                x[A->colind[p]] += A->val[p] * y[i];
        return;
    }
    /* Columns in groups of 8 per thread, so that the rows of a row-major A
     * are read along their length; each x[j] is still the sum over i in
     * ascending order. */
#pragma omp parallel for schedule(static)
    for (int64_t j0 = 0; j0 < A->n; j0 += 8) {
        const int64_t j1 = j0 + 8 < A->n ? j0 + 8 : A->n;
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t i = 0; i < A->m; ++i)
            for (int64_t j = j0; j < j1; ++j)
                acc[j - j0] += a_at(A, i, j) * y[i];
        for (int64_t j = j0; j < j1; ++j)
            x[j] = acc[j - j0];
    }
}

/* Alg. 1 when m >= n, Alg. 2 when m < n.  With lambda > 0 the Tikhonov
 * problem is the over-determined [A; lambda I_n] (tall) or, for m < n, the
 * under-determined [A, lambda I_m] (Sec. 5), so the shape of A decides. */
static int is_tall(const orc_matrix *A)
{
    return A->m >= A->n;
}

/* ====================================================================
 * Sketch (Alg. 1 step 3: A~ = G A;  Alg. 2 step 3: A~ = A G).
 * Both are written as X = G T with T the "tall view" (see header), so X is
 * A~ (tall) or A~^T (fat).  X[i][j] = sum_k G(i,k) T[k][j], k ascending.
 * ==================================================================== */

/* Round a float to the nearest BF16 value (8 significant bits), ties to
 * even, returned as a float. */
float orc_bf16_round(float f)
{
    uint32_t u;
    memcpy(&u, &f, sizeof(u));
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    float r;
    memcpy(&r, &u, sizeof(r));
    return r;
}

/* The sketch; with precision_form the entries of G become bf16(fl32(g))
 * and those of A fl32(a) (the Tikhonov rows keep FP64 lambda g). */
static int64_t sketch_impl(const orc_matrix *A, int64_t s, uint64_t seed, double *X,
                           int precision_form)
{
    if (s <= 0 || A->m <= 0 || A->n <= 0)
        return -1;
    const int tall = is_tall(A);
    const int64_t d = tall ? A->n : A->m;
    memset(X, 0, sizeof(double) * (size_t)s * (size_t)d);
#define G_OF(v) (precision_form ? (double)orc_bf16_round((float)(v)) : (v))
#define A_OF(v) (precision_form ? (double)(float)(v) : (v))

    const int64_t K0 = tall ? A->m : A->n;   /* rows of T before any lambda rows */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s; ++i) {
        double *xi = X + i * d;
        double g4[4];
        int64_t cached_q = -1;
        int64_t K = K0;
        if (A->kind == ORC_CSR && !tall) {
            /* T = A^T: column j of X collects row j of A. */
            for (int64_t j = 0; j < A->m; ++j) {
                double acc = 0.0;
                for (int64_t p = A->rowptr[j]; p < A->rowptr[j + 1]; ++p)
                    acc += G_OF(orc_gauss(seed, (uint64_t)i, (uint64_t)A->colind[p])) * A_OF(A->val[p]);
                xi[j] = acc;
            }
            K = 0; /* the rows of T are done */
        }
        for (int64_t k = 0; k < K; ++k) {
            if (k / 4 != cached_q) {
                cached_q = k / 4;
                gauss_block(seed, (uint64_t)i, (uint64_t)cached_q, g4);
            }
            const double g = G_OF(g4[k % 4]);
            if (A->kind == ORC_CSR) {
                for (int64_t p = A->rowptr[k]; p < A->rowptr[k + 1]; ++p)
                    xi[A->colind[p]] += g * A_OF(A->val[p]);
            } else if (tall) {
                for (int64_t j = 0; j < d; ++j)
                    xi[j] += g * A_OF(a_at(A, k, j));
            } else {
                for (int64_t j = 0; j < d; ++j)
                    xi[j] += g * A_OF(a_at(A, j, k));
            }
        }
        if (A->lambda > 0.0) {
            /* Sec. 5: the rows lambda I_d of the augmented tall view are rows
             * K0 .. K0+d-1 of T (T = [A; lambda I_n] when tall, [A^T; lambda
             * I_m] for the under-determined form [A, lambda I_m]); row K0+c
             * has lambda in column c. */
            for (int64_t c = 0; c < d; ++c)
                xi[c] += orc_gauss(seed, (uint64_t)i, (uint64_t)(K0 + c)) * A->lambda;
        }
    }
#undef G_OF
#undef A_OF
    return d;
}

int64_t orc_sketch(const orc_matrix *A, int64_t s, uint64_t seed, double *X)
{
    return sketch_impl(A, s, seed, X, 0);
}

int64_t orc_sketch_bf16(const orc_matrix *A, int64_t s, uint64_t seed, double *X)
{
    return sketch_impl(A, s, seed, X, 1);
}

/* ====================================================================
 * Economy SVD of the sketch (Alg. 1 step 4, Alg. 2 step 4), computed as
 * Householder QR of X followed by one-sided Jacobi on R^T: if R^T J = W has
 * orthogonal columns, then R^T = W J^T, so the columns of W are
 * V_i sigma_i where V are the right singular vectors of R (and of X).
 * ==================================================================== */

int orc_qr_r(int64_t s, int64_t d, const double *X, double *R)
{
    if (s < d || d <= 0)
        return -1;
    double *Xc = (double *)malloc(sizeof(double) * (size_t)s * (size_t)d); /* column-major */
    double *v = (double *)malloc(sizeof(double) * (size_t)s);
    if (!Xc || !v) {
        free(Xc);
        free(v);
        return -2;
    }
    for (int64_t i = 0; i < s; ++i)
        for (int64_t j = 0; j < d; ++j)
            Xc[j * s + i] = X[i * d + j];

    for (int64_t j = 0; j < d; ++j) {
        double *xj = Xc + j * s;
        double norm2 = 0.0;
        for (int64_t i = j; i < s; ++i)
            norm2 += xj[i] * xj[i];
        const double normx = sqrt(norm2);
        if (normx == 0.0)
            continue; /* nothing to annihilate; R[j][j] = 0 */
        /* Reflector H = I - 2 v v^T / (v^T v) mapping x to alpha e_j, with
         * the sign of alpha opposite to x_j so v_j does not cancel. */
        const double alpha = xj[j] >= 0.0 ? -normx : normx;
        for (int64_t i = j; i < s; ++i)
            v[i] = xj[i];
        v[j] -= alpha;
        double vtv = 0.0;
        for (int64_t i = j; i < s; ++i)
            vtv += v[i] * v[i];
#pragma omp parallel for schedule(static)
        for (int64_t c = j + 1; c < d; ++c) {
            double *xc = Xc + c * s;
            double t = 0.0;
            for (int64_t i = j; i < s; ++i)
                t += v[i] * xc[i];
            const double f = 2.0 * t / vtv;
            for (int64_t i = j; i < s; ++i)
                xc[i] -= f * v[i];
        }
        xj[j] = alpha;
        for (int64_t i = j + 1; i < s; ++i)
            xj[i] = 0.0;
    }
    for (int64_t i = 0; i < d; ++i)
        for (int64_t j = 0; j < d; ++j)
            R[i * d + j] = j >= i ? Xc[j * s + i] : 0.0;
    free(Xc);
    free(v);
    return 0;
}

/* Hestenes one-sided Jacobi, cyclic-by-rows pair order.  The rotation for
 * columns (p, q) is the one that diagonalises their 2 x 2 Gram matrix
 * [[a, g], [g, b]] (Golub & Van Loan, Sec. 8.6): zeta = (b - a) / (2 g),
 * t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2),
 * s = c t.  A pair is skipped once |g| <= d eps sqrt(a b). */
int orc_jacobi_rt(int64_t d, const double *R, double *W, int max_sweeps)
{
    /* Column c of Y = R^T is row c of R, which is contiguous. */
    memcpy(W, R, sizeof(double) * (size_t)d * (size_t)d);
    const double tol = (double)d * DBL_EPSILON;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        int64_t rotations = 0;
        for (int64_t p = 0; p + 1 < d; ++p) {
            for (int64_t q = p + 1; q < d; ++q) {
                double *wp = W + p * d, *wq = W + q * d;
                double a = 0.0, b = 0.0, g = 0.0;
                for (int64_t i = 0; i < d; ++i) {
                    a += wp[i] * wp[i];
                    b += wq[i] * wq[i];
                    g += wp[i] * wq[i];
                }
                if (g == 0.0 || fabs(g) <= tol * sqrt(a) * sqrt(b))
                    continue;
                const double zeta = (b - a) / (2.0 * g);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double sn = c * t;
                for (int64_t i = 0; i < d; ++i) {
                    const double x = wp[i], y = wq[i];
                    wp[i] = c * x - sn * y;
                    wq[i] = sn * x + c * y;
                }
                ++rotations;
            }
        }
        if (rotations == 0)
            return sweep;
    }
    return -1;
}

int64_t orc_precond(int64_t s, int64_t d, const double *X, double rcond,
                    double *sigma, double *P, int *sweeps)
{
    double *R = (double *)malloc(sizeof(double) * (size_t)d * (size_t)d);
    double *W = (double *)malloc(sizeof(double) * (size_t)d * (size_t)d);
    double *nrm = (double *)malloc(sizeof(double) * (size_t)d);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)d);
    if (!R || !W || !nrm || !order) {
        free(R); free(W); free(nrm); free(order);
        return -2;
    }
    orc_qr_r(s, d, X, R);
    int sw = orc_jacobi_rt(d, R, W, 60);
    if (sweeps)
        *sweeps = sw;
    for (int64_t c = 0; c < d; ++c) {
        double acc = 0.0;
        for (int64_t i = 0; i < d; ++i)
            acc += W[c * d + i] * W[c * d + i];
        nrm[c] = sqrt(acc);
        order[c] = c;
    }
    /* Descending order of the column norms (insertion sort; ties keep the
     * lower column index first). */
    for (int64_t c = 1; c < d; ++c) {
        int64_t key = order[c];
        int64_t j = c - 1;
        while (j >= 0 && nrm[order[j]] < nrm[key]) {
            order[j + 1] = order[j];
            --j;
        }
        order[j + 1] = key;
    }
    for (int64_t c = 0; c < d; ++c)
        sigma[c] = nrm[order[c]];
    if (rcond <= 0.0)
        rcond = (double)(s > d ? s : d) * DBL_EPSILON;
    int64_t r = 0;
    while (r < d && sigma[0] > 0.0 && sigma[r] > rcond * sigma[0])
        ++r;
    /* Step 5: N = V_r Sigma_r^{-1}; V_i = W_i / sigma_i, so N_i = W_i / sigma_i^2. */
    for (int64_t i = 0; i < d; ++i)
        for (int64_t c = 0; c < r; ++c)
            P[i * d + c] = W[order[c] * d + i] / (sigma[c] * sigma[c]);
    free(R); free(W); free(nrm); free(order);
    return r;
}

/* ====================================================================
 * Iterative solvers (Alg. 1 step 6, Alg. 2 step 6).
 * ==================================================================== */

static double dot(int64_t n, const double *a, const double *b)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i)
        acc += a[i] * b[i];
    return acc;
}

static double nrm2(int64_t n, const double *a) { return sqrt(dot(n, a, a)); }

/* LSQR: Golub-Kahan bidiagonalisation of K started from b, with the QR
 * factorisation of the bidiagonal updated by Givens rotations (Paige and
 * Saunders, ACM TOMS 8, 1982, Secs. 3-4); stopping rules S1/S2 of Sec. 6
 * with atol = btol = tol and no condition-number limit. */
int64_t orc_lsqr(const orc_linop *K, const double *b, double tol, int64_t maxiter, double *x)
{
    const int64_t m = K->rows, n = K->cols;
    double *u = (double *)malloc(sizeof(double) * (size_t)m);
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *tm = (double *)malloc(sizeof(double) * (size_t)m);
    double *tn = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t j = 0; j < n; ++j)
        x[j] = 0.0;

    double beta = nrm2(m, b);
    int64_t itn = 0;
    int converged = 1;
    if (beta > 0.0) {
        for (int64_t i = 0; i < m; ++i)
            u[i] = b[i] / beta;
        K->mvt(K->ctx, u, v);
        double alpha = nrm2(n, v);
        if (alpha > 0.0) {
            for (int64_t j = 0; j < n; ++j) {
                v[j] /= alpha;
                w[j] = v[j];
            }
            const double bnorm = beta;
            double phibar = beta, rhobar = alpha, anorm2 = 0.0;
            converged = 0;
            while (itn < maxiter) {
                ++itn;
                /* beta_{i+1} u_{i+1} = K v_i - alpha_i u_i */
                K->mv(K->ctx, v, tm);
                for (int64_t i = 0; i < m; ++i)
                    u[i] = tm[i] - alpha * u[i];
                beta = nrm2(m, u);
                anorm2 += alpha * alpha + beta * beta;
                if (beta > 0.0)
                    for (int64_t i = 0; i < m; ++i)
                        u[i] /= beta;
                /* alpha_{i+1} v_{i+1} = K^T u_{i+1} - beta_{i+1} v_i */
                K->mvt(K->ctx, u, tn);
                for (int64_t j = 0; j < n; ++j)
                    v[j] = tn[j] - beta * v[j];
                alpha = nrm2(n, v);
                if (alpha > 0.0)
                    for (int64_t j = 0; j < n; ++j)
                        v[j] /= alpha;
                /* Givens rotation eliminating beta_{i+1}. */
                const double rho = hypot(rhobar, beta);
                const double c = rhobar / rho, sn = beta / rho;
                const double theta = sn * alpha;
                rhobar = -c * alpha;
                const double phi = c * phibar;
                phibar = sn * phibar;
                for (int64_t j = 0; j < n; ++j) {
                    x[j] += (phi / rho) * w[j];
                    w[j] = v[j] - (theta / rho) * w[j];
                }
                const double rnorm = phibar;
                const double arnorm = phibar * alpha * fabs(c);
                const double anorm = sqrt(anorm2);
                const double xnorm = nrm2(n, x);
                const double test2 = rnorm > 0.0 ? arnorm / (anorm * rnorm) : 0.0;
                const double test1 = rnorm / bnorm;
                if (test2 <= tol || test1 <= tol + tol * anorm * xnorm / bnorm) {
                    converged = 1;
                    break;
                }
            }
        }
    }
    free(u); free(v); free(w); free(tm); free(tn);
    return converged ? itn : -itn;
}

int64_t orc_cs_iterations(double sigma_l, double sigma_u, double eps)
{
    const double rate = (sigma_u - sigma_l) / (sigma_u + sigma_l);
    if (rate <= 0.0)
        return 1;
    const double K = ceil((log(eps) - log(2.0)) / log(rate));
    return (int64_t)K + 1;
}

int orc_cs_bounds(int64_t s, int64_t r, double t, double *sigma_l, double *sigma_u)
{
    const double lo = sqrt((double)s) - sqrt((double)r) - t;
    const double hi = sqrt((double)s) + sqrt((double)r) + t;
    if (lo <= 0.0)
        return -1;
    *sigma_u = 1.0 / lo;
    *sigma_l = 1.0 / hi;
    return 0;
}

/* Alg. 3.  The step length printed for k = 1 is d - c^2/(2d); the
 * Chebyshev three-term recurrence it instantiates (Golub & Varga 1961)
 * gives its reciprocal, 1/(d - c^2/(2d)), which is used here. */
int64_t orc_cs(const orc_linop *K, const double *b, double sigma_l, double sigma_u,
               double eps, double *x)
{
    const int64_t m = K->rows, n = K->cols;
    const double d = 0.5 * (sigma_u * sigma_u + sigma_l * sigma_l);
    const double c = 0.5 * (sigma_u * sigma_u - sigma_l * sigma_l);
    const int64_t iters = orc_cs_iterations(sigma_l, sigma_u, eps);
    double *v = (double *)calloc((size_t)n, sizeof(double));
    double *r = (double *)malloc(sizeof(double) * (size_t)m);
    double *tm = (double *)malloc(sizeof(double) * (size_t)m);
    double *tn = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t j = 0; j < n; ++j)
        x[j] = 0.0;
    for (int64_t i = 0; i < m; ++i)
        r[i] = b[i];
    double alpha = 0.0, beta = 0.0;
    for (int64_t k = 0; k < iters; ++k) {
        if (k == 0) {
            beta = 0.0;
            alpha = 1.0 / d;
        } else if (k == 1) {
            beta = 0.5 * (c / d) * (c / d);
            alpha = 1.0 / (d - c * c / (2.0 * d));
        } else {
            beta = (alpha * c / 2.0) * (alpha * c / 2.0);
            alpha = 1.0 / (d - alpha * c * c / 4.0);
        }
        K->mvt(K->ctx, r, tn);                 /* v <- beta v + K^T r */
        for (int64_t j = 0; j < n; ++j)
            v[j] = beta * v[j] + tn[j];
        for (int64_t j = 0; j < n; ++j)        /* x <- x + alpha v    */
            x[j] += alpha * v[j];
        K->mv(K->ctx, v, tm);                  /* r <- r - alpha K v  */
        for (int64_t i = 0; i < m; ++i)
            r[i] -= alpha * tm[i];
    }
    free(v); free(r); free(tm); free(tn);
    return iters;
}

/* ====================================================================
 * Preconditioned operators.
 * Tall (Alg. 1 step 6): K = [A; lambda I] N, rows m (+ n), cols r.
 * Fat  (Alg. 2 step 6): K = M^T A, rows r, cols n.
 * P holds N or M (d x r, leading dimension d).
 * ==================================================================== */

typedef struct {
    const orc_matrix *A;
    const double *P;
    int64_t ldp;    /* leading dimension of P */
    int64_t d, r;
    double *tmp_d;  /* length d (n for tall, m for fat) */
    double *tmp_n;  /* length n */
} precond_ctx;

static void p_times(const precond_ctx *c, const double *y, double *out) /* out = P y */
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < c->d; ++i) {
        double acc = 0.0;
        for (int64_t k = 0; k < c->r; ++k)
            acc += c->P[i * c->ldp + k] * y[k];
        out[i] = acc;
    }
}

static void pt_times(const precond_ctx *c, const double *h, double *out) /* out = P^T h */
{
    /* groups of 8 outputs per thread (P is read along its rows); each
     * out[k] is the sum over i in ascending order */
#pragma omp parallel for schedule(static)
    for (int64_t k0 = 0; k0 < c->r; k0 += 8) {
        const int64_t k1 = k0 + 8 < c->r ? k0 + 8 : c->r;
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t i = 0; i < c->d; ++i)
            for (int64_t k = k0; k < k1; ++k)
                acc[k - k0] += c->P[i * c->ldp + k] * h[i];
        for (int64_t k = k0; k < k1; ++k)
            out[k] = acc[k - k0];
    }
}


static void tall_mv(void *vctx, const double *y, double *out)
{
    precond_ctx *c = (precond_ctx *)vctx;
    p_times(c, y, c->tmp_d);
    orc_matvec(c->A, c->tmp_d, out);
    if (c->A->lambda > 0.0)
        for (int64_t j = 0; j < c->A->n; ++j)
            out[c->A->m + j] = c->A->lambda * c->tmp_d[j];
}

static void tall_mvt(void *vctx, const double *u, double *out)
{
    precond_ctx *c = (precond_ctx *)vctx;
    orc_matvec_t(c->A, u, c->tmp_d);
    if (c->A->lambda > 0.0)
        for (int64_t j = 0; j < c->A->n; ++j)
            c->tmp_d[j] += c->A->lambda * u[c->A->m + j];
    pt_times(c, c->tmp_d, out);
}

/* Fat: K = M^T [A, lambda I_m] on x^ = [x; rho] (rho only when lambda > 0,
 * the under-determined Tikhonov form of Sec. 5). */
static void fat_mv(void *vctx, const double *x, double *out)
{
    precond_ctx *c = (precond_ctx *)vctx;
    orc_matvec(c->A, x, c->tmp_d);
    if (c->A->lambda > 0.0)
        for (int64_t i = 0; i < c->A->m; ++i)
            c->tmp_d[i] += c->A->lambda * x[c->A->n + i];
    pt_times(c, c->tmp_d, out);
}

static void fat_mvt(void *vctx, const double *u, double *out)
{
    precond_ctx *c = (precond_ctx *)vctx;
    p_times(c, u, c->tmp_d);
    orc_matvec_t(c->A, c->tmp_d, out);
    if (c->A->lambda > 0.0)
        for (int64_t i = 0; i < c->A->m; ++i)
            out[c->A->n + i] = c->A->lambda * c->tmp_d[i];
}

/* Conjugate gradients (Hestenes & Stiefel 1952) on K^T K z = rhs from z = 0. */
static int64_t cg_normal(const orc_linop *K, const double *rhs, double rtol, int64_t maxit,
                         double *z)
{
    const int64_t n = K->cols, m = K->rows;
    double *res = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *bp = (double *)malloc(sizeof(double) * (size_t)n);
    double *tm = (double *)malloc(sizeof(double) * (size_t)m);
    for (int64_t j = 0; j < n; ++j) {
        z[j] = 0.0;
        res[j] = rhs[j];
        p[j] = rhs[j];
    }
    double rs = dot(n, res, res);
    const double stop = rtol * sqrt(rs);
    int64_t it = 0;
    while (it < maxit && sqrt(rs) > stop && rs > 0.0) {
        ++it;
        K->mv(K->ctx, p, tm);
        K->mvt(K->ctx, tm, bp);
        const double a = rs / dot(n, p, bp);
        for (int64_t j = 0; j < n; ++j) {
            z[j] += a * p[j];
            res[j] -= a * bp[j];
        }
        const double rs_new = dot(n, res, res);
        const double bta = rs_new / rs;
        for (int64_t j = 0; j < n; ++j)
            p[j] = res[j] + bta * p[j];
        rs = rs_new;
    }
    free(res); free(p); free(bp); free(tm);
    return it;
}

/* The check after a Chebyshev run, an addition to Alg. 3.  The run is
 * exact only when the singular values of K lie in [sigma_L, sigma_U]
 * (Theorem 3 gives that with a probability, Lemma 3).  Within those bounds
 * the normal-equation gradient after the run is the Chebyshev residual
 * polynomial, at most eps in absolute value on [sigma_L^2, sigma_U^2],
 * applied to the starting gradient.  Tall (K = [A; lambda I] N): g =
 * K^T (b - K y) against g0 = K^T b.  Fat (K = M^T A): the system is
 * consistent and the residual c - K x is compared with c.  The run passes
 * when ||g|| <= 2 max(eps, 2^-27) ||g0||: the floor 2^-27 (about sqrt(u))
 * stays above the rounding of the products K y = A (N y), whose relative
 * size grows with kappa(A) (1e-12 at kappa 1e6), while a run outside the
 * bounds grows the gradient instead of shrinking it.  On failure LSQR
 * solves K d = (the residual) from d = 0 and sol += d, or, when the run
 * left a residual larger than the right-hand side (it diverged), sol is
 * reset to 0 and LSQR solves the original system.  Returns the LSQR
 * iterations (0 when the run passed; negative when LSQR did not converge)
 * and sets *fell_back. */
static int64_t cs_check_restart(const orc_linop *K, const double *rhs, double *sol, int tall,
                                double eps, double tol, int64_t maxiter, int *fell_back)
{
    const int64_t rows = K->rows, cols = K->cols;
    double *res = (double *)malloc(sizeof(double) * (size_t)rows);
    double *g = (double *)malloc(sizeof(double) * (size_t)cols);
    K->mv(K->ctx, sol, res);
    for (int64_t i = 0; i < rows; ++i)
        res[i] = rhs[i] - res[i];
    double gn, g0;
    if (tall) {
        K->mvt(K->ctx, res, g);
        gn = nrm2(cols, g);
        K->mvt(K->ctx, rhs, g);
        g0 = nrm2(cols, g);
    } else {
        gn = nrm2(rows, res);
        g0 = nrm2(rows, rhs);
    }
    const double floor_rel = ldexp(1.0, -27);
    const double allow = 2.0 * (eps > floor_rel ? eps : floor_rel) * g0;
    int64_t more = 0;
    *fell_back = 0;
    if (!(isfinite(gn) && gn <= allow)) {
        *fell_back = 1;
        /* LSQR continues from the Chebyshev iterate when its residual is no
         * larger than the right-hand side's, else (a divergent run) from 0 */
        const double rl = nrm2(rows, res), bl = nrm2(rows, rhs);
        if (!(isfinite(rl) && rl <= bl)) {
            for (int64_t j = 0; j < cols; ++j)
                sol[j] = 0.0;
            memcpy(res, rhs, sizeof(double) * (size_t)rows);
        }
        double *d = (double *)malloc(sizeof(double) * (size_t)cols);
        more = orc_lsqr(K, res, tol, maxiter, d);
        for (int64_t j = 0; j < cols; ++j)
            sol[j] += d[j];
        free(d);
    }
    free(res);
    free(g);
    return more;
}

/* Alg. 1/2 steps 6-7 (and reference-mode refinement) with a given
 * preconditioner P (d x r, row-major, leading dimension ldp): N for tall
 * problems, M for fat ones; s is the sketch size behind the Chebyshev
 * bounds.  x (length n) receives the solution.  Returns 0, -3 if the
 * Chebyshev bounds do not exist for (s, r). */
int orc_lsrn_iterate(const orc_matrix *A, const double *b, const double *P, int64_t ldp,
                     int64_t r, int64_t s, const orc_options *opt, double *x, orc_info *info)
{
    const int64_t m = A->m, n = A->n;
    const int tall = is_tall(A);
    const int64_t rows = m + (A->lambda > 0.0 ? n : 0);
    const int64_t d = tall ? n : m;
    /* fat: the unknown of [A, lambda I_m] x^ = b is x^ = [x; rho] */
    const int64_t nl = n + (!tall && A->lambda > 0.0 ? m : 0);
    for (int64_t j = 0; j < n; ++j)
        x[j] = 0.0;
    precond_ctx ctx;
    ctx.A = A;
    ctx.P = P;
    ctx.ldp = ldp;
    ctx.d = d;
    ctx.r = r;
    ctx.tmp_d = (double *)malloc(sizeof(double) * (size_t)d);
    ctx.tmp_n = (double *)malloc(sizeof(double) * (size_t)n);
    orc_linop K;
    K.ctx = &ctx;
    if (tall) {
        K.rows = rows; K.cols = r; K.mv = tall_mv; K.mvt = tall_mvt;
    } else {
        K.rows = r; K.cols = nl; K.mv = fat_mv; K.mvt = fat_mvt;
    }

    double sl = 0.0, su = 0.0;
    const int have_bounds = orc_cs_bounds(s, r, opt->t_margin, &sl, &su) == 0;
    info->sigma_l = sl;
    info->sigma_u = su;
    int64_t maxiter = opt->max_iter;
    if (maxiter <= 0)
        maxiter = have_bounds ? orc_cs_iterations(sl, su, opt->tol) + 10 : 10 * d + 100;
    if (opt->method == ORC_CS && !have_bounds) {
        free(ctx.tmp_d); free(ctx.tmp_n);
        return -3;
    }

    const double t2 = now_s();
    /* Right-hand side of the preconditioned problem: [b; 0] (tall) or M^T b (fat). */
    double *rhs = (double *)calloc((size_t)(tall ? rows : r), sizeof(double));
    if (tall) {
        for (int64_t i = 0; i < m; ++i)
            rhs[i] = b[i];
    } else {
        pt_times(&ctx, b, rhs);
    }
    double *sol = (double *)malloc(sizeof(double) * (size_t)(tall ? r : nl));
    int64_t it;
    if (opt->method == ORC_CS) {
        it = orc_cs(&K, rhs, sl, su, opt->tol, sol);
        int fb = 0;
        /* the default cap follows from the bounds the check found wrong */
        const int64_t cap = opt->max_iter > 0 ? opt->max_iter : 4 * maxiter;
        const int64_t more = cs_check_restart(&K, rhs, sol, tall, opt->tol, opt->tol, cap, &fb);
        info->cs_fallbacks += fb;
        it = more >= 0 ? it + more : -(it - more);
    } else {
        it = orc_lsqr(&K, rhs, opt->tol, maxiter, sol);
    }
    info->converged = it >= 0;
    info->iters = it >= 0 ? it : -it;
    /* the refined unknown: x (tall) or x^ = [x; rho] (fat) */
    double *xh = tall ? x : sol;
    if (tall)
        p_times(&ctx, sol, x); /* Alg. 1 step 7: x = N y */
    const double t3 = now_s();
    info->t_iter = t3 - t2;

    /* Reference-mode refinement. */
    int64_t steps = 0;
    for (int32_t step = 0; step < opt->refine; ++step) {
        double xn = nrm2(tall ? n : nl, xh), dxn = 0.0;
        long double *res = (long double *)malloc(sizeof(long double) * (size_t)m);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) {            /* res = b - A x in long double */
            long double acc = (long double)b[i];
            if (A->kind == ORC_CSR) {
                for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
                    acc -= (long double)A->val[p] * (long double)xh[A->colind[p]];
            } else {
                for (int64_t j = 0; j < n; ++j)
                    acc -= (long double)a_at(A, i, j) * (long double)xh[j];
            }
            if (nl > n)   /* under-determined Tikhonov: b - A x - lambda rho */
                acc -= (long double)A->lambda * (long double)xh[n + i];
            res[i] = acc;
        }
        if (tall) {
            /* h = A^T (b - A x) - lambda^2 x, the normal-equation residual of
             * the (augmented) problem, in long double. */
            long double *h = (long double *)malloc(sizeof(long double) * (size_t)n);
            for (int64_t j = 0; j < n; ++j)
                h[j] = -(long double)A->lambda * (long double)A->lambda * (long double)x[j];
            if (A->kind == ORC_CSR) {
                for (int64_t i = 0; i < m; ++i)
                    for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
                        h[A->colind[p]] += (long double)A->val[p] * res[i];
            } else {
                /* groups of 8 columns per thread; each h[j] still sums over
                 * i in ascending order */
#pragma omp parallel for schedule(static)
                for (int64_t j0 = 0; j0 < n; j0 += 8) {
                    const int64_t j1 = j0 + 8 < n ? j0 + 8 : n;
                    for (int64_t i = 0; i < m; ++i)
                        for (int64_t j = j0; j < j1; ++j)
                            h[j] += (long double)a_at(A, i, j) * res[i];
                }
            }
            double *c = (double *)malloc(sizeof(double) * (size_t)r);
#pragma omp parallel for schedule(static)
            for (int64_t k = 0; k < r; ++k) {
                long double acc = 0.0L;
                for (int64_t i = 0; i < d; ++i)
                    acc += (long double)P[i * ldp + k] * h[i];
                c[k] = (double)acc;
            }
            double *z = (double *)malloc(sizeof(double) * (size_t)r);
            cg_normal(&K, c, 1e-13, 500, z);
            double *dx = (double *)malloc(sizeof(double) * (size_t)n);
            p_times(&ctx, z, dx);
            for (int64_t j = 0; j < n; ++j)
                x[j] += dx[j];
            dxn = nrm2(n, dx);
            free(h); free(c); free(z); free(dx);
        } else {
            /* e = M^T (b - A x - lambda rho) in long double; solve
             * M^T [A, lambda I] dx^ = e with the same method as the main
             * solve. */
            double *e = (double *)malloc(sizeof(double) * (size_t)r);
#pragma omp parallel for schedule(static)
            for (int64_t k = 0; k < r; ++k) {
                long double acc = 0.0L;
                for (int64_t i = 0; i < m; ++i)
                    acc += (long double)P[i * ldp + k] * res[i];
                e[k] = (double)acc;
            }
            double *dx = (double *)malloc(sizeof(double) * (size_t)nl);
            if (opt->method == ORC_CS) {
                orc_cs(&K, e, sl, su, opt->tol, dx);
                int fb = 0;
                cs_check_restart(&K, e, dx, 0, opt->tol, opt->tol,
                                 opt->max_iter > 0 ? opt->max_iter : 4 * maxiter, &fb);
                info->cs_fallbacks += fb;
            } else {
                orc_lsqr(&K, e, opt->tol, maxiter, dx);
            }
            for (int64_t j = 0; j < nl; ++j)
                xh[j] += dx[j];
            dxn = nrm2(nl, dx);
            free(e); free(dx);
        }
        free(res);
        ++steps;
        if (dxn <= 1e-15 * xn)
            break;
    }
    info->refine_steps = steps;
    info->t_refine = now_s() - t3;
    if (!tall)
        memcpy(x, sol, sizeof(double) * (size_t)n);   /* x = the first n entries of x^ */

    free(rhs); free(sol); free(ctx.tmp_d); free(ctx.tmp_n);
    return 0;
}

int orc_lsrn_solve(const orc_matrix *A, const double *b, const orc_options *opt,
                   double *x, orc_info *info, double *sigma_out, double *P_out)
{
    orc_info local;
    if (!info)
        info = &local;
    memset(info, 0, sizeof(*info));
    const int64_t m = A->m, n = A->n;
    if (m <= 0 || n <= 0 || !(opt->gamma > 1.0) || !(opt->tol > 0.0) || A->lambda < 0.0)
        return -1;
    const int tall = is_tall(A);
    const int64_t d = tall ? n : m;
    /* Alg. 1/2 step 1: s = ceil(gamma * d). */
    const int64_t s = (int64_t)ceil(opt->gamma * (double)d);
    info->s = s;
    info->d = d;
    info->tall = tall;

    double t0 = now_s();
    double *X = (double *)malloc(sizeof(double) * (size_t)s * (size_t)d);
    double *sigma = (double *)malloc(sizeof(double) * (size_t)d);
    double *P = (double *)malloc(sizeof(double) * (size_t)d * (size_t)d);
    orc_sketch(A, s, opt->seed, X);
    double t1 = now_s();
    int sweeps = 0;
    int64_t r;
    if (opt->precond == ORC_PRECOND_QR) {
        r = orc_precond_qr(s, d, X, opt->rcond, sigma, P);
        if (r < 0) {
            free(X); free(sigma); free(P);
            return -4; /* rank-deficient sketch: the QR-inverse path needs full rank */
        }
    } else {
        r = orc_precond(s, d, X, opt->rcond, sigma, P, &sweeps);
    }
    double t2 = now_s();
    free(X);
    info->t_sketch = t1 - t0;
    info->t_svd = t2 - t1;
    info->rank = r;
    info->sweeps = sweeps;
    if (sigma_out)
        memcpy(sigma_out, sigma, sizeof(double) * (size_t)d);
    if (P_out)
        memcpy(P_out, P, sizeof(double) * (size_t)d * (size_t)d);
    for (int64_t j = 0; j < n; ++j)
        x[j] = 0.0;
    if (r <= 0) {
        info->converged = 1;
        free(sigma); free(P);
        return 0;
    }

    const int rc = orc_lsrn_iterate(A, b, P, d, r, s, opt, x, info);
    free(sigma); free(P);
    return rc;
}

/* QR-inverse preconditioner: P = R^{-1}, column j of P by back
 * substitution on R p_j = e_j (rows j, j-1, ..., 0). */
int64_t orc_precond_qr(int64_t s, int64_t d, const double *X, double rcond,
                       double *diag_out, double *P)
{
    if (s < d || d <= 0)
        return -1;
    double *R = (double *)malloc(sizeof(double) * (size_t)d * (size_t)d);
    double *dg = (double *)malloc(sizeof(double) * (size_t)d);
    if (!R || !dg) {
        free(R);
        free(dg);
        return -1;
    }
    orc_qr_r(s, d, X, R);
    double dmax = 0.0, dmin = INFINITY;
    for (int64_t i = 0; i < d; ++i) {
        dg[i] = fabs(R[i * d + i]);
        if (dg[i] > dmax) dmax = dg[i];
        if (dg[i] < dmin) dmin = dg[i];
    }
    const double rc = rcond > 0.0 ? rcond : (double)(s > d ? s : d) * DBL_EPSILON;
    if (!(dmin > rc * dmax)) {
        free(R);
        free(dg);
        return -1;
    }
    if (diag_out) {
        /* descending order (insertion sort: d is small in the tests) */
        for (int64_t i = 0; i < d; ++i) {
            double v = dg[i];
            int64_t k = i;
            while (k > 0 && diag_out[k - 1] < v) {
                diag_out[k] = diag_out[k - 1];
                --k;
            }
            diag_out[k] = v;
        }
    }
#pragma omp parallel for schedule(dynamic)
    for (int64_t j = 0; j < d; ++j) {
        for (int64_t i = d - 1; i >= 0; --i) {
            double v;
            if (i > j) {
                v = 0.0;
            } else {
                double t = (i == j) ? 1.0 : 0.0;
                for (int64_t k = i + 1; k <= j; ++k)
                    t -= R[i * d + k] * P[k * d + j];
                v = t / R[i * d + i];
            }
            P[i * d + j] = v;
        }
    }
    free(R);
    free(dg);
    return d;
}

/* ====================================================================
 * Brute force: x = A^+ b (Sec. 2.1: x* = V Sigma^{-1} U^T b) from a
 * one-sided Jacobi SVD in long double with accumulated right vectors.
 * ==================================================================== */

int64_t orc_pinv_solve(const orc_matrix *A, const double *b, double rcond, double *x)
{
    const int64_t m = A->m, n = A->n;
    const int tallA = m >= n;
    /* B (len x k) has columns to orthogonalise: A's columns if tall, A's
     * rows otherwise.  B V = W, so B = W V^T. */
    const int64_t len = tallA ? m : n, k = tallA ? n : m;
    long double *B = (long double *)malloc(sizeof(long double) * (size_t)len * (size_t)k);
    long double *V = (long double *)calloc((size_t)k * (size_t)k, sizeof(long double));
    for (int64_t c = 0; c < k; ++c) {
        for (int64_t i = 0; i < len; ++i)
            B[c * len + i] = tallA ? (long double)a_at(A, i, c) : (long double)a_at(A, c, i);
        V[c * k + c] = 1.0L;
    }
    const long double tol = (long double)len * LDBL_EPSILON;
    for (int sweep = 0; sweep < 80; ++sweep) {
        int64_t rotations = 0;
        for (int64_t p = 0; p + 1 < k; ++p)
            for (int64_t q = p + 1; q < k; ++q) {
                long double *bp = B + p * len, *bq = B + q * len;
                long double a = 0, bb = 0, g = 0;
                for (int64_t i = 0; i < len; ++i) {
                    a += bp[i] * bp[i];
                    bb += bq[i] * bq[i];
                    g += bp[i] * bq[i];
                }
                if (g == 0 || fabsl(g) <= tol * sqrtl(a) * sqrtl(bb))
                    continue;
                long double zeta = (bb - a) / (2 * g);
                long double t = (zeta >= 0 ? 1.0L : -1.0L) / (fabsl(zeta) + sqrtl(1 + zeta * zeta));
                long double c = 1 / sqrtl(1 + t * t), sn = c * t;
                for (int64_t i = 0; i < len; ++i) {
                    long double u = bp[i], w = bq[i];
                    bp[i] = c * u - sn * w;
                    bq[i] = sn * u + c * w;
                }
                long double *vp = V + p * k, *vq = V + q * k;
                for (int64_t i = 0; i < k; ++i) {
                    long double u = vp[i], w = vq[i];
                    vp[i] = c * u - sn * w;
                    vq[i] = sn * u + c * w;
                }
                ++rotations;
            }
        if (rotations == 0)
            break;
    }
    long double smax = 0;
    long double *sg = (long double *)malloc(sizeof(long double) * (size_t)k);
    for (int64_t c = 0; c < k; ++c) {
        long double acc = 0;
        for (int64_t i = 0; i < len; ++i)
            acc += B[c * len + i] * B[c * len + i];
        sg[c] = sqrtl(acc);
        if (sg[c] > smax)
            smax = sg[c];
    }
    if (rcond <= 0.0)
        rcond = (double)(m > n ? m : n) * DBL_EPSILON;
    long double *xl = (long double *)calloc((size_t)n, sizeof(long double));
    int64_t rank = 0;
    for (int64_t c = 0; c < k; ++c) {
        if (!(sg[c] > (long double)rcond * smax) || sg[c] == 0)
            continue;
        ++rank;
        long double *wc = B + c * len, *vc = V + c * k;
        if (tallA) {
            /* A = U S V^T with U_c = W_c / s_c: x += V_c (U_c^T b) / s_c */
            long double ub = 0;
            for (int64_t i = 0; i < m; ++i)
                ub += wc[i] * (long double)b[i];
            ub /= sg[c] * sg[c];
            for (int64_t j = 0; j < n; ++j)
                xl[j] += vc[j] * ub;
        } else {
            /* A^T = W V^T => A = V W^T = V S Uh^T with Uh_c = W_c / s_c:
             * x += Uh_c (V_c^T b) / s_c */
            long double vb = 0;
            for (int64_t i = 0; i < m; ++i)
                vb += vc[i] * (long double)b[i];
            vb /= sg[c] * sg[c];
            for (int64_t j = 0; j < n; ++j)
                xl[j] += wc[j] * vb;
        }
    }
    for (int64_t j = 0; j < n; ++j)
        x[j] = (double)xl[j];
    free(B); free(V); free(sg); free(xl);
    return rank;
}
