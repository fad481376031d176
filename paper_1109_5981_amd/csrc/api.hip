// api.hip -- the extern "C" entry points declared in include/lsrn.h.
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <algorithm>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

namespace lsrn {

static thread_local std::string g_last_error;

void fail(lsrn_status st, const std::string &msg) { throw Error{st, msg}; }

void hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) throw Error{LSRN_E_NOMEM, std::string(what) + ": out of device memory"};
    throw Error{LSRN_E_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}

static thread_local hipStream_t g_alloc_stream = nullptr;

void set_alloc_stream(hipStream_t s) { g_alloc_stream = s; }

static thread_local bool g_graphs_allowed = true;
void set_graphs_allowed(bool on) { g_graphs_allowed = on; }
bool graphs_allowed() { return g_graphs_allowed; }

void DevBuf::alloc(size_t bytes) {
    release();
    if (bytes == 0) return;
    void *p = nullptr;
    const bool async = g_alloc_stream != nullptr;
    hipError_t e = async ? hipMallocAsync(&p, bytes, g_alloc_stream) : hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{LSRN_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                                      hipGetErrorString(e)};
    }
    p_ = p;
    n_ = bytes;
    s_ = g_alloc_stream;
    async_ = async;
}

void DevBuf::release() {
    if (p_) {
        if (async_) (void)hipFreeAsync(p_, s_);
        else (void)hipFree(p_);
    }
    p_ = nullptr;
    n_ = 0;
}

int device_cus() {
    // queried once (a thread-safe static); a host without a device (size
    // queries only) plans for 256 CUs
    static const int cus = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return 256;
        }
        return v > 0 ? v : 256;
    }();
    return cus;
}

StageTimer::StageTimer(hipStream_t s) : s_(s) {}
StageTimer::~StageTimer() {
    for (int i = 0; i < n_; ++i) (void)hipEventDestroy(ev_[i]);
}
void StageTimer::mark() {
    if (n_ >= 16) return;
    LSRN_HIP(hipEventCreate(&ev_[n_]));
    LSRN_HIP(hipEventRecord(ev_[n_], s_));
    ++n_;
}
double StageTimer::elapsed_ms(int i, int j) {
    if (i >= n_ || j >= n_) return 0.0;
    LSRN_HIP(hipEventSynchronize(ev_[j]));
    float ms = 0.f;
    LSRN_HIP(hipEventElapsedTime(&ms, ev_[i], ev_[j]));
    return ms;
}

namespace {

lsrn_options defaults() {
    lsrn_options o;
    std::memset(&o, 0, sizeof(o));
    o.gamma = 2.0;
    o.lambda = 0.0;
    o.tol = 1e-14;
    o.rcond = 0.0;
    o.t_margin = 1.0;
    o.refine_tol = 1e-6;
    o.seed = 0;
    o.max_iter = 0;
    o.method = LSRN_LSQR;
    o.refine = 0;
    return o;
}

void check_options(const lsrn_options &o) {
    LSRN_REQUIRE(o.gamma > 1.0 && std::isfinite(o.gamma), "gamma must be > 1");
    LSRN_REQUIRE(o.tol > 0.0 && o.tol < 1.0, "tol must lie in (0, 1)");
    LSRN_REQUIRE(o.lambda >= 0.0 && std::isfinite(o.lambda), "lambda must be >= 0");
    LSRN_REQUIRE(o.method == LSRN_LSQR || o.method == LSRN_CHEBYSHEV, "unknown method");
    LSRN_REQUIRE(o.refine >= 0 && o.refine <= 100, "refine must lie in [0, 100]");
    LSRN_REQUIRE(o.refine_tol > 0.0 && o.refine_tol < 1.0, "refine_tol must lie in (0, 1)");
    LSRN_REQUIRE(std::isfinite(o.t_margin), "t_margin must be finite");
    LSRN_REQUIRE(o.precond == LSRN_PRECOND_AUTO || o.precond == LSRN_PRECOND_SVD ||
                     o.precond == LSRN_PRECOND_QR,
                 "unknown preconditioner kind");
    LSRN_REQUIRE(o.precision == LSRN_PREC_FP64 || o.precision == LSRN_PREC_MIXED,
                 "unknown precision");
    if (o.precision == LSRN_PREC_MIXED && o.method == LSRN_CHEBYSHEV)
        fail(LSRN_E_UNSUPPORTED, "the Chebyshev bounds do not hold for the precision form's sketch");
}

// The tall view T of A (row-major, K x d): A itself for tall row-major or
// fat column-major storage, otherwise a transposed copy in `buf`.
struct TallView {
    bool tall;
    int64_t K, d;
    const double *T;
    int64_t ldt;
    DevBuf buf;
    const float *T32 = nullptr;  // A stored in FP32 (then T is NULL)
};

void make_view(TallView &v, int64_t m, int64_t n, const double *A, int64_t lda, int32_t layout,
               double lambda, hipStream_t st) {
    LSRN_REQUIRE(layout == LSRN_ROW_MAJOR || layout == LSRN_COL_MAJOR, "unknown layout");
    LSRN_REQUIRE(lda >= (layout == LSRN_ROW_MAJOR ? n : m), "lda too small for the layout");
    v.tall = m >= n;
    v.K = v.tall ? m : n;
    v.d = v.tall ? n : m;
    if ((v.tall && layout == LSRN_ROW_MAJOR) || (!v.tall && layout == LSRN_COL_MAJOR)) {
        v.T = A;
        v.ldt = lda;
        return;
    }
    // tall column-major: stored array is A^T (n x m, ld lda) -> T = A (m x n)
    // fat row-major: stored array is A (m x n, ld lda) -> T = A^T (n x m)
    const int64_t rows = v.tall ? n : m, cols = v.tall ? m : n;
    v.buf.alloc((size_t)rows * (size_t)cols * sizeof(double));
    transpose(rows, cols, A, lda, v.buf.as<double>(), st);
    v.T = v.buf.as<double>();
    v.ldt = rows;
}

// The tall view of FP32 storage (same rules as make_view).
void make_view_f32(TallView &v, int64_t m, int64_t n, const float *A, int64_t lda, int32_t layout,
                   double lambda, hipStream_t st) {
    LSRN_REQUIRE(layout == LSRN_ROW_MAJOR || layout == LSRN_COL_MAJOR, "unknown layout");
    LSRN_REQUIRE(lda >= (layout == LSRN_ROW_MAJOR ? n : m), "lda too small for the layout");
    v.tall = m >= n;
    v.K = v.tall ? m : n;
    v.d = v.tall ? n : m;
    v.T = nullptr;
    if ((v.tall && layout == LSRN_ROW_MAJOR) || (!v.tall && layout == LSRN_COL_MAJOR)) {
        v.T32 = A;
        v.ldt = lda;
        return;
    }
    const int64_t rows = v.tall ? n : m, cols = v.tall ? m : n;
    v.buf.alloc((size_t)rows * (size_t)cols * sizeof(float));
    transpose(rows, cols, A, lda, v.buf.as<float>(), st);
    v.T32 = v.buf.as<float>();
    v.ldt = rows;
}

lsrn_status report(const Error &e) {
    g_last_error = e.message;
    return e.status;
}

#define LSRN_API_BEGIN try {
#define LSRN_API_END                                                   \
    }                                                                  \
    catch (const ::lsrn::Error &e) { return report(e); }               \
    catch (const std::bad_alloc &) {                                   \
        g_last_error = "host allocation failed";                       \
        return LSRN_E_NOMEM;                                           \
    }                                                                  \
    catch (const std::exception &e) {                                  \
        g_last_error = e.what();                                       \
        return LSRN_E_INVALID;                                         \
    }                                                                  \
    return LSRN_OK;

void fill_iter_info(lsrn_info *info, int64_t s, int64_t d, int64_t r, bool tall, const IterResult &ir) {
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->s = s; info->d = d; info->rank = r; info->iters = ir.iters;
    info->refine_steps = ir.refine_steps; info->refine_iters = ir.refine_iters;
    info->fp64_refine_steps = ir.fp64_refine_steps;
    info->cs_fallbacks = ir.cs_fallbacks;
    info->tall = tall; info->converged = ir.converged;
    info->sigma_l = ir.sigma_l; info->sigma_u = ir.sigma_u;
    info->t_iter_ms = ir.t_iter_ms; info->t_refine_ms = ir.t_refine_ms;
    info->t_total_ms = ir.t_iter_ms + ir.t_refine_ms;
    info->t_sweep_kernel_ms = ir.t_sweep_kernel_ms;
    info->sweep_kernels = ir.sweep_kernels;
}

// The oversampling factor that minimises a solve's modelled time, from the
// stage times of one solve measured at gamma0 = s0 / d (the cost terms of
// Sec. 4.3; the choice of gamma of Sec. 6.3): the sketch grows with s; of
// the SVD, the QR part (2 s d^2 flop) grows with s and the Jacobi part
// (11 d^3) does not; the iterations follow the Alg. 3 count for the bounds
// of (s, r) (Theorem 3 with t = 1, the LSQR bound of Theorem 4 behaving
// alike), each at the measured per-iteration time.  gamma runs over
// [gamma_min, gamma_max] in steps of 0.01.
double choose_gamma(int64_t s0, int64_t d, int64_t r, int64_t iters0, double tol, double t_sketch,
                    double t_svd, double t_iter, double gamma_min, double gamma_max) {
    (void)iters0;
    auto count = [&](double s) {
        const double lo = std::sqrt(s) - std::sqrt((double)r) - 1.0;
        if (!(lo > 0.0)) return std::numeric_limits<double>::infinity();
        const double su = 1.0 / lo, sl = 1.0 / (std::sqrt(s) + std::sqrt((double)r) + 1.0);
        const double rate = (su - sl) / (su + sl);
        return std::ceil((std::log(tol) - std::log(2.0)) / std::log(rate)) + 1.0;
    };
    const double k0 = count((double)s0);
    auto model = [&](double s) {
        const double it = std::isfinite(k0) ? t_iter * count(s) / k0 : t_iter;
        return t_sketch * s / (double)s0 +
               t_svd * (2.0 * s + 11.0 * (double)d) / (2.0 * (double)s0 + 11.0 * (double)d) + it;
    };
    double best_g = (double)s0 / (double)d, best_t = std::numeric_limits<double>::infinity();
    for (int i = 0;; ++i) {
        const double g = gamma_min + 0.01 * i;
        if (g > gamma_max + 1e-12) break;
        const double s = std::ceil(g * (double)d);
        const double t = model(s);
        if (t < best_t) {
            best_t = t;
            best_g = g;
        }
    }
    return best_g;
}

// Largest min(m, n) the Jacobi kernels of the SVD handle.
constexpr int64_t kSvdMaxD = 8192;

bool use_qr_inverse(const lsrn_options &opt, int64_t d) {
    if (opt.precond == LSRN_PRECOND_QR) return true;
    if (opt.precond == LSRN_PRECOND_SVD) return false;
    if (d <= kSvdMaxD) return false;
    if (opt.lambda > 0.0) return true;
    fail(LSRN_E_UNSUPPORTED,
         "min(m, n) above 8192 needs lambda > 0 (full-rank QR-inverse preconditioner)");
}

// The automatic choice tries N = R^-1 first: it is kept only when R
// certifies that the SVD would keep every singular value (then the Jacobi
// sweeps, most of the preconditioner's time at every size, are skipped).
bool try_full_rank(const lsrn_options &opt, int64_t d) {
    (void)d;
    return opt.precond == LSRN_PRECOND_AUTO;
}

// Steps 1-5 of a solve, kept for the iterations: the preconditioner and
// (precision form) the FP32 copy of the tall view.
struct Prepared {
    int64_t s = 0, d = 0;
    PrecondResult pr;
    DevBuf sigma, P, T32;
    double sketch_kernel_ms = 0.0;
};

// Steps 1-5 for a dense (dv) or sparse (sv) tall view; tm gets two marks
// (after the sketch, after the preconditioner).
// With `plain`, the sketch G T without the Tikhonov rows is kept there (for
// lsrn_plan_set_lambda); the rows lambda G(:, K + c) are then added by the
// same kernel the sketch launches last, so X is the same bit for bit.
void form_preconditioner(int64_t s, int64_t d, double *X, const lsrn_options &opt, hipStream_t st,
                         Prepared &pp);

void prepare(bool tall, int64_t K, int64_t d, const TallView *dv, const SparseView *sv,
             const lsrn_options &opt, hipStream_t st, StageTimer &tm, Prepared &pp,
             DevBuf *plain = nullptr) {
    const int64_t s = (int64_t)std::ceil(opt.gamma * (double)d);
    const bool qr_inv = use_qr_inverse(opt, d);
    const bool mixed = opt.precision == LSRN_PREC_MIXED;
    if (mixed && sv) fail(LSRN_E_UNSUPPORTED, "the precision form is provided for dense A");
    // FP32 sweeps keep the fat iterate in range(fl32(A)^T); residual
    // refinement cannot remove the part outside range(A^T), so the
    // min-length solution would be off by about kappa(A) 2^-24
    if (mixed && !tall)
        fail(LSRN_E_UNSUPPORTED, "the precision form is provided for over-determined A");
    pp.s = s;
    pp.d = d;
    DevBuf X((size_t)s * (size_t)d * sizeof(double));
    if (mixed && dv && dv->T32)
        fail(LSRN_E_UNSUPPORTED, "FP32 storage of A is solved in FP64 arithmetic (precision FP64)");
    const double lam = plain ? 0.0 : opt.lambda;
    if (sv) {
        sketch_csr(*sv, lam, s, opt.seed, X.as<double>(), st,
                   opt.profile ? &pp.sketch_kernel_ms : nullptr);
    } else if (dv->T32) {
        sketch_rows(K, d, dv->T32, dv->ldt, lam, s, opt.seed, X.as<double>(), st,
                    opt.profile ? &pp.sketch_kernel_ms : nullptr);
    } else if (mixed) {
        pp.T32.alloc((size_t)K * (size_t)dv->ldt * sizeof(float));
        to_f32(K, d, dv->T, dv->ldt, pp.T32.as<float>(), st);
        sketch_rows_bf16(K, d, dv->T, dv->ldt, lam, s, opt.seed, X.as<double>(),
                         st, opt.profile ? &pp.sketch_kernel_ms : nullptr);
    } else {
        sketch_rows(K, d, dv->T, dv->ldt, lam, s, opt.seed, X.as<double>(), st,
                    opt.profile ? &pp.sketch_kernel_ms : nullptr);
    }
    if (plain) {
        plain->alloc((size_t)s * (size_t)d * sizeof(double));
        LSRN_HIP(hipMemcpyAsync(plain->as<double>(), X.as<double>(), (size_t)s * (size_t)d * sizeof(double),
                                hipMemcpyDeviceToDevice, st));
        add_identity_rows(K, d, s, opt.lambda, opt.seed, X.as<double>(), st);
    }
    tm.mark();
    (void)qr_inv;
    form_preconditioner(s, d, X.as<double>(), opt, st, pp);
    tm.mark();
}

// Steps 4-5 on a sketch X (overwritten): sigma, rank and P (SVD), or
// P = R^-1 (the full-rank QR-inverse alternative).
void form_preconditioner(int64_t s, int64_t d, double *X, const lsrn_options &opt, hipStream_t st,
                         Prepared &pp) {
    pp.s = s;
    pp.d = d;
    if (!pp.sigma.bytes()) pp.sigma.alloc((size_t)d * sizeof(double));
    if (!pp.P.bytes()) pp.P.alloc((size_t)d * (size_t)d * sizeof(double));
    pp.pr = use_qr_inverse(opt, d)
                ? precond_qr_inverse(s, d, X, opt.rcond, pp.sigma.as<double>(), pp.P.as<double>(), st)
                : precond(s, d, X, opt.rcond, pp.sigma.as<double>(), pp.P.as<double>(), st,
                          opt.profile != 0, try_full_rank(opt, d));
}

// Steps 6-7 (+ refinement) with a prepared preconditioner.
IterResult run_iterations(bool tall, int64_t K, int64_t d, int64_t n, const TallView *dv,
                          const SparseView *sv, const Prepared &pp, const double *b, double *x,
                          const lsrn_options &opt, hipStream_t st) {
    IterResult ir;
    if (pp.pr.rank <= 0) {
        LSRN_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), st));
        return ir;
    }
    IterProblem pb;
    pb.tall = tall; pb.rows = K; pb.cols = d;
    if (sv) pb.sp = sv;
    else { pb.T = dv->T; pb.T32 = dv->T32; pb.ldt = dv->ldt; }
    pb.lambda = opt.lambda;
    pb.P = pp.P.as<double>(); pb.ldp = d;
    pb.r = pp.pr.rank; pb.s = pp.s;
    if (pp.T32.bytes() > 0) {
        pb.T32 = pp.T32.as<float>();
        pb.kappa_sketch = pp.pr.sigma_min_kept > 0.0 ? pp.pr.sigma_max / pp.pr.sigma_min_kept : 0.0;
        lsrn_options om = opt;
        if (om.refine == 0) om.refine = 10;
        return iterate(pb, b, x, om, st);
    }
    return iterate(pb, b, x, opt, st);
}

lsrn_status finish_info(bool tall, const Prepared &pp, const IterResult &ir, const lsrn_options &opt,
                        lsrn_info *info, StageTimer *tm) {
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->s = pp.s; info->d = pp.d; info->rank = pp.pr.rank; info->iters = ir.iters;
        info->refine_steps = ir.refine_steps; info->refine_iters = ir.refine_iters;
        info->fp64_refine_steps = ir.fp64_refine_steps;
        info->cs_fallbacks = ir.cs_fallbacks;
        info->precond_used = pp.pr.full_rank_inverse ? LSRN_PRECOND_QR : LSRN_PRECOND_SVD;
        info->sweeps = pp.pr.sweeps; info->tall = tall; info->converged = ir.converged;
        info->sigma_l = ir.sigma_l; info->sigma_u = ir.sigma_u;
        info->sigma_max = pp.pr.sigma_max; info->sigma_min_kept = pp.pr.sigma_min_kept;
        if (tm) {
            info->t_sketch_ms = tm->elapsed_ms(0, 1);
            info->t_svd_ms = tm->elapsed_ms(1, 2);
            info->t_total_ms = tm->elapsed_ms(0, 3);
        } else {
            info->t_total_ms = ir.t_iter_ms + ir.t_refine_ms;
        }
        info->t_iter_ms = ir.t_iter_ms;
        info->t_refine_ms = ir.t_refine_ms;
        if (opt.profile) {
            info->t_sketch_kernel_ms = pp.sketch_kernel_ms;
            info->sketch_kernels = tm ? 1 : 0;
            info->t_sweep_kernel_ms = ir.t_sweep_kernel_ms;
            info->sweep_kernels = ir.sweep_kernels;
            info->t_jacobi_kernel_ms = pp.pr.t_jacobi_kernel_ms;
            info->jacobi_kernels = pp.pr.jacobi_kernels;
        }
    }
    if (pp.pr.rank > 0 && !ir.converged) {
        g_last_error = "LSQR reached max_iter";
        return LSRN_E_NOT_CONVERGED;
    }
    return LSRN_OK;
}

// Steps 1-7 for a dense (dv) or sparse (sv) tall view; tm has its first mark.
lsrn_status solve_impl(bool tall, int64_t K, int64_t d, int64_t n, const TallView *dv,
                       const SparseView *sv, const double *b, double *x, const lsrn_options &opt,
                       lsrn_info *info, hipStream_t st, StageTimer &tm) {
    Prepared pp;
    prepare(tall, K, d, dv, sv, opt, st, tm, pp);
    const IterResult ir = run_iterations(tall, K, d, n, dv, sv, pp, b, x, opt, st);
    tm.mark();
    return finish_info(tall, pp, ir, opt, info, &tm);
}

}  // namespace

bool options_valid(const lsrn_options &o) {
    try {
        check_options(o);
        return true;
    } catch (const Error &) {
        return false;
    }
}

}  // namespace lsrn

using namespace lsrn;

struct lsrn_plan {
    bool tall = true, sparse = false;
    int64_t m = 0, n = 0;
    lsrn_options opt{};
    lsrn::TallView dv;
    lsrn::SparseView sv;
    lsrn::Prepared pp;
    lsrn::DevBuf plain;  // opt.keep_sketch: the sketch G T without the Tikhonov rows
};

extern "C" {

void lsrn_default_options(lsrn_options *opt) {
    if (opt) *opt = defaults();
}

const char *lsrn_status_string(lsrn_status st) {
    switch (st) {
        case LSRN_OK: return "ok";
        case LSRN_E_INVALID: return "invalid argument";
        case LSRN_E_NOMEM: return "out of device memory";
        case LSRN_E_HIP: return "HIP runtime error";
        case LSRN_E_NOT_CONVERGED: return "not converged";
        case LSRN_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *lsrn_last_error(void) { return g_last_error.c_str(); }

lsrn_status lsrn_philox_words(uint64_t seed, int64_t row0, int64_t nrows, int64_t q0, int64_t nq,
                              uint32_t *out, void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(nrows >= 0 && nq >= 0 && row0 >= 0 && q0 >= 0, "negative size or offset");
    LSRN_REQUIRE(out || nrows * nq == 0, "out is NULL");
    launch_philox_words(seed, row0, nrows, q0, nq, out, (hipStream_t)stream);
    LSRN_API_END
}

lsrn_status lsrn_gauss_fill(uint64_t seed, int64_t row0, int64_t nrows, int64_t col0, int64_t ncols,
                            double *out, void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(nrows >= 0 && ncols >= 0 && row0 >= 0 && col0 >= 0, "negative size or offset");
    LSRN_REQUIRE(out || nrows * ncols == 0, "out is NULL");
    launch_gauss_fill(seed, row0, nrows, col0, ncols, out, (hipStream_t)stream);
    LSRN_API_END
}

lsrn_status lsrn_sketch_dense(int64_t m, int64_t n, const double *A, int64_t lda, int32_t layout,
                              double lambda, int64_t s, uint64_t seed, double *X, void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(m > 0 && n > 0 && s > 0, "sizes must be positive");
    LSRN_REQUIRE(A && X, "NULL pointer");
    LSRN_REQUIRE(lambda >= 0.0, "lambda must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    TallView v;
    make_view(v, m, n, A, lda, layout, lambda, st);
    sketch_rows(v.K, v.d, v.T, v.ldt, lambda, s, seed, X, st);
    LSRN_HIP(hipStreamSynchronize(st));
    LSRN_API_END
}

lsrn_status lsrn_sketch_dense_noalloc(int64_t m, int64_t n, const double *A, int64_t lda,
                                      int32_t layout, double lambda, int64_t s, uint64_t seed,
                                      double *X, void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(m > 0 && n > 0 && s > 0, "sizes must be positive");
    LSRN_REQUIRE(A && X, "NULL pointer");
    LSRN_REQUIRE(lambda >= 0.0, "lambda must be >= 0");
    LSRN_REQUIRE(layout == LSRN_ROW_MAJOR || layout == LSRN_COL_MAJOR, "unknown layout");
    LSRN_REQUIRE(lda >= (layout == LSRN_ROW_MAJOR ? n : m), "lda too small for the layout");
    const bool tall = m >= n;
    if ((tall && layout != LSRN_ROW_MAJOR) || (!tall && layout != LSRN_COL_MAJOR))
        fail(LSRN_E_UNSUPPORTED,
             "the no-allocation sketch reads A in place: row-major when m >= n, "
             "column-major when m < n");
    sketch_rows_noalloc(tall ? m : n, tall ? n : m, A, lda, lambda, s, seed, X,
                        (hipStream_t)stream);
    LSRN_API_END
}

lsrn_status lsrn_sketch_dense_bf16(int64_t m, int64_t n, const double *A, int64_t lda,
                                   int32_t layout, double lambda, int64_t s, uint64_t seed,
                                   double *X, void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(m > 0 && n > 0 && s > 0, "sizes must be positive");
    LSRN_REQUIRE(A && X, "NULL pointer");
    LSRN_REQUIRE(lambda >= 0.0, "lambda must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    TallView v;
    make_view(v, m, n, A, lda, layout, lambda, st);
    sketch_rows_bf16(v.K, v.d, v.T, v.ldt, lambda, s, seed, X, st);
    LSRN_API_END
}

lsrn_status lsrn_precond(int64_t s, int64_t d, const double *X, double rcond, double *sigma,
                         double *P, int64_t *rank, int64_t *sweeps, void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(d > 0 && s >= d, "need s >= d > 0");
    LSRN_REQUIRE(X && sigma && P && rank, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    DevBuf work((size_t)s * (size_t)d * sizeof(double));
    LSRN_HIP(hipMemcpyAsync(work.as<double>(), X, (size_t)s * (size_t)d * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
    PrecondResult pr = precond(s, d, work.as<double>(), rcond, sigma, P, st);
    *rank = pr.rank;
    if (sweeps) *sweeps = pr.sweeps;
    LSRN_API_END
}

lsrn_status lsrn_precond_qr(int64_t s, int64_t d, const double *X, double rcond, double *sigma,
                            double *P, void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(d > 0 && s >= d, "need s >= d > 0");
    LSRN_REQUIRE(X && sigma && P, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    DevBuf work((size_t)s * (size_t)d * sizeof(double));
    LSRN_HIP(hipMemcpyAsync(work.as<double>(), X, (size_t)s * (size_t)d * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
    precond_qr_inverse(s, d, work.as<double>(), rcond, sigma, P, st);
    LSRN_API_END
}

lsrn_status lsrn_iterate_dense(int64_t m, int64_t n, const double *A, int64_t lda, int32_t layout,
                               const double *b, const double *P, int64_t ldp, int64_t r, int64_t s,
                               double *x, const lsrn_options *opt_in, lsrn_info *info,
                               void *stream) {
    LSRN_API_BEGIN
    const lsrn_options opt = opt_in ? *opt_in : defaults();
    check_options(opt);
    LSRN_REQUIRE(m > 0 && n > 0, "sizes must be positive");
    LSRN_REQUIRE(A && b && x && P, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    TallView v;
    make_view(v, m, n, A, lda, layout, opt.lambda, st);
    LSRN_REQUIRE(r > 0 && r <= v.d && ldp >= r && s > 0, "bad preconditioner shape");
    IterProblem pb;
    pb.tall = v.tall; pb.rows = v.K; pb.cols = v.d; pb.T = v.T; pb.ldt = v.ldt;
    pb.lambda = opt.lambda; pb.P = P; pb.ldp = ldp; pb.r = r; pb.s = s;
    IterResult ir = iterate(pb, b, x, opt, st);
    fill_iter_info(info, s, v.d, r, v.tall, ir);
    if (!ir.converged) {
        g_last_error = "LSQR reached max_iter";
        return LSRN_E_NOT_CONVERGED;
    }
    LSRN_API_END
}

lsrn_status lsrn_solve_dense(int64_t m, int64_t n, const double *A, int64_t lda, int32_t layout,
                             const double *b, double *x, const lsrn_options *opt_in,
                             lsrn_info *info, void *stream) {
    LSRN_API_BEGIN
    const lsrn_options opt = opt_in ? *opt_in : defaults();
    check_options(opt);
    LSRN_REQUIRE(m > 0 && n > 0, "sizes must be positive");
    LSRN_REQUIRE(A && b && x, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    StageTimer tm(st);
    tm.mark();
    TallView v;
    make_view(v, m, n, A, lda, layout, opt.lambda, st);
    return solve_impl(v.tall, v.K, v.d, n, &v, nullptr, b, x, opt, info, st, tm);
    LSRN_API_END
}

lsrn_status lsrn_solve_dense_f32(int64_t m, int64_t n, const float *A, int64_t lda, int32_t layout,
                                 const double *b, double *x, const lsrn_options *opt_in,
                                 lsrn_info *info, void *stream) {
    LSRN_API_BEGIN
    const lsrn_options opt = opt_in ? *opt_in : defaults();
    check_options(opt);
    LSRN_REQUIRE(m > 0 && n > 0, "sizes must be positive");
    LSRN_REQUIRE(A && b && x, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    StageTimer tm(st);
    tm.mark();
    TallView v;
    make_view_f32(v, m, n, A, lda, layout, opt.lambda, st);
    return solve_impl(v.tall, v.K, v.d, n, &v, nullptr, b, x, opt, info, st, tm);
    LSRN_API_END
}

lsrn_status lsrn_solve_csr(int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                           const int32_t *colind, const double *val, const double *b, double *x,
                           const lsrn_options *opt_in, lsrn_info *info, void *stream) {
    LSRN_API_BEGIN
    const lsrn_options opt = opt_in ? *opt_in : defaults();
    check_options(opt);
    LSRN_REQUIRE(m > 0 && n > 0, "sizes must be positive");
    LSRN_REQUIRE(b && x, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    StageTimer tm(st);
    tm.mark();
    SparseView v;
    make_sparse_view(v, m, n, nnz, rowptr, colind, val, st);
    return solve_impl(v.tall, v.K, v.d, n, nullptr, &v, b, x, opt, info, st, tm);
    LSRN_API_END
}

lsrn_status lsrn_solve_op(int64_t m, int64_t n, lsrn_apply_fn apply, void *ctx, const double *b,
                          double *x, const lsrn_options *opt_in, lsrn_info *info, void *stream) {
    LSRN_API_BEGIN
    const lsrn_options opt = opt_in ? *opt_in : defaults();
    check_options(opt);
    LSRN_REQUIRE(m > 0 && n > 0, "sizes must be positive");
    LSRN_REQUIRE(apply && b && x, "NULL pointer");
    if (opt.refine != 0 || opt.precision != LSRN_PREC_FP64)
        fail(LSRN_E_UNSUPPORTED, "an operator A is solved without refinement, in FP64");
    hipStream_t st = (hipStream_t)stream;
    StageTimer tm(st);
    tm.mark();
    OpView ov;
    ov.fn = apply; ov.ctx = ctx; ov.m = m; ov.n = n;
    const bool tall = m >= n;
    const int64_t K = tall ? m : n, d = tall ? n : m;
    Prepared pp;
    pp.d = d;
    pp.s = (int64_t)std::ceil(opt.gamma * (double)d);
    const int64_t s = pp.s;
    // sketch: X^T = T^T G^T, G^T generated in blocks of k columns
    DevBuf X((size_t)s * (size_t)d * sizeof(double));
    {
        DevBuf XT((size_t)s * (size_t)d * sizeof(double));
        const int64_t k = std::max<int64_t>(1, std::min<int64_t>(s, ((int64_t)1 << 27) / K));
        DevBuf Gc((size_t)k * (size_t)K * sizeof(double));
        for (int64_t i0 = 0; i0 < s; i0 += k) {
            const int64_t kk = std::min(k, s - i0);
            launch_gauss_fill(opt.seed, i0, kk, 0, K, Gc.as<double>(), st);
            ov.apply_t(1, kk, Gc.as<double>(), K, XT.as<double>() + i0 * d, d, st);
        }
        transpose(s, d, XT.as<double>(), d, X.as<double>(), st);
        if (opt.lambda > 0.0) add_identity_rows(K, d, s, opt.lambda, opt.seed, X.as<double>(), st);
        LSRN_HIP(hipStreamSynchronize(st));  // before the blocks are freed
    }
    tm.mark();
    pp.sigma.alloc((size_t)d * sizeof(double));
    pp.P.alloc((size_t)d * (size_t)d * sizeof(double));
    pp.pr = use_qr_inverse(opt, d)
                ? precond_qr_inverse(s, d, X.as<double>(), opt.rcond, pp.sigma.as<double>(),
                                     pp.P.as<double>(), st)
                : precond(s, d, X.as<double>(), opt.rcond, pp.sigma.as<double>(), pp.P.as<double>(),
                          st, opt.profile != 0, try_full_rank(opt, d));
    X.release();
    tm.mark();
    IterResult ir;
    if (pp.pr.rank > 0) {
        IterProblem pb;
        pb.tall = tall; pb.rows = K; pb.cols = d; pb.op = &ov;
        pb.lambda = opt.lambda; pb.P = pp.P.as<double>(); pb.ldp = d;
        pb.r = pp.pr.rank; pb.s = s;
        ir = iterate(pb, b, x, opt, st);
    } else {
        LSRN_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), st));
    }
    tm.mark();
    return finish_info(tall, pp, ir, opt, info, &tm);
    LSRN_API_END
}

lsrn_status lsrn_plan_create_dense(int64_t m, int64_t n, const double *A, int64_t lda,
                                   int32_t layout, const lsrn_options *opt_in, lsrn_plan **out,
                                   lsrn_info *info, void *stream) {
    LSRN_API_BEGIN
    const lsrn_options opt = opt_in ? *opt_in : defaults();
    check_options(opt);
    LSRN_REQUIRE(out, "NULL pointer");
    *out = nullptr;
    LSRN_REQUIRE(m > 0 && n > 0, "sizes must be positive");
    LSRN_REQUIRE(A, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    auto plan = std::make_unique<lsrn_plan>();
    plan->m = m; plan->n = n; plan->opt = opt;
    StageTimer tm(st);
    tm.mark();
    make_view(plan->dv, m, n, A, lda, layout, opt.lambda, st);
    plan->tall = plan->dv.tall;
    prepare(plan->tall, plan->dv.K, plan->dv.d, &plan->dv, nullptr, opt, st, tm, plan->pp,
            opt.keep_sketch ? &plan->plain : nullptr);
    tm.mark();
    LSRN_HIP(hipStreamSynchronize(st));
    finish_info(plan->tall, plan->pp, IterResult(), opt, info, &tm);
    *out = plan.release();
    LSRN_API_END
}

lsrn_status lsrn_plan_create_csr(int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                                 const int32_t *colind, const double *val,
                                 const lsrn_options *opt_in, lsrn_plan **out, lsrn_info *info,
                                 void *stream) {
    LSRN_API_BEGIN
    const lsrn_options opt = opt_in ? *opt_in : defaults();
    check_options(opt);
    LSRN_REQUIRE(out, "NULL pointer");
    *out = nullptr;
    LSRN_REQUIRE(m > 0 && n > 0, "sizes must be positive");
    hipStream_t st = (hipStream_t)stream;
    auto plan = std::make_unique<lsrn_plan>();
    plan->m = m; plan->n = n; plan->opt = opt; plan->sparse = true;
    StageTimer tm(st);
    tm.mark();
    make_sparse_view(plan->sv, m, n, nnz, rowptr, colind, val, st);
    plan->tall = plan->sv.tall;
    prepare(plan->tall, plan->sv.K, plan->sv.d, nullptr, &plan->sv, opt, st, tm, plan->pp,
            opt.keep_sketch ? &plan->plain : nullptr);
    tm.mark();
    LSRN_HIP(hipStreamSynchronize(st));
    finish_info(plan->tall, plan->pp, IterResult(), opt, info, &tm);
    *out = plan.release();
    LSRN_API_END
}

lsrn_status lsrn_plan_solve(const lsrn_plan *plan, const double *b, double *x,
                            const lsrn_options *opt_in, lsrn_info *info, void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(plan && b && x, "NULL pointer");
    lsrn_options opt = plan->opt;
    if (opt_in) {
        check_options(*opt_in);
        LSRN_REQUIRE(opt_in->gamma == opt.gamma && opt_in->lambda == opt.lambda &&
                         opt_in->seed == opt.seed && opt_in->rcond == opt.rcond &&
                         opt_in->precond == opt.precond && opt_in->precision == opt.precision,
                     "gamma, lambda, seed, rcond, precond and precision must match the plan");
        opt.tol = opt_in->tol;
        opt.max_iter = opt_in->max_iter;
        opt.method = opt_in->method;
        opt.refine = opt_in->refine;
        opt.refine_tol = opt_in->refine_tol;
        opt.profile = opt_in->profile;
        opt.t_margin = opt_in->t_margin;
    }
    hipStream_t st = (hipStream_t)stream;
    const int64_t K = plan->sparse ? plan->sv.K : plan->dv.K;
    const int64_t d = plan->sparse ? plan->sv.d : plan->dv.d;
    const IterResult ir = run_iterations(plan->tall, K, d, plan->n, plan->sparse ? nullptr : &plan->dv,
                                         plan->sparse ? &plan->sv : nullptr, plan->pp, b, x, opt, st);
    return finish_info(plan->tall, plan->pp, ir, opt, info, nullptr);
    LSRN_API_END
}

lsrn_status lsrn_plan_set_lambda(lsrn_plan *plan, double lambda, lsrn_info *info, void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(plan, "NULL pointer");
    LSRN_REQUIRE(lambda >= 0.0 && std::isfinite(lambda), "lambda must be >= 0");
    LSRN_REQUIRE(plan->plain.bytes() > 0, "the plan was created without keep_sketch");
    hipStream_t st = (hipStream_t)stream;
    lsrn_options opt = plan->opt;
    opt.lambda = lambda;
    const int64_t K = plan->sparse ? plan->sv.K : plan->dv.K;
    const int64_t d = plan->pp.d, s = plan->pp.s;
    (void)use_qr_inverse(opt, d);  // d > 8192 needs lambda > 0: rejected before anything changes
    StageTimer tm(st);
    tm.mark();
    DevBuf X((size_t)s * (size_t)d * sizeof(double));
    LSRN_HIP(hipMemcpyAsync(X.as<double>(), plan->plain.as<double>(), (size_t)s * (size_t)d * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
    // Sec. 5: for a new W only the sketch of W is new
    add_identity_rows(K, d, s, lambda, opt.seed, X.as<double>(), st);
    tm.mark();
    form_preconditioner(s, d, X.as<double>(), opt, st, plan->pp);
    tm.mark();
    LSRN_HIP(hipStreamSynchronize(st));
    plan->opt.lambda = lambda;
    finish_info(plan->tall, plan->pp, IterResult(), opt, info, &tm);
    LSRN_API_END
}

lsrn_status lsrn_tune_gamma(const lsrn_info *measured, double tol, double gamma_min,
                            double gamma_max, double *gamma_out) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(measured && gamma_out, "NULL pointer");
    LSRN_REQUIRE(tol > 0.0 && tol < 1.0, "tol must lie in (0, 1)");
    LSRN_REQUIRE(gamma_min > 1.0 && gamma_max >= gamma_min, "need 1 < gamma_min <= gamma_max");
    const lsrn_info &in = *measured;
    LSRN_REQUIRE(in.d > 0 && in.s > in.d && in.rank > 0 && in.iters > 0,
                 "the measured solve must report s, d, rank and iterations");
    *gamma_out = choose_gamma(in.s, in.d, in.rank, in.iters, tol, in.t_sketch_ms, in.t_svd_ms,
                              in.t_iter_ms, gamma_min, gamma_max);
    LSRN_API_END
}

void lsrn_plan_destroy(lsrn_plan *plan) {
    if (!plan) return;
    (void)hipDeviceSynchronize();
    delete plan;
}

lsrn_status lsrn_sketch_csr(int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                            const int32_t *colind, const double *val, double lambda, int64_t s,
                            uint64_t seed, double *X, void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(m > 0 && n > 0 && s > 0, "sizes must be positive");
    LSRN_REQUIRE(X, "NULL pointer");
    LSRN_REQUIRE(lambda >= 0.0, "lambda must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    SparseView v;
    make_sparse_view(v, m, n, nnz, rowptr, colind, val, st);
    sketch_csr(v, lambda, s, seed, X, st);
    LSRN_API_END
}

lsrn_status lsrn_iterate_csr(int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                             const int32_t *colind, const double *val, const double *b,
                             const double *P, int64_t ldp, int64_t r, int64_t s, double *x,
                             const lsrn_options *opt_in, lsrn_info *info, void *stream) {
    LSRN_API_BEGIN
    const lsrn_options opt = opt_in ? *opt_in : defaults();
    check_options(opt);
    LSRN_REQUIRE(m > 0 && n > 0, "sizes must be positive");
    LSRN_REQUIRE(b && x && P, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    SparseView v;
    make_sparse_view(v, m, n, nnz, rowptr, colind, val, st);
    LSRN_REQUIRE(r > 0 && r <= v.d && ldp >= r && s > 0, "bad preconditioner shape");
    IterProblem pb;
    pb.tall = v.tall; pb.rows = v.K; pb.cols = v.d; pb.sp = &v;
    pb.lambda = opt.lambda; pb.P = P; pb.ldp = ldp; pb.r = r; pb.s = s;
    IterResult ir = iterate(pb, b, x, opt, st);
    fill_iter_info(info, s, v.d, r, v.tall, ir);
    if (!ir.converged) {
        g_last_error = "LSQR reached max_iter";
        return LSRN_E_NOT_CONVERGED;
    }
    LSRN_API_END
}

// The batched solve with one option set per problem (ov[p]); lsrn_solve_batch
// passes the same set for all.  Throws; the entry points report.
static lsrn_status solve_batch_body(int32_t count, const int64_t *m, const int64_t *n,
                                    const double *const *A, const int64_t *lda, const double *const *b,
                                    double *const *x, const std::vector<lsrn_options> &ov,
                                    lsrn_info *infos, hipStream_t st) {
    for (int32_t p = 0; p < count; ++p) {
        const lsrn_options &opt = ov[(size_t)p];
        check_options(opt);
        // the precision form is accepted and runs in FP64 like the rest
        if (opt.lambda != 0.0 || opt.precond == LSRN_PRECOND_QR)
            fail(LSRN_E_UNSUPPORTED, "the batched path runs with the automatic or SVD preconditioner, "
                                     "without lambda");
        // the preconditioners of the batch are formed together with one cutoff
        LSRN_REQUIRE(opt.rcond == ov[0].rcond, "batched problems need the same rcond");
    }
    for (int32_t p = 0; p < count; ++p) {
        LSRN_REQUIRE(m[p] >= n[p] && n[p] > 0 && n[p] <= 512, "batched problems need m >= n, 0 < n <= 512");
        LSRN_REQUIRE(A[p] && b[p] && x[p] && lda[p] >= n[p], "bad batched problem");
    }
    StageTimer tm(st);
    tm.mark();
    std::vector<IterProblem> pbs((size_t)count);
    std::vector<const double *> bs((size_t)count);
    std::vector<double *> xs((size_t)count);
    // the sketches, sigmas and preconditioners of all problems carved from
    // one allocation each (32-double alignment)
    std::vector<double *> Xp((size_t)count), Pp((size_t)count), sp((size_t)count);
    std::vector<PrecondResult> prs((size_t)count);
    std::vector<int64_t> ss((size_t)count);
    auto carve = [](size_t elems) { return (std::max<size_t>(elems, 1) + 31) & ~(size_t)31; };
    size_t nx = 0, np = 0, ns = 0;
    for (int32_t p = 0; p < count; ++p) {
        const int64_t d = n[p];
        ss[(size_t)p] = (int64_t)std::ceil(ov[(size_t)p].gamma * (double)d);
        nx += carve((size_t)ss[(size_t)p] * (size_t)d);
        np += carve((size_t)d * (size_t)d);
        ns += carve((size_t)d);
    }
    DevBuf Xpool(std::max<size_t>(nx, 1) * sizeof(double)), Ppool(std::max<size_t>(np, 1) * sizeof(double));
    DevBuf Spool(std::max<size_t>(ns, 1) * sizeof(double));
    size_t ox = 0, op = 0, os = 0;
    for (int32_t p = 0; p < count; ++p) {
        const size_t d = (size_t)n[p];
        Xp[(size_t)p] = Xpool.as<double>() + ox;
        Pp[(size_t)p] = Ppool.as<double>() + op;
        sp[(size_t)p] = Spool.as<double>() + os;
        ox += carve((size_t)ss[(size_t)p] * d);
        op += carve(d * d);
        os += carve(d);
    }
    std::vector<uint64_t> seeds((size_t)count);
    for (int32_t p = 0; p < count; ++p) seeds[(size_t)p] = ov[(size_t)p].seed;
    if (count > 0)
        sketch_rows_batch(count, m, n, A, lda, ss.data(), seeds.data(), Xp.data(), st);
    std::vector<char> tfr((size_t)count);
    for (int32_t p = 0; p < count; ++p) tfr[(size_t)p] = try_full_rank(ov[(size_t)p], n[p]) ? 1 : 0;
    precond_batch(count, ss.data(), n, Xp.data(), count > 0 ? ov[0].rcond : 0.0, sp.data(), Pp.data(),
                  prs.data(), st, tfr.data());
    Xpool.release();
    Spool.release();
    for (int32_t p = 0; p < count; ++p) {
        const int64_t d = n[p];
        IterProblem &pb = pbs[(size_t)p];
        pb.tall = true; pb.rows = m[p]; pb.cols = d; pb.T = A[p]; pb.ldt = lda[p];
        pb.P = Pp[(size_t)p]; pb.ldp = d; pb.r = prs[(size_t)p].rank; pb.s = ss[(size_t)p];
        bs[(size_t)p] = b[p];
        xs[(size_t)p] = x[p];
    }
    tm.mark();
    // rank-0 problems (A = 0) are answered directly; the rest iterate together
    std::vector<IterProblem> live;
    std::vector<const double *> lb;
    std::vector<double *> lx;
    std::vector<int32_t> idx;
    std::vector<lsrn_options> lo;
    for (int32_t p = 0; p < count; ++p) {
        if (pbs[(size_t)p].r > 0) {
            lo.push_back(ov[(size_t)p]);
            live.push_back(pbs[(size_t)p]);
            lb.push_back(bs[(size_t)p]);
            lx.push_back(xs[(size_t)p]);
            idx.push_back(p);
        } else {
            LSRN_HIP(hipMemsetAsync(x[p], 0, (size_t)n[p] * sizeof(double), st));
        }
    }
    std::vector<IterResult> irs = iterate_batch_tall(live, lb, lx, lo, st);
    tm.mark();
    bool all_conv = true;
    std::vector<IterResult> full((size_t)count);
    for (size_t k = 0; k < idx.size(); ++k) full[(size_t)idx[k]] = irs[k];
    for (int32_t p = 0; p < count; ++p) {
        all_conv = all_conv && full[(size_t)p].converged;
        if (!infos) continue;
        lsrn_info &in = infos[p];
        std::memset(&in, 0, sizeof(in));
        in.s = ss[(size_t)p]; in.d = n[p]; in.rank = prs[(size_t)p].rank;
        in.iters = full[(size_t)p].iters; in.sweeps = prs[(size_t)p].sweeps; in.tall = 1;
        in.refine_steps = full[(size_t)p].refine_steps; in.refine_iters = full[(size_t)p].refine_iters;
        in.cs_fallbacks = full[(size_t)p].cs_fallbacks;
        in.precond_used = prs[(size_t)p].full_rank_inverse ? LSRN_PRECOND_QR : LSRN_PRECOND_SVD;
        in.converged = full[(size_t)p].converged;
        in.sigma_l = full[(size_t)p].sigma_l; in.sigma_u = full[(size_t)p].sigma_u;
        in.sigma_max = prs[(size_t)p].sigma_max; in.sigma_min_kept = prs[(size_t)p].sigma_min_kept;
        in.t_svd_ms = tm.elapsed_ms(0, 1);   // sketches + preconditioners of the whole batch
        in.t_iter_ms = tm.elapsed_ms(1, 2);  // batched iterations (and refinement) of the whole batch
        in.t_total_ms = tm.elapsed_ms(0, 2);
    }
    if (!all_conv) {
        g_last_error = "LSQR reached max_iter for at least one problem";
        return LSRN_E_NOT_CONVERGED;
    }
    return LSRN_OK;
}

lsrn_status lsrn_solve_batch(int32_t count, const int64_t *m, const int64_t *n,
                             const double *const *A, const int64_t *lda, const double *const *b,
                             double *const *x, const lsrn_options *opt_in, lsrn_info *infos,
                             void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(count >= 0, "count must be >= 0");
    LSRN_REQUIRE(count == 0 || (m && n && A && lda && b && x), "NULL pointer");
    const std::vector<lsrn_options> ov((size_t)count, opt_in ? *opt_in : defaults());
    return solve_batch_body(count, m, n, A, lda, b, x, ov, infos, (hipStream_t)stream);
    LSRN_API_END
}

lsrn_status lsrn_solve_batch_opts(int32_t count, const int64_t *m, const int64_t *n,
                                  const double *const *A, const int64_t *lda, const double *const *b,
                                  double *const *x, const lsrn_options *opts, lsrn_info *infos,
                                  void *stream) {
    LSRN_API_BEGIN
    LSRN_REQUIRE(count >= 0, "count must be >= 0");
    LSRN_REQUIRE(count == 0 || (m && n && A && lda && b && x && opts), "NULL pointer");
    const std::vector<lsrn_options> ov(opts, opts + count);
    return solve_batch_body(count, m, n, A, lda, b, x, ov, infos, (hipStream_t)stream);
    LSRN_API_END
}

size_t lsrn_workspace_bytes(int64_t m, int64_t n, int32_t layout, const lsrn_options *opt_in) try {
    const lsrn_options opt = opt_in ? *opt_in : defaults();
    if (m <= 0 || n <= 0 || !(opt.gamma > 1.0)) return 0;
    const bool tall = m >= n;
    const int64_t K = tall ? m : n, d = tall ? n : m;
    const int64_t s = (int64_t)std::ceil(opt.gamma * (double)d);
    size_t bytes = 0;
    if ((tall && layout != LSRN_ROW_MAJOR) || (!tall && layout != LSRN_COL_MAJOR))
        bytes += (size_t)m * (size_t)n * sizeof(double);
    bytes += (size_t)s * d * sizeof(double);                 // sketch
    bytes += sketch_workspace_bytes(K, d, s);
    bytes += precond_workspace_bytes(s, d);
    bytes += (size_t)d * d * sizeof(double) * 2 + (size_t)d * sizeof(double);  // P, P^T, sigma
    bytes += (size_t)(K + d) * sizeof(double) * 3;           // long vectors
    bytes += (size_t)1024 * d * sizeof(double) * 3;          // sweep partials
    if (opt.precision == LSRN_PREC_MIXED)                    // FP32 copy, bf16(G)
        bytes += (size_t)K * d * sizeof(float) + sketch_bf16_g_bytes(K, d, s);
    return bytes;
} catch (...) {
    return 0;
}

size_t lsrn_workspace_bytes_csr(int64_t m, int64_t n, int64_t nnz, const lsrn_options *opt_in) try {
    const lsrn_options opt = opt_in ? *opt_in : defaults();
    if (m <= 0 || n <= 0 || nnz < 0 || !(opt.gamma > 1.0)) return 0;
    const bool tall = m >= n;
    const int64_t K = tall ? m : n, d = tall ? n : m;
    const int64_t s = (int64_t)std::ceil(opt.gamma * (double)d);
    const int64_t rows = K + (opt.lambda > 0.0 ? d : 0);
    size_t bytes = sparse_view_bytes(m, n, nnz);               // transposed structure
    bytes += (size_t)nnz * 36;                                 // sketch order + sort temporaries
    bytes += sketch_csr_tile_bytes(K, d, nnz, s);              // group offsets, partial sketches
    bytes += (size_t)s * d * sizeof(double);                   // sketch
    bytes += precond_workspace_bytes(s, d) + (size_t)d * d * sizeof(double);  // QR-inverse (its R^-1 counted above)
    bytes += (size_t)d * d * sizeof(double) * 2 + (size_t)d * sizeof(double);  // P, P^T, sigma
    bytes += (size_t)rows * sizeof(double) * 5;                // long vectors
    return bytes;
} catch (...) {
    return 0;
}

}  // extern "C"
