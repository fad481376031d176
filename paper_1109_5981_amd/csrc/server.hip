// server.hip -- the serving runtime: continuous admission of least-squares
// solves of different shapes, by device-memory footprint, onto a pool of
// HIP streams.
//
// Requests queue in arrival order.  A request is admitted when a stream is
// free and its footprint (the matrix copies and workspace the solve
// allocates, from the workspace queries) fits in the budget next to the
// solves already running; a request larger than the whole budget runs
// alone.  Each worker thread owns one stream and allocates stream-ordered,
// so the kernels of admitted solves overlap on the device and a request
// that arrives while others run starts as soon as a slot and memory free
// up.  Every solve runs the same kernels in the same order as a call of
// lsrn_solve_dense / lsrn_solve_csr on its own, so its result does not
// depend on what else is running.
//
// Requests the batched path covers (dense row-major over-determined LSQR
// or Chebyshev with n <= 512, lambda = 0 and the default rank cutoff; the
// precision form's requests among them run in FP64 there) queue apart:
// batcher threads (one per two worker streams), each on a stream of its
// own, take all of them that are waiting when free (up to kMaxBatch,
// within the budget) and solve
// them together with lsrn_solve_batch_opts, so that the iterations of
// requests that arrived close together advance in shared launches.  A
// batched request's result equals the same request batched alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

struct lsrn_server {
    struct Request {
        int64_t id = 0;
        bool csr = false;
        int64_t m = 0, n = 0, lda = 0, nnz = 0;
        int32_t layout = 0;
        const double *A = nullptr;
        const int64_t *rowptr = nullptr;
        const int32_t *colind = nullptr;
        const double *val = nullptr;
        const double *b = nullptr;
        double *x = nullptr;
        lsrn_options opt{};
        bool batch = false;  // solved by the batcher
        int64_t batch_size = 0;
        size_t bytes = 0;
        double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
        bool done = false;
        lsrn_status status = LSRN_OK;
        lsrn_info info{};
        std::string error;
    };

    int device = 0;
    size_t budget = 0;
    size_t in_use = 0;
    int running = 0;
    bool stopping = false;
    int64_t next_id = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending, pending_batch;
    std::unordered_map<int64_t, std::unique_ptr<Request>> requests;
    std::vector<std::thread> workers;
    static constexpr int kMaxBatch = 256;

    // A request goes to the batcher only when the batched call would take
    // it (valid options included): one bad request must not fail a batch.
    static bool batchable(const Request &r) {
        const lsrn_options &o = r.opt;
        if (r.csr || r.layout != LSRN_ROW_MAJOR || r.m < r.n || r.n > 512 || r.lda < r.n ||
            !lsrn::options_valid(o) || o.lambda != 0.0 || o.precond == LSRN_PRECOND_QR || o.rcond != 0.0)
            return false;
        if (o.method == LSRN_CHEBYSHEV) {
            // the bounds must hold at full rank (a failure would fail the batch)
            const double s = std::ceil(o.gamma * (double)r.n);
            return std::sqrt(s) - std::sqrt((double)r.n) - o.t_margin > 0.0;
        }
        return true;
    }

    void finish(Request *r, lsrn_status s, const lsrn_info &info, const std::string &err) {
        r->status = s;
        r->info = info;
        if (s != LSRN_OK) r->error = err;
        r->t_done = now_ms();
        r->done = true;
        in_use -= r->bytes;
        --running;
    }

    // Takes every waiting batched request that fits (at least one when
    // nothing runs), solves them together and completes them.
    void batcher() {
        (void)hipSetDevice(device);
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
        lsrn::set_alloc_stream(st);
        // the batched iterations replay graph chunks, captured thread-local
        // so that the workers' allocations stay legal meanwhile
        std::vector<Request *> batch;
        for (;;) {
            batch.clear();
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    if (stopping && pending_batch.empty()) return true;
                    if (pending_batch.empty()) return false;
                    return in_use + pending_batch.front()->bytes <= budget || running == 0;
                });
                if (pending_batch.empty()) break;
                // one method a batch: a batch runs its Chebyshev steps before
                // its LSQR iterations, so mixing the two would hold the LSQR
                // requests back; the others wait for the next batch (in order)
                const int32_t method = pending_batch.front()->opt.method;
                for (auto it = pending_batch.begin(); it != pending_batch.end() && (int)batch.size() < kMaxBatch;) {
                    Request *r = *it;
                    if (r->opt.method != method) {
                        ++it;
                        continue;
                    }
                    if (!(in_use + r->bytes <= budget || (batch.empty() && running == 0))) break;
                    it = pending_batch.erase(it);
                    in_use += r->bytes;
                    ++running;
                    r->t_start = now_ms();
                    batch.push_back(r);
                }
                for (Request *r : batch) r->batch_size = (int64_t)batch.size();
            }
            const int n = (int)batch.size();
            std::vector<int64_t> m(n), nn(n), lda(n);
            std::vector<const double *> A(n), b(n);
            std::vector<double *> x(n);
            std::vector<lsrn_options> opts(n);
            std::vector<lsrn_info> infos(n);
            for (int k = 0; k < n; ++k) {
                const Request &r = *batch[(size_t)k];
                m[k] = r.m; nn[k] = r.n; lda[k] = r.lda; A[k] = r.A; b[k] = r.b; x[k] = r.x;
                opts[k] = r.opt;
            }
            std::memset(infos.data(), 0, infos.size() * sizeof(lsrn_info));
            lsrn_status s = lsrn_solve_batch_opts(n, m.data(), nn.data(), A.data(), lda.data(), b.data(),
                                                  x.data(), opts.data(), infos.data(), st);
            if (hipStreamSynchronize(st) != hipSuccess && (s == LSRN_OK || s == LSRN_E_NOT_CONVERGED))
                s = LSRN_E_HIP;
            const std::string err = s != LSRN_OK ? lsrn_last_error() : std::string();
            {
                std::lock_guard<std::mutex> lk(mu);
                for (int k = 0; k < n; ++k) {
                    // not converged is per problem; any other failure is the batch's
                    lsrn_status sk = s;
                    if (s == LSRN_OK || s == LSRN_E_NOT_CONVERGED)
                        sk = infos[(size_t)k].converged ? LSRN_OK : LSRN_E_NOT_CONVERGED;
                    finish(batch[(size_t)k], sk, infos[(size_t)k],
                           sk == LSRN_E_NOT_CONVERGED ? "LSQR reached max_iter" : err);
                }
            }
            cv_work.notify_all();
            cv_done.notify_all();
        }
        lsrn::set_alloc_stream(nullptr);
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }

    static double now_ms() {
        using namespace std::chrono;
        return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
    }

    void worker() {
        (void)hipSetDevice(device);
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
        lsrn::set_alloc_stream(st);
        lsrn::set_graphs_allowed(false);
        for (;;) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    if (stopping && pending.empty()) return true;
                    if (pending.empty()) return false;
                    const size_t need = pending.front()->bytes;
                    return in_use + need <= budget || running == 0;
                });
                if (pending.empty()) break;
                r = pending.front();
                pending.pop_front();
                in_use += r->bytes;
                ++running;
                r->t_start = now_ms();
            }
            lsrn_info info;
            std::memset(&info, 0, sizeof(info));
            lsrn_status s;
            if (r->csr)
                s = lsrn_solve_csr(r->m, r->n, r->nnz, r->rowptr, r->colind, r->val, r->b, r->x, &r->opt,
                                   &info, st);
            else
                s = lsrn_solve_dense(r->m, r->n, r->A, r->lda, r->layout, r->b, r->x, &r->opt, &info,
                                     st);
            if (hipStreamSynchronize(st) != hipSuccess && s == LSRN_OK) s = LSRN_E_HIP;
            {
                std::lock_guard<std::mutex> lk(mu);
                finish(r, s, info, s != LSRN_OK ? std::string(lsrn_last_error()) : std::string());
            }
            cv_work.notify_all();
            cv_done.notify_all();
        }
        lsrn::set_alloc_stream(nullptr);
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
};

namespace {
thread_local std::string g_server_error;

lsrn_status server_fail(lsrn_status s, const char *msg) {
    g_server_error = msg;
    return s;
}
}  // namespace

extern "C" {

lsrn_status lsrn_server_create(int64_t hbm_budget_bytes, int32_t streams, lsrn_server **out) {
    if (!out || streams <= 0 || streams > 64 || hbm_budget_bytes <= 0)
        return server_fail(LSRN_E_INVALID, "need out != NULL, 0 < streams <= 64, budget > 0");
    *out = nullptr;
    try {
        auto *srv = new lsrn_server();
        if (hipGetDevice(&srv->device) != hipSuccess) {
            delete srv;
            return server_fail(LSRN_E_HIP, "no current HIP device");
        }
        srv->budget = (size_t)hbm_budget_bytes;
        for (int i = 0; i < streams; ++i) srv->workers.emplace_back([srv] { srv->worker(); });
        for (int i = 0; i < std::max(1, streams / 2); ++i) srv->workers.emplace_back([srv] { srv->batcher(); });
        *out = srv;
        return LSRN_OK;
    } catch (...) {
        return server_fail(LSRN_E_NOMEM, "could not start the server threads");
    }
}

static lsrn_status enqueue(lsrn_server *srv, std::unique_ptr<lsrn_server::Request> r, int64_t *ticket) {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return server_fail(LSRN_E_INVALID, "server is shutting down");
    r->id = srv->next_id++;
    r->t_submit = lsrn_server::now_ms();
    *ticket = r->id;
    (r->batch ? srv->pending_batch : srv->pending).push_back(r.get());
    srv->requests.emplace(r->id, std::move(r));
    // workers and batchers wait on this condition for different queues
    srv->cv_work.notify_all();
    return LSRN_OK;
}

lsrn_status lsrn_server_submit_dense(lsrn_server *srv, int64_t m, int64_t n, const double *A,
                                     int64_t lda, int32_t layout, const double *b, double *x,
                                     const lsrn_options *opt, int64_t *ticket) {
    if (!srv || !ticket || !A || !b || !x || m <= 0 || n <= 0)
        return server_fail(LSRN_E_INVALID, "bad request");
    auto r = std::make_unique<lsrn_server::Request>();
    r->m = m; r->n = n; r->A = A; r->lda = lda; r->layout = layout; r->b = b; r->x = x;
    if (opt) r->opt = *opt;
    else lsrn_default_options(&r->opt);
    // served solves never tune: timing launch shapes while other solves
    // share the device would be noise, and a new table entry would change
    // the summation order of later requests of the same shape
    r->opt.autotune = 0;
    r->batch = lsrn_server::batchable(*r);
    r->bytes = lsrn_workspace_bytes(m, n, layout, &r->opt);
    // the FP32 copy of A (the batched path computes in FP64 and makes none)
    if (r->opt.precision == LSRN_PREC_MIXED && !r->batch) r->bytes += (size_t)m * (size_t)n * sizeof(float);
    return enqueue(srv, std::move(r), ticket);
}

lsrn_status lsrn_server_submit_csr(lsrn_server *srv, int64_t m, int64_t n, int64_t nnz,
                                   const int64_t *rowptr, const int32_t *colind, const double *val,
                                   const double *b, double *x, const lsrn_options *opt,
                                   int64_t *ticket) {
    if (!srv || !ticket || !rowptr || !b || !x || m <= 0 || n <= 0 || nnz < 0)
        return server_fail(LSRN_E_INVALID, "bad request");
    auto r = std::make_unique<lsrn_server::Request>();
    r->csr = true;
    r->m = m; r->n = n; r->nnz = nnz; r->rowptr = rowptr; r->colind = colind; r->val = val;
    r->b = b; r->x = x;
    if (opt) r->opt = *opt;
    else lsrn_default_options(&r->opt);
    r->opt.autotune = 0;  // as for dense requests
    r->bytes = lsrn_workspace_bytes_csr(m, n, nnz, &r->opt);
    return enqueue(srv, std::move(r), ticket);
}

lsrn_status lsrn_server_wait(lsrn_server *srv, int64_t ticket, lsrn_info *info,
                             lsrn_server_timing *timing) {
    if (!srv) return server_fail(LSRN_E_INVALID, "NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->requests.find(ticket);
    if (it == srv->requests.end()) return server_fail(LSRN_E_INVALID, "unknown ticket");
    lsrn_server::Request *r = it->second.get();
    srv->cv_done.wait(lk, [&] { return r->done; });
    if (info) *info = r->info;
    if (timing) {
        timing->queue_ms = r->t_start - r->t_submit;
        timing->run_ms = r->t_done - r->t_start;
        timing->latency_ms = r->t_done - r->t_submit;
        timing->footprint_bytes = (int64_t)r->bytes;
        timing->batch_size = r->batch_size;
    }
    const lsrn_status s = r->status;
    if (s != LSRN_OK) g_server_error = r->error;
    srv->requests.erase(it);
    return s;
}

lsrn_status lsrn_server_stats(lsrn_server *srv, int64_t *pending, int64_t *running,
                              int64_t *bytes_in_use) {
    if (!srv) return server_fail(LSRN_E_INVALID, "NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (pending) *pending = (int64_t)(srv->pending.size() + srv->pending_batch.size());
    if (running) *running = srv->running;
    if (bytes_in_use) *bytes_in_use = (int64_t)srv->in_use;
    return LSRN_OK;
}

const char *lsrn_server_last_error(void) { return g_server_error.c_str(); }

void lsrn_server_destroy(lsrn_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->workers) t.join();
    delete srv;
}

}  // extern "C"
