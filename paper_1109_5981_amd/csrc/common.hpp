// common.hpp -- shared host/device helpers of liblsrn (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>

#include "lsrn.h"

namespace lsrn {

// ----------------------------------------------------------------- errors

struct Error {
    lsrn_status status;
    std::string message;
};

[[noreturn]] void fail(lsrn_status st, const std::string &msg);
void hip_check(hipError_t e, const char *what);

#define LSRN_HIP(call) ::lsrn::hip_check((call), #call)
#define LSRN_REQUIRE(cond, msg)                              \
    do {                                                     \
        if (!(cond)) ::lsrn::fail(LSRN_E_INVALID, (msg));    \
    } while (0)

// Device buffer owned by the library.  Allocated with hipMalloc, or with
// stream-ordered hipMallocAsync on the thread's allocation stream when one
// is set (the serving runtime does, so that concurrent solves do not
// synchronise the device on every free).
class DevBuf {
  public:
    DevBuf() = default;
    explicit DevBuf(size_t bytes) { alloc(bytes); }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p_(o.p_), n_(o.n_), s_(o.s_), async_(o.async_) {
        o.p_ = nullptr;
        o.n_ = 0;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p_ = o.p_; n_ = o.n_; s_ = o.s_; async_ = o.async_;
            o.p_ = nullptr;
            o.n_ = 0;
        }
        return *this;
    }
    void alloc(size_t bytes);
    void release();
    template <class T> T *as() const { return static_cast<T *>(p_); }
    size_t bytes() const { return n_; }

  private:
    void *p_ = nullptr;
    size_t n_ = 0;
    hipStream_t s_ = nullptr;
    bool async_ = false;
};

// Stream for stream-ordered allocations of DevBufs made on this thread
// (nullptr: plain hipMalloc / hipFree).
void set_alloc_stream(hipStream_t s);
// True when the options pass the checks every solve makes (no throw).
bool options_valid(const lsrn_options &o);

// Whether this thread may capture iteration chunks into HIP graphs (the
// serving workers do not: a capture there can be invalidated by device-wide
// work other threads issue meanwhile).
void set_graphs_allowed(bool on);
bool graphs_allowed();

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Number of compute units of the current device (cached).
int device_cus();

// Event-based stage timer on a stream.
class StageTimer {
  public:
    explicit StageTimer(hipStream_t s);
    ~StageTimer();
    void mark();                 // record an event now
    double elapsed_ms(int i, int j);  // between marks i and j (synchronises)
    int count() const { return n_; }

  private:
    hipStream_t s_;
    hipEvent_t ev_[16];
    int n_ = 0;
};

// ---------------------------------------------------------- device helpers

// Sum over the 64 lanes of a wavefront by xor butterflies; every lane ends
// with the same value (each level adds the same two partial sums).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum for blockDim.x = NT (multiple of 64); `scratch` holds
// NT/64 doubles.  Every thread receives the same result (fixed order).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *scratch) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += scratch[w];
    return t;
}

// Double-double arithmetic (Dekker 1971; Knuth TAOCP vol. 2, 4.2.2):
// value = hi + lo with |lo| <= ulp(hi)/2.  The error-free transformations
// below rely on every product and sum being rounded on its own: each body
// turns floating-point contraction off, or the compiler (HIP contracts by
// default) would fuse a rounded product into a later sum and the error
// terms would no longer be exact.
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
#pragma clang fp contract(off)
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__device__ __forceinline__ dd quick_two_sum(double a, double b) {
#pragma clang fp contract(off)
    double s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
#pragma clang fp contract(off)
    double p = a * b;
    return {p, fma(a, b, -p)};
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

// a += x * y with x*y formed exactly.
__device__ __forceinline__ dd dd_fma(dd a, double x, double y) {
#pragma clang fp contract(off)
    return dd_add(a, two_prod(x, y));
}

// a += x * (y.hi + y.lo), the product kept to double-double accuracy.
__device__ __forceinline__ dd dd_fma_dd(dd a, double x, dd y) {
#pragma clang fp contract(off)
    dd p = two_prod(x, y.hi);
    p.lo = fma(x, y.lo, p.lo);
    return dd_add(a, p);
}

__device__ __forceinline__ dd dd_shfl_xor(dd v, int off) {
    return {__shfl_xor(v.hi, off, 64), __shfl_xor(v.lo, off, 64)};
}

// Double-double butterfly sum over a wavefront.  Partners add the same two
// values in swapped order; dd_add is not commutative bit-for-bit, so the
// lower lane's value always goes first to keep every lane identical.
__device__ __forceinline__ dd wave_sum_dd(dd v) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        dd o = dd_shfl_xor(v, off);
        v = (lane & off) ? dd_add(o, v) : dd_add(v, o);
    }
    return v;
}

}  // namespace lsrn
