// rng.hip -- kernels that expose the Gaussian stream of the sketch (Alg. 1/2
// step 2) for inspection: raw Philox words and entries of G.
#include "internal.hpp"
#include "rng.hpp"

namespace lsrn {

__global__ void __launch_bounds__(256)
philox_words_kernel(uint64_t seed, int64_t row0, int64_t nrows, int64_t q0, int64_t nq,
                    uint32_t *__restrict__ out) {
    const int64_t total = nrows * nq;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / nq, j = t % nq;
        const Words4 w = philox_block(seed, (uint64_t)(row0 + r), (uint64_t)(q0 + j));
        uint4 v;
        v.x = w.w0; v.y = w.w1; v.z = w.w2; v.w = w.w3;
        reinterpret_cast<uint4 *>(out)[t] = v;
    }
}

__global__ void __launch_bounds__(256)
gauss_fill_kernel(uint64_t seed, int64_t row0, int64_t nrows, int64_t col0, int64_t ncols,
                  double *__restrict__ out) {
    const int64_t total = nrows * ncols;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / ncols, c = t % ncols;
        const uint64_t col = (uint64_t)(col0 + c);
        double g[4];
        gauss4(seed, (uint64_t)(row0 + r), col >> 2, g);
        out[t] = g[col & 3];
    }
}

static int grid_for(int64_t total) {
    const int64_t b = ceil_div(total, 256);
    return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

void launch_philox_words(uint64_t seed, int64_t row0, int64_t nrows, int64_t q0, int64_t nq,
                         uint32_t *out, hipStream_t s) {
    if (nrows <= 0 || nq <= 0) return;
    philox_words_kernel<<<grid_for(nrows * nq), 256, 0, s>>>(seed, row0, nrows, q0, nq, out);
    LSRN_HIP(hipGetLastError());
}

void launch_gauss_fill(uint64_t seed, int64_t row0, int64_t nrows, int64_t col0, int64_t ncols,
                       double *out, hipStream_t s) {
    if (nrows <= 0 || ncols <= 0) return;
    gauss_fill_kernel<<<grid_for(nrows * ncols), 256, 0, s>>>(seed, row0, nrows, col0, ncols, out);
    LSRN_HIP(hipGetLastError());
}

}  // namespace lsrn
