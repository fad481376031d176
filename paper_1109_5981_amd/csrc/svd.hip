// svd.hip -- economy SVD of the sketch and the preconditioner (Alg. 1/2
// steps 4-5).
//
// X (s x d, column-major) = Q R by Householder reflections; then one-sided
// (Hestenes) Jacobi orthogonalises the columns of Y = R^T: Y J = W.  Since
// R^T = W J^T, the columns of W are V_i sigma_i with V the right singular
// vectors of X, so N = V_r Sigma_r^{-1} = W_r Sigma_r^{-2} needs no
// accumulated rotations.  r counts sigma_i > rcond sigma_1.
#include <algorithm>
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

// Apply the nb reflectors of a panel, in order, to the trailing columns
// c >= p0 + nb: one column per workgroup, held in registers.
template <int NT, int EPT>
__global__ void __launch_bounds__(NT)
qr_apply_kernel(double *__restrict__ X, int64_t s, int64_t p0, int nb, const double *__restrict__ V,
                const double *__restrict__ beta) {
    __shared__ double scratch[NT / 64];
    const int64_t c = p0 + nb + blockIdx.x;
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

// Rotation of columns (wp, wq) of length len, one wavefront; returns 1 if
// the pair was rotated.  Golub & Van Loan Sec. 8.6 formula.
__device__ __forceinline__ int rotate_pair(double *wp, double *wq, int len, double tol) {
    const int lane = threadIdx.x & 63;
    double a = 0.0, b = 0.0, g = 0.0;
    for (int i = lane; i < len; i += 64) {
        const double x = wp[i], y = wq[i];
        a += x * x;
        b += y * y;
        g += x * y;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    g = wave_sum(g);
    if (g == 0.0 || fabs(g) <= tol * sqrt(a) * sqrt(b)) return 0;
    const double zeta = (b - a) / (2.0 * g);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
    const double c = 1.0 / sqrt(1.0 + t * t);
    const double sn = c * t;
    for (int i = lane; i < len; i += 64) {
        const double x = wp[i], y = wq[i];
        wp[i] = c * x - sn * y;
        wq[i] = sn * x + c * y;
    }
    return 1;
}

// Whole matrix in LDS (d <= 128), all sweeps in one workgroup.
__global__ void __launch_bounds__(1024)
jacobi_small_kernel(double *__restrict__ Y, int d, int max_sweeps, double tol,
                    int *__restrict__ sweeps_out) {
    extern __shared__ double W[];  // d * d, column p at W + p*d
    __shared__ int rot;
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const int nw = blockDim.x >> 6;
    for (int t = tid; t < d * d; t += blockDim.x) W[t] = Y[t];
    const int n = d + (d & 1);
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if (tid == 0) rot = 0;
        __syncthreads();
        int mine = 0;
        for (int round = 0; round < n - 1; ++round) {
            for (int k = wid; k < n / 2; k += nw) {
                int p, q;
                rr_pair(n, round, k, p, q);
                if (p < d && q < d) {
                    if (p > q) { const int tmp = p; p = q; q = tmp; }
                    mine += rotate_pair(W + p * d, W + q * d, d, tol);
                }
            }
            __syncthreads();
        }
        if (lane == 0 && mine) atomicAdd(&rot, mine);
        __syncthreads();
        const int total = rot;
        __syncthreads();
        if (total == 0) break;
    }
    for (int t = tid; t < d * d; t += blockDim.x) Y[t] = W[t];
    if (tid == 0) *sweeps_out = sweep + 1;
}

// One round of the block round robin: workgroup k takes column blocks
// (bi, bj) of width bw into LDS and rotates every pair among those 2 bw
// columns (round robin on 2 bw players), then writes them back.
__global__ void __launch_bounds__(256)
jacobi_block_round_kernel(double *__restrict__ Y, int d, int bw, int nblocks, int round,
                          double tol, int *__restrict__ rot_count) {
    extern __shared__ double W[];  // 2*bw columns of length d
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    int bi, bj;
    rr_pair(nblocks, round, blockIdx.x, bi, bj);
    const int nloc = 2 * bw;
    // load
    for (int cl = 0; cl < nloc; ++cl) {
        const int blk = cl < bw ? bi : bj;
        const int64_t col = (int64_t)blk * bw + (cl % bw);
        const double *src = Y + col * d;
        double *dst = W + (int64_t)cl * d;
        for (int i = tid; i < d; i += 256) dst[i] = src[i];
    }
    __syncthreads();
    int mine = 0;
    for (int sub = 0; sub < nloc - 1; ++sub) {
        for (int k = wid; k < nloc / 2; k += 4) {
            int p, q;
            rr_pair(nloc, sub, k, p, q);
            // keep the global column order inside a pair
            const int64_t gp = (int64_t)(p < bw ? bi : bj) * bw + (p % bw);
            const int64_t gq = (int64_t)(q < bw ? bi : bj) * bw + (q % bw);
            if (gp > gq) { const int tmp = p; p = q; q = tmp; }
            mine += rotate_pair(W + (int64_t)p * d, W + (int64_t)q * d, d, tol);
        }
        __syncthreads();
    }
    for (int cl = 0; cl < nloc; ++cl) {
        const int blk = cl < bw ? bi : bj;
        const int64_t col = (int64_t)blk * bw + (cl % bw);
        double *dst = Y + col * d;
        const double *src = W + (int64_t)cl * d;
        for (int i = tid; i < d; i += 256) dst[i] = src[i];
    }
    if (lane == 0 && mine) atomicAdd(rot_count, mine);
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

int grid1d(int64_t total) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(total, 256), 16384)); }

template <int NT, int EPT>
void launch_apply(double *X, int64_t s, int64_t p0, int nb, int64_t ncols, const double *V,
                  const double *beta, hipStream_t st) {
    qr_apply_kernel<NT, EPT><<<(unsigned)ncols, NT, 0, st>>>(X, s, p0, nb, V, beta);
}

size_t lds_limit() {
    static size_t lim = 0;
    if (!lim) {
        int dev = 0, v = 0;
        LSRN_HIP(hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        lim = (size_t)v;
    }
    return lim;
}

}  // namespace

size_t precond_workspace_bytes(int64_t s, int64_t d) {
    const int64_t dcols = round_up(d, 64) + 64;
    return sizeof(double) * ((size_t)s * QNB + QNB + (size_t)d * dcols + 2 * (size_t)d) +
           sizeof(int64_t) * (size_t)d + 64;
}

PrecondResult precond(int64_t s, int64_t d, double *X, double rcond, double *sigma, double *P,
                      hipStream_t st) {
    LSRN_REQUIRE(s >= d && d > 0, "precond: need s >= d > 0");
    PrecondResult res;

    // ---- Householder QR
    DevBuf Vb((size_t)s * QNB * sizeof(double)), betab(QNB * sizeof(double));
    for (int64_t p0 = 0; p0 < d; p0 += QNB) {
        const int nb = (int)std::min<int64_t>(QNB, d - p0);
        qr_panel_kernel<<<1, 1024, 0, st>>>(X, s, p0, nb, Vb.as<double>(), betab.as<double>());
        LSRN_HIP(hipGetLastError());
        const int64_t ncols = d - p0 - nb;
        if (ncols > 0) {
            const int64_t rows = s - p0;
            if (rows <= 256 * 4) launch_apply<256, 4>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            else if (rows <= 256 * 8) launch_apply<256, 8>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            else if (rows <= 256 * 16) launch_apply<256, 16>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            else if (rows <= 256 * 32) launch_apply<256, 32>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            else if (rows <= 1024 * 16) launch_apply<1024, 16>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            else if (rows <= 1024 * 40) launch_apply<1024, 40>(X, s, p0, nb, ncols, Vb.as<double>(), betab.as<double>(), st);
            else fail(LSRN_E_UNSUPPORTED, "precond: sketch has too many rows for the QR kernels");
            LSRN_HIP(hipGetLastError());
        }
    }

    // ---- Jacobi on Y = R^T
    const double tol = (double)d * DBL_EPSILON;
    const int max_sweeps = 60;
    const size_t lds = lds_limit();
    int bw = 1;
    while ((size_t)(4 * bw) * (size_t)d * sizeof(double) <= lds && bw < 8) bw *= 2;
    const bool small = (size_t)d * (size_t)d * sizeof(double) <= lds && d <= 128;
    int64_t nblocks = ceil_div(d, bw);
    nblocks += nblocks & 1;
    const int64_t dcols = small ? d : nblocks * bw;
    DevBuf Yb((size_t)d * (size_t)dcols * sizeof(double));
    double *Y = Yb.as<double>();
    r_to_y_kernel<<<grid1d(d * dcols), 256, 0, st>>>(X, s, d, dcols, Y);
    LSRN_HIP(hipGetLastError());

    DevBuf cnt(2 * sizeof(int));
    int *dcnt = cnt.as<int>();
    if (small) {
        const size_t bytes = (size_t)d * d * sizeof(double);
        if (bytes > 65536)
            LSRN_HIP(hipFuncSetAttribute((const void *)jacobi_small_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
        jacobi_small_kernel<<<1, 1024, bytes, st>>>(Y, (int)d, max_sweeps, tol, dcnt);
        LSRN_HIP(hipGetLastError());
        int sw = 0;
        LSRN_HIP(hipMemcpyAsync(&sw, dcnt, sizeof(int), hipMemcpyDeviceToHost, st));
        LSRN_HIP(hipStreamSynchronize(st));
        res.sweeps = sw;
    } else {
        const size_t bytes = (size_t)(2 * bw) * (size_t)d * sizeof(double);
        LSRN_REQUIRE(bytes <= lds, "precond: sketch too wide for the LDS Jacobi kernel");
        if (bytes > 65536)
            LSRN_HIP(hipFuncSetAttribute((const void *)jacobi_block_round_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
        int sweep = 0;
        for (; sweep < max_sweeps; ++sweep) {
            LSRN_HIP(hipMemsetAsync(dcnt, 0, sizeof(int), st));
            for (int round = 0; round < nblocks - 1; ++round) {
                jacobi_block_round_kernel<<<(unsigned)(nblocks / 2), 256, bytes, st>>>(
                    Y, (int)d, bw, (int)nblocks, round, tol, dcnt);
            }
            LSRN_HIP(hipGetLastError());
            int rot = 0;
            LSRN_HIP(hipMemcpyAsync(&rot, dcnt, sizeof(int), hipMemcpyDeviceToHost, st));
            LSRN_HIP(hipStreamSynchronize(st));
            if (rot == 0) break;
        }
        res.sweeps = sweep + 1;
    }

    // ---- singular values, order, rank, N
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
    return res;
}

}  // namespace lsrn
