// Batch statistics of the tallies: mean of the normalised bin flux over
// all histories and the variance of the batch means (batches of contiguous
// histories; replica statistics as in Section 3.3), two-pass in FP64.
#include "k_common.hpp"

namespace mcdc {
namespace {

// Sum the X copies of every batch into copy 0, in a fixed order (one
// thread per batch and bin; the fold then reads one copy per batch).
__global__ void __launch_bounds__(256) k_sum_copies(double *S, int64_t n, int B, int X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * n) return;
    const int64_t b = t / n, j = t % n;
    double *base = S + b * X * n + j;
    double v = base[0];
    for (int x = 1; x < X; ++x) v += base[(int64_t)x * n];
    base[0] = v;
}

// Raw sum of batch b in bin j over the first X of its copies (fixed
// order); batches lie bstride elements apart, copies n apart (n = doubles
// per copy).
__device__ __forceinline__ double batch_sum(const double *S, int64_t bstride, int64_t n, int X, int b, int64_t j) {
    double v = 0.0;
    for (int x = 0; x < X; ++x) v += S[(int64_t)b * bstride + (int64_t)x * n + j];
    return v;
}

// One thread per tally bin j: S points at bin 0 of batch 0, copy 0 of
// [B][X][cstride] raw sums (X copies per batch); norm_j = dt_k * V_s, or
// V_s alone without time_norm (the flux at an instant).
__global__ void __launch_bounds__(256) k_fold(const double *__restrict__ S, int64_t ntally, int64_t cstride,
                                              int64_t bstride, int B, int X, uint64_t N, int G, int nts,
                                              const double *__restrict__ bin_norm,
                                              const double *__restrict__ time_norm,
                                              double *mean, double *var, double *raw) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntally) return;
    const int64_t k = j / ((int64_t)G * nts);
    const int s = (int)(j % nts);
    const double norm = (time_norm ? time_norm[k] : 1.0) * bin_norm[s];
    double total = 0.0;
    for (int b = 0; b < B; ++b) total += batch_sum(S, bstride, cstride, X, b, j);
    if (raw) raw[j] = total;
    if (mean) mean[j] = total / ((double)N * norm);
    if (var) {
        double mb_sum = 0.0;
        for (int b = 0; b < B; ++b) {
            const uint64_t nb = ((uint64_t)(b + 1) * N) / B - ((uint64_t)b * N) / B;
            mb_sum += batch_sum(S, bstride, cstride, X, b, j) / ((double)nb * norm);
        }
        const double mbar = mb_sum / B;
        double acc = 0.0;
        for (int b = 0; b < B; ++b) {
            const uint64_t nb = ((uint64_t)(b + 1) * N) / B - ((uint64_t)b * N) / B;
            const double d = batch_sum(S, bstride, cstride, X, b, j) / ((double)nb * norm) - mbar;
            acc += d * d;
        }
        var[j] = (B > 1) ? acc / ((double)B * (double)(B - 1)) : 0.0;
    }
}

// Leakage per face: same statistics with unit normalisation (L is
// [B][XL][n], XL copies per batch).
__global__ void k_fold_leak(const double *__restrict__ L, int n, int64_t bstride, int B, int XL, uint64_t N,
                            double *mean, double *var) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double total = 0.0, mb_sum = 0.0;
    for (int b = 0; b < B; ++b) {
        const uint64_t nb = ((uint64_t)(b + 1) * N) / B - ((uint64_t)b * N) / B;
        const double v = batch_sum(L, bstride, n, XL, b, j);
        total += v;
        mb_sum += v / (double)nb;
    }
    if (mean) mean[j] = total / (double)N;
    if (var) {
        const double mbar = mb_sum / B;
        double acc = 0.0;
        for (int b = 0; b < B; ++b) {
            const uint64_t nb = ((uint64_t)(b + 1) * N) / B - ((uint64_t)b * N) / B;
            const double d = batch_sum(L, bstride, n, XL, b, j) / (double)nb - mbar;
            acc += d * d;
        }
        var[j] = (B > 1) ? acc / ((double)B * (double)(B - 1)) : 0.0;
    }
}

// Sum x and x^2 of per-history detector scores (weight-window runs, where a
// history's score is assembled from several particles).
__global__ void __launch_bounds__(256) k_qoi_reduce(const double *__restrict__ q, uint64_t n,
                                                    double *sums) {
    __shared__ double red[2][256];
    double a = 0.0, b = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double v = q[i];
        a += v;
        b += v * v;
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dev::atomic_add_f64(sums, red[0][0]);
        dev::atomic_add_f64(sums + 1, red[1][0]);
    }
}

}  // namespace

int launch_fold(const DevProblem &P, double *S, double *L, int B, int X, int XL, uint64_t N,
                const double *bin_norm_dev, const double *time_norm_dev, double *mean,
                double *var, double *raw, double *leak_mean, double *leak_var,
                double *tc_mean, double *tc_var, hipStream_t st) {
    const int bs = 256;
    const int64_t s_stride = (int64_t)X * P.tstride, l_stride = (int64_t)XL * P.K * P.G * 6;
    if (!P.tc_on) tc_mean = tc_var = nullptr;
    if ((mean || var || raw || tc_mean || tc_var) && X > 1) {
        hipLaunchKernelGGL(k_sum_copies, dim3((unsigned)(((int64_t)B * P.tstride + bs - 1) / bs)), dim3(bs), 0,
                           st, S, P.tstride, B, X);
        X = 1;
    }
    if ((leak_mean || leak_var) && XL > 1) {
        const int64_t n = (int64_t)P.K * P.G * 6;
        hipLaunchKernelGGL(k_sum_copies, dim3((unsigned)(((int64_t)B * n + bs - 1) / bs)), dim3(bs), 0, st,
                           L, n, B, XL);
        XL = 1;
    }
    if (mean || var || raw) {
        const unsigned grid = (unsigned)((P.ntally + bs - 1) / bs);
        hipLaunchKernelGGL(k_fold, dim3(grid), dim3(bs), 0, st, S, P.ntally, P.tstride, s_stride, B, X, N, P.G,
                           P.nts, bin_norm_dev, time_norm_dev, mean, var, raw);
    }
    if (tc_mean || tc_var) {
        // the time-crossing part of each copy: flux at an instant, no dt
        const unsigned grid = (unsigned)((P.ntally + bs - 1) / bs);
        hipLaunchKernelGGL(k_fold, dim3(grid), dim3(bs), 0, st, (const double *)(S + P.ntally), P.ntally,
                           P.tstride, s_stride, B, X, N, P.G, P.nts, bin_norm_dev, (const double *)nullptr,
                           tc_mean, tc_var, (double *)nullptr);
    }
    if (leak_mean || leak_var) {
        const int n = P.K * P.G * 6;
        hipLaunchKernelGGL(k_fold_leak, dim3((n + bs - 1) / bs), dim3(bs), 0, st, L, n, l_stride, B, XL, N,
                           leak_mean, leak_var);
    }
    return (int)hipGetLastError();
}

int launch_qoi_reduce(const double *qoi_hist, uint64_t n, double *qoi_sums, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t grid = (n + 255) / 256;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_qoi_reduce, dim3((unsigned)grid), dim3(256), 0, st, qoi_hist, n,
                       qoi_sums);
    return (int)hipGetLastError();
}

}  // namespace mcdc

namespace mcdc {
namespace {

// Fill with zeros using vector stores (a kernel rather than a memset so a
// captured graph replays it safely).
__global__ void k_zero(uint4 *p, size_t n16, unsigned char *tail, size_t ntail) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t j = i; j < n16; j += stride) p[j] = make_uint4(0u, 0u, 0u, 0u);
    if (i < ntail) tail[i] = 0;
}

}  // namespace

int launch_zero(void *p, size_t bytes, hipStream_t st) {
    if (bytes == 0 || p == nullptr) return hipSuccess;
    const size_t n16 = bytes / 16;
    const size_t ntail = bytes - n16 * 16;
    size_t grid = (n16 + 255) / 256;
    if (grid > 4096) grid = 4096;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)grid), dim3(256), 0, st, (uint4 *)p, n16,
                       (unsigned char *)p + n16 * 16, ntail);
    return (int)hipGetLastError();
}

}  // namespace mcdc
