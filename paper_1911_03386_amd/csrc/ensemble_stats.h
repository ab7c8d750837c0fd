// Device-side ensemble statistics of a coarsening-rate series, shared by the
// Cahn-Hilliard ensembles (ch_kernels.hip) and the droplet ensembles
// (dp_kernels.hip): the moments of eq. (mup), the window average of
// eq. (beta0_stats), the variance slope mu_2 = k t, and histograms of beta.
// Each caller's kernel supplies how beta_m(t_j) is read and how t_j is
// formed; everything here is deterministic except the histogram counts, which
// are integer atomics (order-independent).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ens_stats {

constexpr int kThreads = 256;   // block size of the statistics kernels
constexpr int kMaxMoments = 8;  // mu_1 .. mu_8

// fixed-order block sum of one double per thread (result valid in thread 0);
// sh holds kThreads / 64 doubles
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();  // sh free from any earlier use
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (tid == 0)
        for (int w = 0; w < kThreads / 64; ++w) r += sh[w];
    return r;
}

// One block per sample j (grid-strided over j < count): mu_1 = mean over
// the nm selected members of beta(i, j), then mu_p = mean of
// (beta - mu_1)^p, p = 2..pmax (two passes over the members, thread-strided
// sums in member order, then a fixed tree).  out[j * kMaxMoments + p - 1].
template <typename Beta>
__device__ void moments(const Beta& beta, int32_t nm, int64_t count, int32_t pmax, double* out)
{
    __shared__ double sh[kThreads / 64];
    __shared__ double mean_sh;
    for (int64_t j = blockIdx.x; j < count; j += gridDim.x) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nm; i += kThreads) s += beta(i, j);
        const double tot = block_sum(s, sh);
        if (threadIdx.x == 0) mean_sh = tot / nm;
        __syncthreads();
        const double mu1 = mean_sh;
        double acc[kMaxMoments];
#pragma unroll
        for (int p = 0; p < kMaxMoments; ++p) acc[p] = 0.0;
        for (int i = threadIdx.x; i < nm; i += kThreads) {
            const double d = beta(i, j) - mu1;
            double dp = d;
#pragma unroll
            for (int p = 1; p < kMaxMoments; ++p) {
                dp *= d;
                acc[p] += dp;
            }
        }
        double* o = out + j * kMaxMoments;
        if (threadIdx.x == 0) o[0] = mu1;
#pragma unroll
        for (int p = 1; p < kMaxMoments; ++p) {
            if (p >= pmax) break;  // uniform over the block
            const double r = block_sum(acc[p], sh);
            if (threadIdx.x == 0) o[p] = r / nm;
        }
        __syncthreads();  // mean_sh is rewritten for the next sample
    }
}

// Over the samples j0..j1 (one block): beta0 = time average of mu_1 by the
// trapezoid rule on the sample grid (spacing `step`, t_j = time(j)), and
// k = least-squares slope of mu_2 = k t through the origin; out = {beta0, k}.
template <typename Time>
__device__ void window(const double* mom, int64_t j0, int64_t j1, double step, const Time& time, double* out)
{
    __shared__ double sh[kThreads / 64];
    double a = 0.0, b = 0.0, c = 0.0;  // trapezoid sum, sum t mu2, sum t^2
    for (int64_t j = j0 + threadIdx.x; j <= j1; j += kThreads) {
        const double t = time(j);
        b += t * mom[j * kMaxMoments + 1];
        c += t * t;
        if (j < j1) a += 0.5 * step * (mom[j * kMaxMoments] + mom[(j + 1) * kMaxMoments]);
    }
    const double A = block_sum(a, sh);
    const double B = block_sum(b, sh);
    const double Cc = block_sum(c, sh);
    if (threadIdx.x == 0) {
        out[0] = (j1 > j0) ? A / ((double)(j1 - j0) * step) : __builtin_nan("");
        out[1] = (Cc > 0.0) ? B / Cc : __builtin_nan("");
    }
}

// Histogram of beta(i, j) over the nm members and the samples j0..j1 (grid
// stride): nbins equal bins of [lo, hi) in counts[1..nbins], counts[0] below
// lo, counts[nbins + 1] at or above hi, NaN not counted.  A value's bin is
// floor((beta - lo) nbins / (hi - lo)) in FP64, capped at nbins - 1.
template <typename Beta>
__device__ void histogram(const Beta& beta, int32_t nm, int64_t j0, int64_t j1, double lo, double hi,
                          int32_t nbins, unsigned long long* counts)
{
    const int64_t total = (j1 - j0 + 1) * (int64_t)nm;
    const double scale = nbins / (hi - lo);
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = j0 + it / nm;
        const int i = (int)(it - (j - j0) * nm);
        const double b = beta(i, j);
        if (isnan(b)) continue;
        int bin;
        if (b < lo)
            bin = 0;
        else if (b >= hi)
            bin = nbins + 1;
        else
            bin = 1 + min(nbins - 1, (int)((b - lo) * scale));
        atomicAdd(counts + bin, 1ull);
    }
}

}  // namespace ens_stats
