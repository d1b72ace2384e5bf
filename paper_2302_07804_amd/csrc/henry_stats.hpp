// henry_stats.hpp -- statistics of sampled time series on the device
// (Sec. 4: the quantiles of Figs. 4 and 6, the first-passage times of
// Figs. 5 and 7).  Deterministic: fixed-order sums, a bitonic sort in LDS,
// integer counts.
#pragma once

#include <hip/hip_runtime.h>

#include "henry_mlmc.hpp"

namespace henry {

constexpr int kMaxStatSamples = 8192;  // LDS sort buffer: 64 KiB of doubles
constexpr int kMaxQuantiles = 16;

struct Probs {
    double p[kMaxQuantiles];
    int n;
};

// Order for the sort: numbers ascending, NaN after every number.
__device__ inline bool after(double a, double b) { return a > b || (a != a && b == b); }

// Sum over a 256-thread block in a fixed order (four wavefronts).
__device__ inline double block_sum256(double v, double* red) {
    v = wave_sum_d(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// One 256-thread block per column v of x[nsamples][nvals] (minus x_sub, the
// same shape, when given: level differences of paired samples): mean, unbiased
// variance and the quantiles of Hyndman and Fan's type 7 (the linear
// interpolation between order statistics x_(lo) and x_(lo+1) at
// h = (n - 1) p).  P (a power of two >= nsamples) doubles of dynamic LDS.
__global__ void __launch_bounds__(256) sample_stats_kernel(const double* x, const double* x_sub, int nsamples,
                                                           int nvals, int P, Probs probs, double* mean, double* var,
                                                           double* q) {
    extern __shared__ double buf[];
    __shared__ double red[4];
    const int v = blockIdx.x;
    auto value = [&](int i) {
        double a = x[(size_t)i * nvals + v];
        if (x_sub) a -= x_sub[(size_t)i * nvals + v];
        return a;
    };
    // P == 0 (no quantiles): no sort buffer, the samples are read twice
    double s = 0.0;
    if (P > 0) {
        for (int i = threadIdx.x; i < P; i += blockDim.x) {
            const double a = i < nsamples ? value(i) : __builtin_nan("");
            buf[i] = a;
            if (i < nsamples) s += a;
        }
    } else {
        for (int i = threadIdx.x; i < nsamples; i += blockDim.x) s += value(i);
    }
    const double mu = block_sum256(s, red) / nsamples;
    double d2 = 0.0;
    for (int i = threadIdx.x; i < nsamples; i += blockDim.x) {
        const double d = (P > 0 ? buf[i] : value(i)) - mu;
        d2 += d * d;
    }
    const double s2 = block_sum256(d2, red);
    if (threadIdx.x == 0) {
        mean[v] = mu;
        var[v] = nsamples > 1 ? s2 / (nsamples - 1) : 0.0;
    }
    // bitonic sort of buf[0 .. P-1]
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            __syncthreads();
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const double a = buf[i], b = buf[ixj];
                    const bool up = (i & k) == 0;
                    if (up ? after(a, b) : after(b, a)) {
                        buf[i] = b;
                        buf[ixj] = a;
                    }
                }
            }
        }
    __syncthreads();
    if (threadIdx.x < probs.n) {
        const double h = (nsamples - 1) * probs.p[threadIdx.x];
        const int lo = (int)floor(h);
        const int hi = lo + 1 < nsamples ? lo + 1 : nsamples - 1;
        const double a = buf[lo], b = buf[hi];
        q[(size_t)threadIdx.x * nvals + v] = a + (h - lo) * (b - a);
    }
}

// First passage per sample: the first record k = 1..nrec whose value
// trace[s][k-1][col] (records of `stride` values) lies below (below != 0)
// or above the threshold; 0 if none does.
__global__ void first_passage_kernel(const double* trace, int nsamples, int nrec, int stride, int col, double thr,
                                     int below, int32_t* t_out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsamples) return;
    int t = 0;
    for (int k = 0; k < nrec; ++k) {
        const double a = trace[((size_t)s * nrec + k) * stride + col];
        if (below ? a < thr : a > thr) {
            t = k + 1;
            break;
        }
    }
    t_out[s] = t;
}

// hist[b] = #{s : t[s] == b}, b = 0..nrec: one thread per bin.
__global__ void passage_hist_kernel(const int32_t* t, int nsamples, int nrec, int32_t* hist) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nrec) return;
    int c = 0;
    for (int s = 0; s < nsamples; ++s) c += t[s] == b;
    hist[b] = c;
}

}  // namespace henry
