// henry_mlmc.hpp -- MLMC level-difference statistics on the device (Sec. 3:
// telescoping estimator eq:EgL / eq:A, Def. eq:Yell with g_{-1} = 0).
//
// Y_l = g_l - I g_{l-1} per sample, where I injects the coarse field
// (half the cells per direction) piecewise-constantly onto the fine grid.
// Mean and unbiased variance per cell: one wavefront per cell, lanes stride
// over the samples in a fixed order, then a butterfly of wavefront shuffles
// (deterministic).  Two passes: mean first, then sum of squared deviations.
#pragma once

#include <hip/hip_runtime.h>

namespace henry {

__device__ inline double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline double y_sample(const double* cf, const double* cc, int s, int cell, int ccell, int cells,
                                  int ccells) {
    double y = cf[(size_t)s * cells + cell];
    if (cc) y -= cc[(size_t)s * ccells + ccell];
    return y;
}

// grid: one wavefront per fine cell of this level.
__global__ void mlmc_field_stats_kernel(const double* cf, const double* cc, int m, int nx, int ny, double* mean,
                                        double* var) {
    const int lane = threadIdx.x & 63;
    const int cell = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int cells = nx * ny;
    if (cell >= cells) return;
    const int i = cell % nx, j = cell / nx;
    const int cnx = nx / 2;
    const int ccell = (j >> 1) * cnx + (i >> 1);
    const int ccells = cells / 4;
    double s = 0.0;
    for (int k = lane; k < m; k += 64) s += y_sample(cf, cc, k, cell, ccell, cells, ccells);
    const double mu = wave_sum_d(s) / m;
    double q = 0.0;
    for (int k = lane; k < m; k += 64) {
        const double dlt = y_sample(cf, cc, k, cell, ccell, cells, ccells) - mu;
        q += dlt * dlt;
    }
    const double v = wave_sum_d(q) / (m - 1);
    if (lane == 0) { mean[cell] = mu; var[cell] = v; }
}

// One wavefront per level: QoI difference statistics.
__global__ void mlmc_qoi_stats_kernel(const double* qf, const double* qc, int m, double* out2) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int k = lane; k < m; k += 64) s += qf[k] - (qc ? qc[k] : 0.0);
    const double mu = wave_sum_d(s) / m;
    double q = 0.0;
    for (int k = lane; k < m; k += 64) {
        const double dlt = qf[k] - (qc ? qc[k] : 0.0) - mu;
        q += dlt * dlt;
    }
    const double v = wave_sum_d(q) / (m - 1);
    if (lane == 0) { out2[0] = mu; out2[1] = v; }
}

struct LevelPtrs {
    const double* mean[16];
    const double* var[16];
    int m[16];
    int nx[16];
};

// Telescoped E[c] on the finest grid and the estimator variance (single
// block, fixed summation order): var_est[0] = sum_l V_l / m_l for the QoI
// (qstats holds V_l), var_est[1] = max over finest cells of the same sum for
// the field.
__global__ void mlmc_combine_kernel(LevelPtrs lp, int L, int nxL, int nyL, const double* qstats, double* Ec,
                                    double* var_est) {
    __shared__ double red[16];
    const int cells = nxL * nyL;
    double vmax = 0.0;
    for (int cell = threadIdx.x; cell < cells; cell += blockDim.x) {
        const int i = cell % nxL, j = cell / nxL;
        double e = 0.0, v = 0.0;
        for (int l = 0; l <= L; ++l) {
            const int sh = L - l;
            const int c = (j >> sh) * lp.nx[l] + (i >> sh);
            e += lp.mean[l][c];
            v += lp.var[l][c] / lp.m[l];
        }
        Ec[cell] = e;
        vmax = fmax(vmax, v);
    }
    for (int o = 32; o > 0; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = vmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = fmax(r, red[k]);
        double vq = 0.0;
        for (int l = 0; l <= L; ++l) vq += qstats[2 * l + 1] / lp.m[l];
        var_est[0] = vq;
        var_est[1] = r;
    }
}

// Partial sums of the telescoping estimator and of its variance over levels
// 0..l for every l (fixed order, FP64): one thread per quantity.
constexpr int kMaxTelescopeLevels = 16;
struct TelescopePtrs {
    const double* mean[kMaxTelescopeLevels];
    const double* var[kMaxTelescopeLevels];
    long long off[kMaxTelescopeLevels];
    double m[kMaxTelescopeLevels];
};

__global__ void mlmc_telescope_kernel(TelescopePtrs tp, int nlevels, int nvals, double* pmean, double* pvar) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvals) return;
    double e = 0.0, w = 0.0;
    for (int l = 0; l < nlevels; ++l) {
        e += tp.mean[l][tp.off[l] + v];
        pmean[(size_t)l * nvals + v] = e;
        if (tp.var[0]) {
            w += tp.var[l][tp.off[l] + v] / tp.m[l];
            pvar[(size_t)l * nvals + v] = w;
        }
    }
}

}  // namespace henry
