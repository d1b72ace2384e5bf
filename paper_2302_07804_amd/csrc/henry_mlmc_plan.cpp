// henry_mlmc_plan.cpp -- host-side planning of an MLMC run (Sec. 3): the
// sample allocation of eq:M_ell and the convergence-rate fits and bias
// estimate behind the MSE split eq:MSE.  Plain host arithmetic; the solves
// and the level statistics run on the GPU (henry_solve_batch,
// mlmc_level_estimate).
#include <cmath>
#include <cstdint>

#include "henry.h"

namespace {

// Least-squares slope of y against x = first .. first+n-1.
double ls_slope(const double* y, int first, int n) {
    double sx = 0.0, sy = 0.0;
    for (int k = 0; k < n; ++k) { sx += first + k; sy += y[k]; }
    const double mx = sx / n, my = sy / n;
    double sxy = 0.0, sxx = 0.0;
    for (int k = 0; k < n; ++k) {
        const double dx = (first + k) - mx;
        sxy += dx * (y[k] - my);
        sxx += dx * dx;
    }
    return sxy / sxx;
}

}  // namespace

extern "C" {

int henry_mlmc_allocate(int32_t nlevels, const double* V, const double* s, double eps2, int64_t* m_out,
                        double* cost_out) {
    if (nlevels < 1 || !V || !s || !m_out || !(eps2 > 0.0) || !std::isfinite(eps2)) return HENRY_EINVAL;
    for (int l = 0; l < nlevels; ++l)
        if (!(V[l] >= 0.0) || !std::isfinite(V[l]) || !(s[l] > 0.0) || !std::isfinite(s[l])) return HENRY_EINVAL;
    // eq:M_ell: m_l = ceil(eps^-2 sqrt(V_l / s_l) sum_i sqrt(V_i s_i)), the
    // minimiser of the cost sum m_l s_l at estimator variance sum V_l / m_l = eps^2
    double tot = 0.0;
    for (int l = 0; l < nlevels; ++l) tot += std::sqrt(V[l] * s[l]);
    for (int l = 0; l < nlevels; ++l) {
        const double x = std::ceil(std::sqrt(V[l] / s[l]) * tot / eps2);
        if (!(x < 9.0e18)) return HENRY_EINVAL;
        m_out[l] = (int64_t)x;
    }
    if (cost_out) *cost_out = tot * tot / eps2;
    return HENRY_OK;
}

int henry_mlmc_rates(int32_t nlevels, const double* mean, const double* var, int32_t first, double* alpha,
                     double* beta, double* bias) {
    if (!mean || !var || !alpha || !beta || first < 0 || nlevels - first < 2 || nlevels > 64) return HENRY_EINVAL;
    double ym[64], yv[64];
    const int n = nlevels - first;
    for (int k = 0; k < n; ++k) {
        const double a = std::fabs(mean[first + k]), v = var[first + k];
        if (!(a > 0.0) || !(v > 0.0) || !std::isfinite(a) || !std::isfinite(v)) return HENRY_EINVAL;
        ym[k] = std::log2(a);
        yv[k] = std::log2(v);
    }
    // |E[Y_l]| ~ 2^(-alpha l), V_l ~ 2^(-beta l)
    *alpha = -ls_slope(ym, first, n);
    *beta = -ls_slope(yv, first, n);
    if (bias) {
        // the next level would add about |E[Y_L]| 2^-alpha, the ones after it a
        // geometric series: |E[g] - E[g_L]| ~ |E[Y_L]| / (2^alpha - 1)
        const double r = std::exp2(*alpha) - 1.0;
        *bias = r > 0.0 ? std::fabs(mean[nlevels - 1]) / r : INFINITY;
    }
    return HENRY_OK;
}

}  // extern "C"
