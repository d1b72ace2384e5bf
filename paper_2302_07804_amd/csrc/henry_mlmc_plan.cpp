// henry_mlmc_plan.cpp -- host-side planning of an MLMC run (Sec. 3): the
// sample allocation of eq:M_ell and the convergence-rate fits and bias
// estimate behind the MSE split eq:MSE; and the quasi-Monte Carlo points of
// the reference mean (abstract; Sec. 4, Fig. 11).  Plain host arithmetic; the solves
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

constexpr int kPrimes[16] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53};

// Radical inverse of k in base b: the base-b digits of k mirrored about the
// radix point.  The mirrored digits form an integer R over b^n (n = number of
// digits); for k < 2^31 and b <= 53 both are below 2^37, so the one division
// gives the correctly rounded value.
double radical_inverse(int64_t k, int b) {
    int64_t R = 0, D = 1;
    for (; k > 0; k /= b) {
        R = R * b + k % b;
        D *= b;
    }
    return (double)R / (double)D;
}

}  // namespace

extern "C" {

int henry_qmc_points(int64_t first, int64_t count, int32_t dim, const double* shift, double* xi) {
    if (first < 0 || count < 0 || count > (int64_t(1) << 31) - first || dim < 1 || dim > 16) return HENRY_EINVAL;
    if (count > 0 && !xi) return HENRY_EINVAL;
    if (shift)
        for (int d = 0; d < dim; ++d)
            if (!(shift[d] >= 0.0 && shift[d] < 1.0)) return HENRY_EINVAL;
    for (int64_t k = 0; k < count; ++k)
        for (int d = 0; d < dim; ++d) {
            double u = radical_inverse(first + k, kPrimes[d]);
            if (shift) {
                u += shift[d];
                if (u >= 1.0) u -= 1.0;  // the rotation is taken modulo 1
            }
            xi[k * dim + d] = 2.0 * u - 1.0;
        }
    return HENRY_OK;
}

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
