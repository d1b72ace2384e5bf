// henry_kl.hpp -- host construction of Karhunen-Loeve bases for the random
// porosity and log-permeability fields (Sec. 2.2 of the paper treats both as
// uncertain inputs; the field model is a truncated KL expansion).
//
// Covariance: separable squared exponential on D = [0,2] x [-1,0],
//   C(x, x') = exp(-(x1-x1')^2 / (2 l^2)) exp(-(x2-x2')^2 / (2 l^2)).
// 1D eigenpairs by the Nystrom method: Gauss-Legendre nodes and weights
// (Newton iteration on the Legendre polynomial), the symmetric matrix
// W^1/2 C W^1/2 diagonalised by cyclic Jacobi rotations, eigenfunctions
// normalised to unit L2 norm under the quadrature and signed positive at
// the first node, evaluated at cell centres by Nystrom interpolation
//   e(x) = (1/lam) sum_j w_j C(x, x_j) e(x_j).
// 2D modes: products of 1D modes, ordered by decreasing eigenvalue (ties by
// (a + b, a)).  Everything here is FP64 host code, run once per grid.
#pragma once

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

namespace henry {
namespace kl {

// n-point Gauss-Legendre rule on [-1, 1].
inline void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double pn = (n == 1) ? z : p1, pm = (n == 1) ? 1.0 : p0;
            dp = n * (z * pn - pm) / (z * z - 1.0);
            const double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Cyclic Jacobi eigen-decomposition of the symmetric n x n matrix A (row
// major, overwritten).  Returns eigenvalues; V holds eigenvectors as
// columns.
inline std::vector<double> jacobi_eig(std::vector<double>& A, int n, std::vector<double>& V) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double a = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += a;
                if (i != j) off += a;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    std::vector<double> lam(n);
    for (int i = 0; i < n; ++i) lam[i] = A[(size_t)i * n + i];
    return lam;
}

// First `m` eigenpairs of the 1D kernel on [a, b], evaluated at `pts`.
inline void nystrom_1d(double a, double b, double l, int nq, int m, const std::vector<double>& pts,
                       std::vector<double>& lam_out, std::vector<double>& vals /* [m][pts] */) {
    std::vector<double> t, w;
    gauss_legendre(nq, t, w);
    std::vector<double> x(nq);
    for (int i = 0; i < nq; ++i) {
        x[i] = 0.5 * (b - a) * t[i] + 0.5 * (b + a);
        w[i] *= 0.5 * (b - a);
    }
    // The decomposition depends only on (a, b, l, nq): every grid shares it.
    static std::mutex mu;
    static std::map<std::tuple<double, double, double, int>, std::pair<std::vector<double>, std::vector<double>>>
        cache;
    std::vector<double> lam, V;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find({a, b, l, nq});
        if (it != cache.end()) {
            lam = it->second.first;
            V = it->second.second;
        }
    }
    if (lam.empty()) {
        std::vector<double> A((size_t)nq * nq);
        for (int i = 0; i < nq; ++i)
            for (int j = 0; j < nq; ++j) {
                const double d = x[i] - x[j];
                A[(size_t)i * nq + j] = std::sqrt(w[i]) * std::exp(-d * d / (2.0 * l * l)) * std::sqrt(w[j]);
            }
        lam = jacobi_eig(A, nq, V);
        std::lock_guard<std::mutex> lock(mu);
        cache[{a, b, l, nq}] = {lam, V};
    }
    std::vector<int> ord(nq);
    for (int i = 0; i < nq; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int p, int q) { return lam[p] > lam[q]; });
    lam_out.assign(m, 0.0);
    vals.assign((size_t)m * pts.size(), 0.0);
    for (int k = 0; k < m; ++k) {
        const int c = ord[k];
        std::vector<double> e(nq);
        for (int i = 0; i < nq; ++i) e[i] = V[(size_t)i * nq + c] / std::sqrt(w[i]);
        if (e[0] < 0)
            for (double& v : e) v = -v;
        lam_out[k] = lam[c];
        for (size_t p = 0; p < pts.size(); ++p) {
            double s = 0.0;
            for (int j = 0; j < nq; ++j) {
                const double d = pts[p] - x[j];
                s += w[j] * std::exp(-d * d / (2.0 * l * l)) * e[j];
            }
            vals[(size_t)k * pts.size() + p] = s / lam[c];
        }
    }
}

// nmodes 2D modes at the cell centres of an nx x ny grid (h = 1/ny):
// lam[nmodes], modes[nmodes][ny][nx].
inline void basis_2d(int nx, int ny, int nmodes, double l, int nq, std::vector<double>& lam,
                     std::vector<double>& modes) {
    const double h = 1.0 / ny;
    std::vector<double> xc(nx), yc(ny);
    for (int i = 0; i < nx; ++i) xc[i] = (i + 0.5) * h;
    for (int j = 0; j < ny; ++j) yc[j] = -1.0 + (j + 0.5) * h;
    std::vector<double> lx, ly, ex, ey;
    nystrom_1d(0.0, 2.0, l, nq, nmodes, xc, lx, ex);
    nystrom_1d(-1.0, 0.0, l, nq, nmodes, yc, ly, ey);
    std::vector<std::tuple<double, int, int, int>> cand;
    for (int a = 0; a < nmodes; ++a)
        for (int b = 0; b < nmodes; ++b) cand.emplace_back(lx[a] * ly[b], a + b, a, b);
    std::sort(cand.begin(), cand.end(), [](const auto& p, const auto& q) {
        if (std::get<0>(p) != std::get<0>(q)) return std::get<0>(p) > std::get<0>(q);
        if (std::get<1>(p) != std::get<1>(q)) return std::get<1>(p) < std::get<1>(q);
        return std::get<2>(p) < std::get<2>(q);
    });
    lam.assign(nmodes, 0.0);
    modes.assign((size_t)nmodes * nx * ny, 0.0);
    for (int k = 0; k < nmodes; ++k) {
        const auto& c = cand[k];
        lam[k] = std::get<0>(c);
        const int a = std::get<2>(c), b = std::get<3>(c);
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                modes[(size_t)k * nx * ny + (size_t)j * nx + i] = ey[(size_t)b * ny + j] * ex[(size_t)a * nx + i];
    }
}

}  // namespace kl
}  // namespace henry
