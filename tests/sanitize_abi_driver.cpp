// Driver for a sanitizer build of the C-ABI library's host code
// (AddressSanitizer and UndefinedBehaviorSanitizer on the host side only,
// no GPU needed): the host-side entry points with valid and invalid
// arguments, and the compute entry points' argument validation, which runs
// before anything touches a device.  Exits 0 when every call returns the
// expected code; the sanitizers abort on a memory error.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "henry.h"

static int fails = 0;
#define EXPECT(cond)                                                                          \
    do {                                                                                      \
        if (!(cond)) {                                                                        \
            std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
            ++fails;                                                                          \
        }                                                                                     \
    } while (0)

int main() {
    for (int code = -6; code <= 1; ++code) EXPECT(henry_strerror(code) != nullptr);
    henry_opts_t o;
    henry_opts_default(&o);
    henry_opts_default(nullptr);

    // sample generators
    std::vector<double> xi(17 * 3), xk(5 * 41);
    EXPECT(henry_sample_xi(7, 2, (int64_t)1 << 32, 17, 3, xi.data()) == HENRY_OK);
    EXPECT(henry_sample_xi(7, -1, 0, 17, 3, xi.data()) == HENRY_EINVAL);
    EXPECT(henry_sample_xi(7, 0, 0, 17, 3, nullptr) == HENRY_EINVAL);
    EXPECT(henry_sample_xi_kl(7, 6, 3, 5, xk.data()) == HENRY_OK);
    EXPECT(henry_sample_xi_kl(7, 6, 3, -1, xk.data()) == HENRY_EINVAL);

    // QMC points, up to the largest index the call accepts
    std::vector<double> hq(64 * 16);
    const double sh[3] = {0.25, 0.5, 0.999};
    EXPECT(henry_qmc_points(1, 64, 16, nullptr, hq.data()) == HENRY_OK);
    EXPECT(henry_qmc_points(((int64_t)1 << 31) - 64, 64, 3, sh, hq.data()) == HENRY_OK);
    EXPECT(henry_qmc_points(((int64_t)1 << 31) - 63, 64, 3, sh, hq.data()) == HENRY_EINVAL);
    EXPECT(henry_qmc_points(INT64_MAX, 1, 3, nullptr, hq.data()) == HENRY_EINVAL);
    EXPECT(henry_qmc_points(1, 4, 17, nullptr, hq.data()) == HENRY_EINVAL);

    // MLMC planning
    {
        const double V[4] = {1e-3, 1e-4, 2e-5, 4e-6}, s[4] = {1.0, 4.0, 16.0, 64.0};
        const double mean[4] = {0.5, 0.02, 0.01, 0.005};
        int64_t mm[4];
        double cost = 0.0, a = 0.0, bt = 0.0, bias = 0.0;
        EXPECT(henry_mlmc_allocate(4, V, s, 1e-6, mm, &cost) == HENRY_OK && mm[0] > mm[3]);
        EXPECT(henry_mlmc_allocate(4, V, s, 0.0, mm, &cost) == HENRY_EINVAL);
        EXPECT(henry_mlmc_rates(4, mean, V, 1, &a, &bt, &bias) == HENRY_OK && a > 0.0);
        EXPECT(henry_mlmc_rates(65, mean, V, 1, &a, &bt, &bias) == HENRY_EINVAL);
    }

    // KL basis on small grids, and its argument checks
    for (int ny : {1, 2, 8, 16}) {
        const int nx = 2 * ny;
        std::vector<double> lam(20), modes((size_t)20 * nx * ny);
        EXPECT(henry_kl_basis(nx, ny, 20, 0.3, 200, lam.data(), modes.data()) == HENRY_OK);
    }
    {
        std::vector<double> lam(20), modes(20 * 128);
        EXPECT(henry_kl_basis(16, 8, 0, 0.3, 200, lam.data(), modes.data()) == HENRY_EINVAL);
        EXPECT(henry_kl_basis(16, 9, 20, 0.3, 200, lam.data(), modes.data()) == HENRY_EINVAL);
        EXPECT(henry_kl_basis(16, 8, 20, -1.0, 200, lam.data(), modes.data()) == HENRY_EINVAL);
    }

    // workspace sizing and option validation
    std::vector<henry_grid_t> ok = {{16, 8, 50, 0}, {256, 128, 800, 0}, {1024, 512, 3200, 0}, {2, 1, 1, 0}};
    size_t bytes = 0;
    EXPECT(henry_workspace_bytes(nullptr, ok.data(), (int32_t)ok.size(), &o, &bytes) == HENRY_OK && bytes > 0);
    EXPECT(henry_workspace_bytes(nullptr, ok.data(), 0, &o, &bytes) == HENRY_OK);
    EXPECT(henry_workspace_bytes(nullptr, ok.data(), 1, &o, nullptr) == HENRY_EINVAL);
    for (henry_grid_t bad : {henry_grid_t{16, 16, 50, 0}, henry_grid_t{24, 12, 50, 0}, henry_grid_t{16, 8, 0, 0},
                             henry_grid_t{2048, 1024, 10, 0}, henry_grid_t{16, 8, 5, 1}})
        EXPECT(henry_workspace_bytes(nullptr, &bad, 1, &o, &bytes) == HENRY_EINVAL);
    henry_opts_t b = o;
    b.cluster = 3;
    EXPECT(henry_workspace_bytes(nullptr, ok.data(), 1, &b, &bytes) == HENRY_EINVAL);
    b = o;
    b.threads = 96;
    EXPECT(henry_workspace_bytes(nullptr, ok.data(), 1, &b, &bytes) == HENRY_EINVAL);
    EXPECT(henry_adjoint_workspace_bytes(nullptr, ok.data(), 2, &o, 20, &bytes) == HENRY_OK && bytes > 0);
    EXPECT(henry_adjoint_workspace_bytes(nullptr, ok.data(), 2, &o, 0, &bytes) == HENRY_EINVAL);

    // compute entry points reject a missing context before any device work
    double d = 0.0;
    int32_t st = 0;
    EXPECT(henry_solve_batch(nullptr, ok.data(), 1, HENRY_FIELD_CLOSED3, &d, nullptr, nullptr, nullptr, nullptr, &o,
                             &d, nullptr, &d, &st, nullptr, &d, 8, nullptr) == HENRY_EINVAL);
    EXPECT(henry_residual_batch(nullptr, ok.data(), 1, HENRY_FIELD_CLOSED3, &d, nullptr, nullptr, nullptr, &d, &d, &d,
                                &d, &d, &d, 8, nullptr) == HENRY_EINVAL);
    EXPECT(henry_adjoint_batch(nullptr, ok.data(), 1, HENRY_FIELD_CLOSED3, &d, nullptr, nullptr, nullptr, &o, 10, 1e-8,
                               10, &d, nullptr, nullptr, nullptr, nullptr, &st, nullptr, &d, 8, nullptr) == HENRY_EINVAL);
    EXPECT(henry_solve_batch_static(nullptr, ok.data(), 1, HENRY_FIELD_CLOSED3, &d, nullptr, nullptr, nullptr,
                                    nullptr, &o, &d, nullptr, &d, &st, nullptr, nullptr) == HENRY_EINVAL);
    int32_t m[2] = {4, 4};
    EXPECT(mlmc_level_estimate(nullptr, 1, ok.data(), m, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr) == HENRY_EINVAL);
    // time series and statistics: argument checks (an empty batch with a
    // placeholder handle passes them and returns before touching it)
    {
        henry_ctx* handle = reinterpret_cast<henry_ctx*>(&d);
        const double pts[4] = {1.6, -0.95, 1.85, -0.95}, far[2] = {2.5, -0.5}, probs[2] = {0.25, 0.75};
        EXPECT(henry_solve_batch_trace(handle, ok.data(), 0, HENRY_FIELD_CLOSED3, nullptr, nullptr, nullptr, nullptr,
                                       nullptr, &o, 10, 2, pts, 0.012178, &d, nullptr, nullptr, nullptr, nullptr,
                                       nullptr, nullptr, 0, nullptr) == HENRY_OK);
        EXPECT(henry_solve_batch_trace(handle, ok.data(), 0, HENRY_FIELD_CLOSED3, nullptr, nullptr, nullptr, nullptr,
                                       nullptr, &o, 10, 1, far, 0.012178, &d, nullptr, nullptr, nullptr, nullptr,
                                       nullptr, nullptr, 0, nullptr) == HENRY_EINVAL);
        EXPECT(henry_solve_batch_trace(nullptr, ok.data(), 1, HENRY_FIELD_CLOSED3, nullptr, nullptr, nullptr, nullptr,
                                       nullptr, &o, 51, 2, pts, 0.012178, &d, nullptr, nullptr, nullptr, nullptr,
                                       nullptr, nullptr, 0, nullptr) == HENRY_EINVAL);
        EXPECT(henry_sample_stats(handle, 8193, 3, &d, nullptr, 2, probs, &d, &d, &d, nullptr) == HENRY_EINVAL);
        EXPECT(henry_first_passage(handle, 10, 5, 3, 3, &d, 0.5, 1, &st, &st, nullptr) == HENRY_EINVAL);
        EXPECT(henry_level_smooth(nullptr, 16, 8, 0, HENRY_PREC_MIXED, 1, &d, &d, &d, &d, 4096, nullptr) ==
               HENRY_EINVAL);
        EXPECT(henry_level_smooth(handle, 16, 8, 3, HENRY_PREC_MIXED, 1, &d, &d, &d, &d, 4096, nullptr) ==
               HENRY_EINVAL);
        EXPECT(henry_level_smooth(handle, 16, 8, 0, HENRY_PREC_MIXED, 1, &d, &d, &d, &d, 64, nullptr) ==
               HENRY_ENOMEM);
    }
    // estimator sums: argument checks, and an empty set of quantities returns
    // before touching the (placeholder) context
    {
        henry_ctx* handle = reinterpret_cast<henry_ctx*>(&d);
        const double* mp[2] = {&d, &d};
        const int32_t mm2[2] = {4, 1}, m0[2] = {4, 0};
        const int64_t off[2] = {0, 3}, boff[2] = {0, -1};
        EXPECT(henry_mlmc_telescope(handle, 2, 0, mp, mp, mm2, off, &d, &d, nullptr) == HENRY_OK);
        EXPECT(henry_mlmc_telescope(nullptr, 2, 1, mp, mp, mm2, off, &d, &d, nullptr) == HENRY_EINVAL);
        EXPECT(henry_mlmc_telescope(handle, 17, 1, mp, mp, mm2, off, &d, &d, nullptr) == HENRY_EINVAL);
        EXPECT(henry_mlmc_telescope(handle, 2, 1, mp, mp, m0, off, &d, &d, nullptr) == HENRY_EINVAL);
        EXPECT(henry_mlmc_telescope(handle, 2, 1, mp, mp, mm2, boff, &d, &d, nullptr) == HENRY_EINVAL);
        EXPECT(henry_mlmc_telescope(handle, 2, 1, mp, mp, mm2, off, &d, nullptr, nullptr) == HENRY_EINVAL);
    }
    int32_t t = 0;
    EXPECT(henry_tune_set(nullptr, 16, HENRY_PREC_MIXED, 128, 0, -1) == HENRY_EINVAL);
    EXPECT(henry_tune_get(nullptr, 16, HENRY_PREC_MIXED, &t, nullptr, nullptr) == HENRY_EINVAL);
    EXPECT(henry_profile_last(nullptr, nullptr, 0, &t) == HENRY_EINVAL);
    EXPECT(henry_ctx_set_kl(nullptr, 16, 8, 0.3, 0.1, 0.5) == HENRY_EINVAL);

    // a context needs a device: without one (or with bad constants) creation fails cleanly
    henry_phys_t ph = {1000.0, 1025.0, 1e-3, 9.81, 1.886e-5, 0.35, 1.0194e-9, 6.6e-5, 3.6e4};
    henry_ctx* ctx = nullptr;
    EXPECT(henry_ctx_create(&ctx, nullptr, 0) == HENRY_EINVAL);
    henry_phys_t bad = ph;
    bad.mu = -1.0;
    EXPECT(henry_ctx_create(&ctx, &bad, 0) == HENRY_EINVAL);
    EXPECT(henry_ctx_create(&ctx, &ph, -1) == HENRY_EINVAL);
    henry_ctx_destroy(nullptr);

    if (fails) return 1;
    std::printf("sanitized C ABI host code: all calls as expected\n");
    return 0;
}
