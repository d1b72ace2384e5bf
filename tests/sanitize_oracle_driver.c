/* Driver for a sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host code only): every entry point on tiny
 * grids, including the degenerate 2x1 grid, trajectories, the adjoint and
 * the tangent, and the invalid-argument paths.  Exits 0 when every call
 * returns the expected code; the sanitizers abort on a memory error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "henry_oracle.h"

static int fails = 0;
#define EXPECT(cond)                                                       \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
            ++fails;                                                       \
        }                                                                  \
    } while (0)

static void grid_case(const oracle_phys* ph, int nx, int ny, int nsteps) {
    const int n = nx * ny;
    double xi[3];
    oracle_sample_xi(0, 0, 7, 1, 3, xi);
    double *phi = malloc(sizeof(double) * n), *K = malloc(sizeof(double) * n);
    double q = 0.0;
    EXPECT(oracle_fields_closed(ph, nx, ny, xi, phi, K, &q) == 0);
    double *p = malloc(sizeof(double) * n), *c = malloc(sizeof(double) * n), *cn = malloc(sizeof(double) * n);
    double *Rp = malloc(sizeof(double) * n), *Rc = malloc(sizeof(double) * n);
    for (int k = 0; k < n; ++k) {
        const int j = k / nx;
        c[k] = 0.3 + 0.01 * (k % 7);
        cn[k] = 0.29;
        p[k] = 1000.0 * 9.81 * (1.0 - (j + 0.5) / ny);
    }
    EXPECT(oracle_residual(ph, nx, ny, nsteps, phi, K, q, p, c, cn, Rp, Rc) == 0);
    double* J = malloc(sizeof(double) * 4 * n * n);
    EXPECT(oracle_jacobian_dense(ph, nx, ny, nsteps, phi, K, q, p, c, cn, J) == 0);
    double *pout = malloc(sizeof(double) * n), *cout = malloc(sizeof(double) * n);
    double *ptraj = malloc(sizeof(double) * n * (nsteps + 1)), *ctraj = malloc(sizeof(double) * n * (nsteps + 1));
    double Q = 0.0;
    int32_t* iters = malloc(sizeof(int32_t) * nsteps);
    EXPECT(oracle_solve(ph, nx, ny, nsteps, phi, K, q, NULL, pout, cout, &Q, iters, ptraj, ctraj) == 0);
    EXPECT(isfinite(Q) && Q == oracle_qoi(ph, nx, ny, phi, cout));
    double *gphi = malloc(sizeof(double) * n), *gK = malloc(sizeof(double) * n), gq = 0.0, Qa = 0.0;
    EXPECT(oracle_adjoint(ph, nx, ny, nsteps, phi, K, q, &Qa, gphi, gK, &gq) == 0);
    double *vphi = malloc(sizeof(double) * n), *vK = malloc(sizeof(double) * n), Qt = 0.0, dQ = 0.0;
    for (int k = 0; k < n; ++k) { vphi[k] = 1e-3 * phi[k]; vK[k] = 1e-2 * K[k]; }
    EXPECT(oracle_tangent(ph, nx, ny, nsteps, phi, K, q, vphi, vK, 1e-7, &Qt, &dQ) == 0);
    /* invalid grids */
    EXPECT(oracle_residual(ph, nx + 1, ny, nsteps, phi, K, q, p, c, cn, Rp, Rc) != 0);
    EXPECT(oracle_solve(ph, nx, ny, 0, phi, K, q, NULL, pout, cout, &Q, iters, NULL, NULL) != 0);
    free(phi); free(K); free(p); free(c); free(cn); free(Rp); free(Rc); free(J);
    free(pout); free(cout); free(ptraj); free(ctraj); free(gphi); free(gK); free(vphi); free(vK); free(iters);
}

int main(void) {
    const oracle_phys ph = {1000.0, 1025.0, 1e-3, 9.81, 1.886e-5, 0.35, 1.0194e-9, 6.6e-5, 3.6e4};
    uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {0, 0}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    double xi[41 * 3];
    oracle_sample_xi(123, 4, (int64_t)1 << 33, 3, 41, xi);
    grid_case(&ph, 2, 1, 3);
    grid_case(&ph, 4, 2, 5);
    grid_case(&ph, 16, 8, 10);
    /* banded solve of a small diagonally dominant tridiagonal system (dense
     * storage), both ways */
    double A[6 * 6] = {0}, b[6], x[6];
    for (int i = 0; i < 6; ++i) {
        A[i * 6 + i] = 4.0;
        if (i > 0) A[i * 6 + i - 1] = -1.0;
        if (i < 5) A[i * 6 + i + 1] = -1.0;
        b[i] = 1.0 + i;
    }
    EXPECT(oracle_band_solve_dense(6, 1, 1, A, b, x, 0) == 0);
    EXPECT(oracle_band_solve_dense(6, 1, 1, A, b, x, 1) == 0);
    if (fails) return 1;
    printf("sanitized oracle: all calls as expected\n");
    return 0;
}
