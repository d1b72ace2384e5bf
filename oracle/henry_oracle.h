/*
 * henry_oracle.h -- interface of the FP64 CPU oracle (test infrastructure).
 * Only the tests and the benchmark's CPU-baseline leg use it.  Return codes:
 * 0 ok, -1 invalid argument, -2 out of memory, -3 singular Jacobian,
 * -4 Newton did not converge in 30 iterations, -5 non-finite update.
 */
#ifndef HENRY_ORACLE_H
#define HENRY_ORACLE_H
#include <stdint.h>

typedef struct {
    double rho0, rho1, mu, g, D, phi0, k0, q_in, T; /* SI units */
} oracle_phys;

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void oracle_sample_xi(uint64_t seed, int32_t level, int64_t first, int64_t count, int32_t dim, double* out);
int oracle_fields_closed(const oracle_phys* ph, int32_t nx, int32_t ny, const double* xi,
                         double* phi, double* K, double* q);
int oracle_residual(const oracle_phys* ph, int32_t nx, int32_t ny, int32_t nsteps,
                    const double* phi, const double* K, double q,
                    const double* p, const double* c, const double* cn, double* Rp, double* Rc);
int oracle_jacobian_dense(const oracle_phys* ph, int32_t nx, int32_t ny, int32_t nsteps,
                          const double* phi, const double* K, double q,
                          const double* p, const double* c, const double* cn, double* J);
int oracle_band_solve_dense(int32_t n, int32_t kl, int32_t ku, const double* A, const double* b, double* x,
                            int32_t trans);
double oracle_qoi(const oracle_phys* ph, int32_t nx, int32_t ny, const double* phi, const double* c);
/* iters: NULL or [nsteps] Newton iterations per step; p_traj, c_traj: NULL
 * or [nsteps + 1][ny][nx] states from the initial one on. */
int oracle_solve(const oracle_phys* ph, int32_t nx, int32_t ny, int32_t nsteps,
                 const double* phi, const double* K, double q, const double* c0,
                 double* p_out, double* c_out, double* qoi, int32_t* iters,
                 double* p_traj, double* c_traj);
int oracle_adjoint(const oracle_phys* ph, int32_t nx, int32_t ny, int32_t nsteps,
                   const double* phi, const double* K, double q,
                   double* qoi, double* dq_dphi, double* dq_dK, double* dq_dq);
int oracle_tangent(const oracle_phys* ph, int32_t nx, int32_t ny, int32_t nsteps,
                   const double* phi, const double* K, double q,
                   const double* v_phi, const double* v_K, double v_q,
                   double* qoi, double* dqoi);
#endif
