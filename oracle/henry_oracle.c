/*
 * henry_oracle.c -- plain, slow, FP64 CPU oracle for the Henry saltwater
 * intrusion solves that the multilevel Monte Carlo method of
 * Litvinenko, Logashenko, Tempone, Vasilyeva, Wittum (arXiv 2302.07804)
 * runs once per random sample and per level.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; it exists so that the tests and the benchmark's CPU
 * baseline can check the GPU path against an independent implementation.
 * It shares no code, header, table or helper with the HIP sources.
 *
 * What it computes (all FP64, compiled with -ffp-contract=off):
 *   - the governing equations of Sec. 2.1 (fluid mass conservation
 *     e_cont_eq, salt transport e_tran_eq, Darcy's law e_Darcy_vel, the
 *     linear density law e_lin_density, diffusion tensor e_mol_diff, the
 *     boundary and initial conditions of Sec. 2.1 / Fig. 1a), discretised
 *     on a cell-centred finite-volume grid with donor-cell upwinding and
 *     implicit Euler with a fixed step (Sec. 2.3 fixes implicit Euler and a
 *     constant tau; the spatial scheme is the cell-centred reading, which
 *     is documented beside the design);
 *   - each implicit step solved by Newton's method (Sec. 2.3) with the exact
 *     Jacobian obtained from forward-mode dual numbers and a banded LU with
 *     partial pivoting written here;
 *   - the quantity of interest "salt mass in x < 1 at T";
 *   - the discrete adjoint and tangent-linear models of the time-stepping
 *     map (not in the paper: used to check the GPU adjoint);
 *   - the random-input model: porosity, permeability and recharge from
 *     xi ~ U[-1,1]^3 (Sec. 2.2 treats these three as the uncertain inputs;
 *     the closed forms are the workload's field definitions), with
 *     xi drawn by Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
 *
 * Layout conventions of every array argument: cell fields are [ny][nx]
 * row-major (x fastest), j = 0 is the bottom row (y = -1 + h/2), i = 0 the
 * left column (x = h/2).  Inside the banded solver the unknowns are
 * interleaved (p, c) per cell with y fastest, which gives half-bandwidth
 * 2*ny + 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "henry_oracle.h"

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as   */
/* 1, 2, 3", SC'11), written from its published definition.            */
/* ------------------------------------------------------------------ */
static void philox_round(uint32_t ctr[4], const uint32_t key[2])
{
    const uint64_t a = (uint64_t)0xD2511F53u * ctr[0];
    const uint64_t b = (uint64_t)0xCD9E8D57u * ctr[2];
    const uint32_t hi_a = (uint32_t)(a >> 32), lo_a = (uint32_t)a;
    const uint32_t hi_b = (uint32_t)(b >> 32), lo_b = (uint32_t)b;
    uint32_t out0 = hi_b ^ ctr[1] ^ key[0];
    uint32_t out1 = lo_b;
    uint32_t out2 = hi_a ^ ctr[3] ^ key[1];
    uint32_t out3 = lo_a;
    ctr[0] = out0; ctr[1] = out1; ctr[2] = out2; ctr[3] = out3;
}

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t ctr[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t key[2] = {key_in[0], key_in[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { key[0] += 0x9E3779B9u; key[1] += 0xBB67AE85u; }
        philox_round(ctr, key);
    }
    memcpy(out, ctr, sizeof(ctr));
}

/* xi for sample key (seed, level, index), component d, uniform on [-1,1).
 * One Philox block per pair of components: counter = (d/2, level, index
 * low word, index high word), key = (seed low word, seed high word).  The
 * component takes words (2e, 2e+1), e = d mod 2, as the low/high halves of a
 * 64-bit integer, keeps its top 53 bits x, and returns x*2^-52 - 1, which is
 * exact in FP64. */
void oracle_sample_xi(uint64_t seed, int32_t level, int64_t first, int64_t count, int32_t dim, double* out)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t s = 0; s < count; ++s) {
        const uint64_t idx = (uint64_t)(first + s);
        for (int32_t d = 0; d < dim; d += 2) {
            const uint32_t ctr[4] = {(uint32_t)(d / 2), (uint32_t)level, (uint32_t)idx, (uint32_t)(idx >> 32)};
            uint32_t w[4];
            oracle_philox4x32_10(ctr, key, w);
            for (int e = 0; e < 2 && d + e < dim; ++e) {
                const uint64_t word = ((uint64_t)w[2 * e + 1] << 32) | (uint64_t)w[2 * e];
                const uint64_t x = word >> 11;
                out[s * dim + d + e] = (double)x * 0x1p-52 - 1.0;
            }
        }
    }
}

/* Random fields of the workload at cell centres (point values):
 *   phi = phi0 (1 + 0.2 xi1 cos(pi x/2) cos(pi y)),
 *   K   = k0 exp(0.5 xi2 sin(pi x/2)),
 *   q   = q_in (1 + 0.2 xi3).
 * Porosity, permeability and recharge are the uncertain inputs of Sec. 2.2. */
int oracle_fields_closed(const oracle_phys* ph, int32_t nx, int32_t ny, const double* xi,
                         double* phi, double* K, double* q)
{
    if (nx <= 0 || ny <= 0 || nx != 2 * ny) return -1;
    const double h = 1.0 / ny;
    for (int j = 0; j < ny; ++j) {
        const double y = -1.0 + (j + 0.5) * h;
        for (int i = 0; i < nx; ++i) {
            const double x = (i + 0.5) * h;
            phi[j * nx + i] = ph->phi0 * (1.0 + 0.2 * xi[0] * cos(M_PI * x / 2.0) * cos(M_PI * y));
            K[j * nx + i] = ph->k0 * exp(0.5 * xi[1] * sin(M_PI * x / 2.0));
        }
    }
    *q = ph->q_in * (1.0 + 0.2 * xi[2]);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Forward-mode dual numbers with a fixed set of derivative slots.      */
/* ------------------------------------------------------------------ */
enum { S_PP = 0, S_CP, S_PQ, S_CQ, S_PHIP, S_PHIQ, S_KP, S_KQ, S_Q, S_CNP, NSLOT };

typedef struct { double v; double d[NSLOT]; } dn;

static dn dcst(double v) { dn r; r.v = v; memset(r.d, 0, sizeof(r.d)); return r; }
static dn dvar(double v, int slot) { dn r = dcst(v); r.d[slot] = 1.0; return r; }
static dn dadd(dn a, dn b) { for (int k = 0; k < NSLOT; ++k) a.d[k] += b.d[k]; a.v += b.v; return a; }
static dn dsub(dn a, dn b) { for (int k = 0; k < NSLOT; ++k) a.d[k] -= b.d[k]; a.v -= b.v; return a; }
static dn dscl(dn a, double s) { for (int k = 0; k < NSLOT; ++k) a.d[k] *= s; a.v *= s; return a; }
static dn dmul(dn a, dn b)
{
    dn r; r.v = a.v * b.v;
    for (int k = 0; k < NSLOT; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
static dn ddiv(dn a, dn b)
{
    dn r; r.v = a.v / b.v;
    for (int k = 0; k < NSLOT; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
    return r;
}

/* Density law e_lin_density: rho(c) = rho0 + (rho1 - rho0) c. */
static dn rho_of(const oracle_phys* ph, dn c) { return dadd(dcst(ph->rho0), dscl(c, ph->rho1 - ph->rho0)); }

/* ------------------------------------------------------------------ */
/* Discrete fluxes.  All fluxes are outward from cell P, per metre of  */
/* depth; the face length h over the centre distance h is 1 for        */
/* interior faces and 2 for boundary faces (half-cell distance).       */
/* ------------------------------------------------------------------ */

/* Interior face between P and its neighbour Q, either to the east
 * (vertical = 0) or to the north (vertical = 1).  Darcy's law
 * e_Darcy_vel with gravity (0, -g): the vertical flux carries the
 * buoyancy term rho_f g h.  Face values: harmonic K and phi, arithmetic
 * density.  Salt flux: donor-cell advection plus diffusion with the
 * tensor e_mol_diff, D_f = phi_f D. */
static void face_flux(const oracle_phys* ph, double h, int vertical,
                      dn pP, dn cP, dn pQ, dn cQ, dn phiP, dn phiQ, dn KP, dn KQ, dn* M, dn* F)
{
    dn rhof = dscl(dadd(rho_of(ph, cP), rho_of(ph, cQ)), 0.5);
    dn Kf = ddiv(dscl(dmul(KP, KQ), 2.0), dadd(KP, KQ));
    dn phif = ddiv(dscl(dmul(phiP, phiQ), 2.0), dadd(phiP, phiQ));
    dn lam = dscl(dmul(rhof, Kf), 1.0 / ph->mu);
    dn dif = dscl(dmul(rhof, phif), ph->D);
    dn dp = dsub(pQ, pP);
    if (vertical) dp = dadd(dp, dscl(rhof, ph->g * h));
    *M = dscl(dmul(lam, dp), -1.0);
    dn cup = (M->v >= 0.0) ? cP : cQ;
    *F = dsub(dmul(*M, cup), dmul(dif, dsub(cQ, cP)));
}

/* Right boundary x = 2: seawater, c = 1, p = -rho1 g y (Sec. 2.1). */
static void right_flux(const oracle_phys* ph, double yj, dn pP, dn cP, dn phiP, dn KP, dn* M, dn* F)
{
    dn rhoB = dscl(dadd(rho_of(ph, cP), dcst(ph->rho1)), 0.5);
    dn pB = dcst(-ph->rho1 * ph->g * yj);
    *M = dscl(dmul(dmul(rhoB, KP), dsub(pB, pP)), -2.0 / ph->mu);
    dn cup = (M->v >= 0.0) ? cP : dcst(1.0);
    dn dif = dscl(dmul(rhoB, phiP), 2.0 * ph->D);
    *F = dsub(dmul(*M, cup), dmul(dif, dsub(dcst(1.0), cP)));
}

/* Left boundary x = 0: prescribed inflow of fresh water, rho q . e_x =
 * rho0 q (Sec. 2.1), c = 0.  The inflow carries no salt; salt may
 * still diffuse across the face towards c = 0. */
static void left_flux(const oracle_phys* ph, double h, dn cP, dn phiP, dn qv, dn* M, dn* F)
{
    *M = dscl(qv, -ph->rho0 * h);
    dn rhoB = dscl(dadd(rho_of(ph, cP), dcst(ph->rho0)), 0.5);
    dn dif = dscl(dmul(rhoB, phiP), 2.0 * ph->D);
    *F = dmul(dif, cP); /* -2 rho_B phi_P D (0 - c_P) */
}

/* ------------------------------------------------------------------ */
/* Assembly.  One routine produces the residual and, on request, the    */
/* Jacobian (banded or dense), products with parameter derivatives, and */
/* the diagonal derivative with respect to the previous c.              */
/* ------------------------------------------------------------------ */
typedef struct {
    const oracle_phys* ph;
    int nx, ny;
    double h, tau;
    const double* phi; const double* K; double q;     /* [ny][nx] */
} prob_t;

typedef struct {
    double* R;          /* [2n] interleaved residual, band ordering     */
    /* banded Jacobian: row-major rows of width W, row r stores columns
     * r - kl ... r - kl + W - 1 */
    double* band; int kl, W;
    double* dense;      /* [2n][2n] or NULL                             */
    const double* lam;  /* adjoint weights [2n] for lam^T dR/dtheta     */
    double* g_phi; double* g_K; double* g_q;         /* [ny][nx], scalar */
    const double* v_phi; const double* v_K; double v_q; /* tangent dir  */
    double* dR_tl;      /* [2n] (dR/dtheta) v                           */
    double* dR_dcn;     /* [2n] diagonal dR/dc^{n-1}                    */
} sink_t;

static inline int uidx(const prob_t* pb, int i, int j, int v) { return 2 * (i * pb->ny + j) + v; }
static inline int fidx(const prob_t* pb, int i, int j) { return j * pb->nx + i; }

static void band_add(sink_t* s, int r, int col, double val)
{
    s->band[(size_t)r * s->W + (col - r + s->kl)] += val;
}

/* Scatter sign*V into residual row r.  P/Q are (i,j) cell coordinates; Q
 * may be absent (qi < 0). */
static void scatter(const prob_t* pb, sink_t* s, int r, double sign, const dn* V,
                    int pi, int pj, int qi, int qj)
{
    const int n2 = 2 * pb->nx * pb->ny;
    s->R[r] += sign * V->v;
    const int cols[4] = {uidx(pb, pi, pj, 0), uidx(pb, pi, pj, 1),
                         qi >= 0 ? uidx(pb, qi, qj, 0) : -1, qi >= 0 ? uidx(pb, qi, qj, 1) : -1};
    for (int k = 0; k < 4; ++k) {
        if (cols[k] < 0 || V->d[k] == 0.0) continue;
        if (s->band) band_add(s, r, cols[k], sign * V->d[k]);
        if (s->dense) s->dense[(size_t)r * n2 + cols[k]] += sign * V->d[k];
    }
    const int fp = fidx(pb, pi, pj), fq = qi >= 0 ? fidx(pb, qi, qj) : -1;
    if (s->lam) {
        const double w = s->lam[r] * sign;
        s->g_phi[fp] += w * V->d[S_PHIP];
        s->g_K[fp] += w * V->d[S_KP];
        if (fq >= 0) { s->g_phi[fq] += w * V->d[S_PHIQ]; s->g_K[fq] += w * V->d[S_KQ]; }
        *s->g_q += w * V->d[S_Q];
    }
    if (s->dR_tl) {
        double t = V->d[S_PHIP] * s->v_phi[fp] + V->d[S_KP] * s->v_K[fp] + V->d[S_Q] * s->v_q;
        if (fq >= 0) t += V->d[S_PHIQ] * s->v_phi[fq] + V->d[S_KQ] * s->v_K[fq];
        s->dR_tl[r] += sign * t;
    }
    if (s->dR_dcn) s->dR_dcn[r] += sign * V->d[S_CNP];
}

/* R^p_P = (h^2/tau) phi_P (rho(c_P) - rho(c^n_P)) + sum_f M_f   (e_cont_eq)
 * R^c_P = (h^2/tau) phi_P (rho(c_P) c_P - rho(c^n_P) c^n_P) + sum_f F_f
 *                                                            (e_tran_eq) */
static void assemble(const prob_t* pb, const double* p, const double* c, const double* cn, sink_t* s)
{
    const oracle_phys* ph = pb->ph;
    const int nx = pb->nx, ny = pb->ny;
    const double h = pb->h, acc = h * h / pb->tau;
    for (int i = 0; i < nx; ++i) {
        for (int j = 0; j < ny; ++j) {
            const int f = fidx(pb, i, j);
            dn pP = dvar(p[f], S_PP), cP = dvar(c[f], S_CP);
            dn phiP = dvar(pb->phi[f], S_PHIP), KP = dvar(pb->K[f], S_KP);
            dn cnP = dvar(cn[f], S_CNP);
            /* accumulation */
            dn rP = rho_of(ph, cP), rN = rho_of(ph, cnP);
            dn Ap = dscl(dmul(phiP, dsub(rP, rN)), acc);
            dn Ac = dscl(dmul(phiP, dsub(dmul(rP, cP), dmul(rN, cnP))), acc);
            scatter(pb, s, uidx(pb, i, j, 0), 1.0, &Ap, i, j, -1, -1);
            scatter(pb, s, uidx(pb, i, j, 1), 1.0, &Ac, i, j, -1, -1);
            dn M, F;
            /* east face: interior or the seawater boundary */
            if (i + 1 < nx) {
                const int g = fidx(pb, i + 1, j);
                face_flux(ph, h, 0, pP, cP, dvar(p[g], S_PQ), dvar(c[g], S_CQ), phiP,
                          dvar(pb->phi[g], S_PHIQ), KP, dvar(pb->K[g], S_KQ), &M, &F);
                scatter(pb, s, uidx(pb, i, j, 0), 1.0, &M, i, j, i + 1, j);
                scatter(pb, s, uidx(pb, i, j, 1), 1.0, &F, i, j, i + 1, j);
                /* the same face seen from Q: flux leaves Q with opposite
                 * sign; derivative slots P/Q keep referring to (i,j) and
                 * (i+1,j) */
                scatter(pb, s, uidx(pb, i + 1, j, 0), -1.0, &M, i, j, i + 1, j);
                scatter(pb, s, uidx(pb, i + 1, j, 1), -1.0, &F, i, j, i + 1, j);
            } else {
                const double yj = -1.0 + (j + 0.5) * h;
                right_flux(ph, yj, pP, cP, phiP, KP, &M, &F);
                scatter(pb, s, uidx(pb, i, j, 0), 1.0, &M, i, j, -1, -1);
                scatter(pb, s, uidx(pb, i, j, 1), 1.0, &F, i, j, -1, -1);
            }
            /* north face: interior or the impermeable top (no flux) */
            if (j + 1 < ny) {
                const int g = fidx(pb, i, j + 1);
                face_flux(ph, h, 1, pP, cP, dvar(p[g], S_PQ), dvar(c[g], S_CQ), phiP,
                          dvar(pb->phi[g], S_PHIQ), KP, dvar(pb->K[g], S_KQ), &M, &F);
                scatter(pb, s, uidx(pb, i, j, 0), 1.0, &M, i, j, i, j + 1);
                scatter(pb, s, uidx(pb, i, j, 1), 1.0, &F, i, j, i, j + 1);
                scatter(pb, s, uidx(pb, i, j + 1, 0), -1.0, &M, i, j, i, j + 1);
                scatter(pb, s, uidx(pb, i, j + 1, 1), -1.0, &F, i, j, i, j + 1);
            }
            /* west boundary: recharge; bottom face: impermeable (no flux) */
            if (i == 0) {
                left_flux(ph, h, cP, phiP, dvar(pb->q, S_Q), &M, &F);
                scatter(pb, s, uidx(pb, i, j, 0), 1.0, &M, i, j, -1, -1);
                scatter(pb, s, uidx(pb, i, j, 1), 1.0, &F, i, j, -1, -1);
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Banded LU with partial pivoting (row interchanges interleaved with   */
/* elimination).  Row r holds columns r-kl .. r-kl+W-1, W = 2kl+ku+1.  */
/* ------------------------------------------------------------------ */
static inline double* bat(double* B, int W, int kl, int r, int col) { return &B[(size_t)r * W + (col - r + kl)]; }

static int band_lu(double* B, int n, int kl, int ku, int* piv)
{
    const int W = 2 * kl + ku + 1;
    for (int k = 0; k < n; ++k) {
        const int last = (k + kl < n - 1) ? k + kl : n - 1;
        int pr = k; double best = fabs(*bat(B, W, kl, k, k));
        for (int r = k + 1; r <= last; ++r) {
            const double a = fabs(*bat(B, W, kl, r, k));
            if (a > best) { best = a; pr = r; }
        }
        piv[k] = pr;
        if (best == 0.0) return -1;
        const int cend = (k + kl + ku < n - 1) ? k + kl + ku : n - 1;
        if (pr != k)
            for (int col = k; col <= cend; ++col) {
                double t = *bat(B, W, kl, k, col);
                *bat(B, W, kl, k, col) = *bat(B, W, kl, pr, col);
                *bat(B, W, kl, pr, col) = t;
            }
        const double dkk = *bat(B, W, kl, k, k);
        for (int r = k + 1; r <= last; ++r) {
            double* lrk = bat(B, W, kl, r, k);
            if (*lrk == 0.0) continue;
            const double l = *lrk / dkk;
            *lrk = l;
            for (int col = k + 1; col <= cend; ++col) *bat(B, W, kl, r, col) -= l * *bat(B, W, kl, k, col);
        }
    }
    return 0;
}

/* Solve A x = b in place (trans = 0) or A^T x = b (trans = 1). */
static void band_solve(double* B, int n, int kl, int ku, const int* piv, double* b, int trans)
{
    const int W = 2 * kl + ku + 1, uw = kl + ku;
    if (!trans) {
        for (int k = 0; k < n; ++k) {
            if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
            const int last = (k + kl < n - 1) ? k + kl : n - 1;
            for (int r = k + 1; r <= last; ++r) b[r] -= *bat(B, W, kl, r, k) * b[k];
        }
        for (int r = n - 1; r >= 0; --r) {
            double acc = b[r];
            const int cend = (r + uw < n - 1) ? r + uw : n - 1;
            for (int col = r + 1; col <= cend; ++col) acc -= *bat(B, W, kl, r, col) * b[col];
            b[r] = acc / *bat(B, W, kl, r, r);
        }
    } else {
        /* U^T y = b */
        for (int r = 0; r < n; ++r) {
            double acc = b[r];
            const int c0 = (r - uw > 0) ? r - uw : 0;
            for (int k = c0; k < r; ++k) acc -= *bat(B, W, kl, k, r) * b[k];
            b[r] = acc / *bat(B, W, kl, r, r);
        }
        /* then the transposed unit-lower factors and interchanges, last first */
        for (int k = n - 1; k >= 0; --k) {
            const int last = (k + kl < n - 1) ? k + kl : n - 1;
            double acc = b[k];
            for (int r = k + 1; r <= last; ++r) acc -= *bat(B, W, kl, r, k) * b[r];
            b[k] = acc;
            if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
        }
    }
}

/* Test hook: factor a dense matrix restricted to its band and solve. */
int oracle_band_solve_dense(int32_t n, int32_t kl, int32_t ku, const double* A, const double* b, double* x, int32_t trans)
{
    const int W = 2 * kl + ku + 1;
    double* B = calloc((size_t)n * W, sizeof(double));
    int* piv = malloc(sizeof(int) * n);
    if (!B || !piv) { free(B); free(piv); return -2; }
    for (int r = 0; r < n; ++r)
        for (int col = r - kl; col <= r + ku; ++col)
            if (col >= 0 && col < n) *bat(B, W, kl, r, col) = A[(size_t)r * n + col];
    int rc = band_lu(B, n, kl, ku, piv);
    if (rc == 0) {
        memcpy(x, b, sizeof(double) * n);
        band_solve(B, n, kl, ku, piv, x, trans);
    }
    free(B); free(piv);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Public single-evaluation entry points (tests).                        */
/* ------------------------------------------------------------------ */
static int check_prob(const oracle_phys* ph, int nx, int ny, int nsteps)
{
    if (!ph || nx <= 0 || ny <= 0 || nx != 2 * ny || nsteps <= 0) return -1;
    return 0;
}

static void set_prob(prob_t* pb, const oracle_phys* ph, int nx, int ny, int nsteps,
                     const double* phi, const double* K, double q)
{
    pb->ph = ph; pb->nx = nx; pb->ny = ny; pb->h = 1.0 / ny; pb->tau = ph->T / nsteps;
    pb->phi = phi; pb->K = K; pb->q = q;
}

int oracle_residual(const oracle_phys* ph, int32_t nx, int32_t ny, int32_t nsteps,
                    const double* phi, const double* K, double q,
                    const double* p, const double* c, const double* cn, double* Rp, double* Rc)
{
    if (check_prob(ph, nx, ny, nsteps)) return -1;
    prob_t pb; set_prob(&pb, ph, nx, ny, nsteps, phi, K, q);
    const int n = nx * ny;
    double* R = calloc((size_t)2 * n, sizeof(double));
    if (!R) return -2;
    sink_t s; memset(&s, 0, sizeof(s)); s.R = R;
    assemble(&pb, p, c, cn, &s);
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            Rp[j * nx + i] = R[uidx(&pb, i, j, 0)];
            Rc[j * nx + i] = R[uidx(&pb, i, j, 1)];
        }
    free(R);
    return 0;
}

/* Dense Jacobian dR/du, rows/cols in the interleaved y-fastest ordering
 * u = 2*(i*ny + j) + {0: p, 1: c}. */
int oracle_jacobian_dense(const oracle_phys* ph, int32_t nx, int32_t ny, int32_t nsteps,
                          const double* phi, const double* K, double q,
                          const double* p, const double* c, const double* cn, double* J)
{
    if (check_prob(ph, nx, ny, nsteps)) return -1;
    prob_t pb; set_prob(&pb, ph, nx, ny, nsteps, phi, K, q);
    const int n2 = 2 * nx * ny;
    double* R = calloc((size_t)n2, sizeof(double));
    if (!R) return -2;
    memset(J, 0, sizeof(double) * (size_t)n2 * n2);
    sink_t s; memset(&s, 0, sizeof(s)); s.R = R; s.dense = J;
    assemble(&pb, p, c, cn, &s);
    free(R);
    return 0;
}

/* Quantity of interest: salt mass in x < 1, Q = h^2 sum phi rho(c) c. */
static double qoi_of(const prob_t* pb, const double* c)
{
    const oracle_phys* ph = pb->ph;
    double Q = 0.0;
    for (int j = 0; j < pb->ny; ++j)
        for (int i = 0; i < pb->nx / 2; ++i) {
            const int f = fidx(pb, i, j);
            const double rho = ph->rho0 + (ph->rho1 - ph->rho0) * c[f];
            Q += pb->phi[f] * rho * c[f];
        }
    return Q * pb->h * pb->h;
}

double oracle_qoi(const oracle_phys* ph, int32_t nx, int32_t ny, const double* phi, const double* c)
{
    prob_t pb; set_prob(&pb, ph, nx, ny, 1, phi, phi, 0.0);
    return qoi_of(&pb, c);
}

/* ------------------------------------------------------------------ */
/* Newton time stepping (Sec. 2.3: implicit Euler, fixed tau, Newton).  */
/* ------------------------------------------------------------------ */
typedef struct {
    prob_t pb;
    int n, n2, kl, ku, W;
    double *R, *B, *dx;
    int* piv;
} work_t;

static int work_init(work_t* w, const prob_t* pb)
{
    w->pb = *pb;
    w->n = pb->nx * pb->ny; w->n2 = 2 * w->n;
    w->kl = 2 * pb->ny + 1; w->ku = w->kl; w->W = 2 * w->kl + w->ku + 1;
    w->R = calloc((size_t)w->n2, sizeof(double));
    w->dx = calloc((size_t)w->n2, sizeof(double));
    w->B = calloc((size_t)w->n2 * w->W, sizeof(double));
    w->piv = malloc(sizeof(int) * (size_t)w->n2);
    return (w->R && w->dx && w->B && w->piv) ? 0 : -2;
}
static void work_free(work_t* w) { free(w->R); free(w->dx); free(w->B); free(w->piv); }

/* Assemble R and the banded J at (p, c; cn) and LU-factor J. */
static int factor_at(work_t* w, const double* p, const double* c, const double* cn)
{
    memset(w->R, 0, sizeof(double) * w->n2);
    memset(w->B, 0, sizeof(double) * (size_t)w->n2 * w->W);
    sink_t s; memset(&s, 0, sizeof(s));
    s.R = w->R; s.band = w->B; s.kl = w->kl; s.W = w->W;
    assemble(&w->pb, p, c, cn, &s);
    return band_lu(w->B, w->n2, w->kl, w->ku, w->piv);
}

/* One implicit step: Newton from the current (p, c) until the corrections
 * fall below 1e-13 in c and 1e-13 rho1 g in p, then one more iteration. */
static int newton_step(work_t* w, double* p, double* c, const double* cn, int* iters)
{
    const prob_t* pb = &w->pb;
    const double ptol = 1e-13 * pb->ph->rho1 * pb->ph->g, ctol = 1e-13;
    int extra = 0, it;
    double last_dp = INFINITY, last_dc = INFINITY;
    for (it = 0; it < 30; ++it) {
        if (factor_at(w, p, c, cn)) return -3;
        for (int k = 0; k < w->n2; ++k) w->dx[k] = -w->R[k];
        band_solve(w->B, w->n2, w->kl, w->ku, w->piv, w->dx, 0);
        double mdp = 0.0, mdc = 0.0;
        for (int i = 0; i < pb->nx; ++i)
            for (int j = 0; j < pb->ny; ++j) {
                const int f = fidx(pb, i, j);
                const double dp = w->dx[uidx(pb, i, j, 0)], dc = w->dx[uidx(pb, i, j, 1)];
                p[f] += dp; c[f] += dc;
                if (fabs(dp) > mdp) mdp = fabs(dp);
                if (fabs(dc) > mdc) mdc = fabs(dc);
            }
        if (!isfinite(mdp) || !isfinite(mdc)) return -5;
        last_dp = mdp; last_dc = mdc;
        if (extra) { ++it; break; }
        if (mdc <= ctol && mdp <= ptol) extra = 1;
    }
    if (iters) *iters = it;
    if (!extra) {
        /* rounding floor: accept corrections a hundred times the target */
        if (last_dc <= 100 * ctol && last_dp <= 100 * ptol) return 0;
        return -4;
    }
    return 0;
}

int oracle_solve(const oracle_phys* ph, int32_t nx, int32_t ny, int32_t nsteps,
                 const double* phi, const double* K, double q, const double* c0,
                 double* p_out, double* c_out, double* qoi, int32_t* iters,
                 double* p_traj, double* c_traj)
{
    if (check_prob(ph, nx, ny, nsteps)) return -1;
    prob_t pb; set_prob(&pb, ph, nx, ny, nsteps, phi, K, q);
    work_t w;
    if (work_init(&w, &pb)) { work_free(&w); return -2; }
    const int n = nx * ny;
    double* cn = malloc(sizeof(double) * n);
    if (!cn) { work_free(&w); return -2; }
    /* initial state: c = 0 (Sec. 2.1); p only seeds Newton: fresh hydrostatic */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double y = -1.0 + (j + 0.5) * pb.h;
            p_out[j * nx + i] = -ph->rho0 * ph->g * y;
            c_out[j * nx + i] = c0 ? c0[j * nx + i] : 0.0;
        }
    if (c_traj) memcpy(c_traj, c_out, sizeof(double) * n);
    if (p_traj) memcpy(p_traj, p_out, sizeof(double) * n);
    int rc = 0;
    for (int s = 0; s < nsteps && rc == 0; ++s) {
        memcpy(cn, c_out, sizeof(double) * n);
        int it = 0;
        rc = newton_step(&w, p_out, c_out, cn, &it);
        if (iters) iters[s] = it;
        if (c_traj) memcpy(c_traj + (size_t)(s + 1) * n, c_out, sizeof(double) * n);
        if (p_traj) memcpy(p_traj + (size_t)(s + 1) * n, p_out, sizeof(double) * n);
    }
    if (qoi) *qoi = qoi_of(&pb, c_out);
    free(cn);
    work_free(&w);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Discrete adjoint and tangent-linear models of the step map.           */
/* R^n(u^n, c^{n-1}; theta) = 0, n = 1..N, Q = Q(c^N; phi).               */
/*   (J^N)^T lam^N = (dQ/du^N)^T,                                         */
/*   (J^n)^T lam^n = -(dR^{n+1}/dc^n)^T lam^{n+1},                        */
/*   dQ/dtheta = dQ/dtheta|_explicit - sum_n (lam^n)^T dR^n/dtheta.       */
/* theta = (phi per cell, K per cell, q).                                 */
/* ------------------------------------------------------------------ */
int oracle_adjoint(const oracle_phys* ph, int32_t nx, int32_t ny, int32_t nsteps,
                   const double* phi, const double* K, double q,
                   double* qoi, double* dq_dphi, double* dq_dK, double* dq_dq)
{
    if (check_prob(ph, nx, ny, nsteps)) return -1;
    const int n = nx * ny;
    double* pt = malloc(sizeof(double) * (size_t)(nsteps + 1) * n);
    double* ct = malloc(sizeof(double) * (size_t)(nsteps + 1) * n);
    double* pf = malloc(sizeof(double) * n);
    double* cf = malloc(sizeof(double) * n);
    if (!pt || !ct || !pf || !cf) { free(pt); free(ct); free(pf); free(cf); return -2; }
    int rc = oracle_solve(ph, nx, ny, nsteps, phi, K, q, NULL, pf, cf, qoi, NULL, pt, ct);
    if (rc) { free(pt); free(ct); free(pf); free(cf); return rc; }

    prob_t pb; set_prob(&pb, ph, nx, ny, nsteps, phi, K, q);
    work_t w;
    if (work_init(&w, &pb)) { work_free(&w); free(pt); free(ct); free(pf); free(cf); return -2; }
    double* lam = calloc((size_t)w.n2, sizeof(double));
    double* dcn = calloc((size_t)w.n2, sizeof(double));
    double* scratchR = calloc((size_t)w.n2, sizeof(double));
    memset(dq_dphi, 0, sizeof(double) * n);
    memset(dq_dK, 0, sizeof(double) * n);
    *dq_dq = 0.0;
    /* explicit dependence of Q on phi and on c^N */
    const double h2 = pb.h * pb.h;
    const double* cN = ct + (size_t)nsteps * n;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx / 2; ++i) {
            const int f = j * nx + i;
            const double rho = ph->rho0 + (ph->rho1 - ph->rho0) * cN[f];
            dq_dphi[f] += h2 * rho * cN[f];
            lam[uidx(&pb, i, j, 1)] = h2 * phi[f] * (ph->rho0 + 2.0 * (ph->rho1 - ph->rho0) * cN[f]);
        }
    for (int s = nsteps; s >= 1; --s) {
        const double* ps = pt + (size_t)s * n;
        const double* cs = ct + (size_t)s * n;
        const double* cprev = ct + (size_t)(s - 1) * n;
        if (factor_at(&w, ps, cs, cprev)) { rc = -3; break; }
        band_solve(w.B, w.n2, w.kl, w.ku, w.piv, lam, 1);
        /* gradient contribution and the coupling to the previous step */
        memset(dcn, 0, sizeof(double) * w.n2);
        sink_t sk; memset(&sk, 0, sizeof(sk));
        memset(scratchR, 0, sizeof(double) * w.n2);
        sk.R = scratchR; sk.lam = lam; sk.g_phi = dq_dphi; sk.g_K = dq_dK; sk.g_q = dq_dq;
        sk.dR_dcn = dcn;
        /* accumulate -lam^T dR/dtheta: negate lam temporarily */
        for (int k = 0; k < w.n2; ++k) lam[k] = -lam[k];
        assemble(&pb, ps, cs, cprev, &sk);
        for (int k = 0; k < w.n2; ++k) lam[k] = -lam[k];
        /* rhs for step s-1: -(dR^s/dc^{s-1})^T lam^s, diagonal per cell */
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j) {
                const int up = uidx(&pb, i, j, 0), uc = uidx(&pb, i, j, 1);
                const double r = -(dcn[up] * lam[up] + dcn[uc] * lam[uc]);
                lam[up] = 0.0;
                lam[uc] = r;
            }
    }
    free(lam); free(dcn); free(scratchR);
    work_free(&w);
    free(pt); free(ct); free(pf); free(cf);
    return rc;
}

int oracle_tangent(const oracle_phys* ph, int32_t nx, int32_t ny, int32_t nsteps,
                   const double* phi, const double* K, double q,
                   const double* v_phi, const double* v_K, double v_q,
                   double* qoi, double* dqoi)
{
    if (check_prob(ph, nx, ny, nsteps)) return -1;
    const int n = nx * ny;
    double* pt = malloc(sizeof(double) * (size_t)(nsteps + 1) * n);
    double* ct = malloc(sizeof(double) * (size_t)(nsteps + 1) * n);
    double* pf = malloc(sizeof(double) * n);
    double* cf = malloc(sizeof(double) * n);
    if (!pt || !ct || !pf || !cf) { free(pt); free(ct); free(pf); free(cf); return -2; }
    int rc = oracle_solve(ph, nx, ny, nsteps, phi, K, q, NULL, pf, cf, qoi, NULL, pt, ct);
    if (rc) { free(pt); free(ct); free(pf); free(cf); return rc; }
    prob_t pb; set_prob(&pb, ph, nx, ny, nsteps, phi, K, q);
    work_t w;
    if (work_init(&w, &pb)) { work_free(&w); free(pt); free(ct); free(pf); free(cf); return -2; }
    double* du = calloc((size_t)w.n2, sizeof(double));   /* du^{s-1}, then du^s */
    double* rhs = calloc((size_t)w.n2, sizeof(double));
    double* dcn = calloc((size_t)w.n2, sizeof(double));
    double* scratchR = calloc((size_t)w.n2, sizeof(double));
    for (int s = 1; s <= nsteps && rc == 0; ++s) {
        const double* ps = pt + (size_t)s * n;
        const double* cs = ct + (size_t)s * n;
        const double* cprev = ct + (size_t)(s - 1) * n;
        memset(rhs, 0, sizeof(double) * w.n2);
        memset(dcn, 0, sizeof(double) * w.n2);
        memset(scratchR, 0, sizeof(double) * w.n2);
        sink_t sk; memset(&sk, 0, sizeof(sk));
        sk.R = scratchR; sk.v_phi = v_phi; sk.v_K = v_K; sk.v_q = v_q; sk.dR_tl = rhs; sk.dR_dcn = dcn;
        assemble(&pb, ps, cs, cprev, &sk);
        /* J^s du^s = -(dR/dtheta v + dR/dc^{s-1} dc^{s-1}) */
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j) {
                const int up = uidx(&pb, i, j, 0), uc = uidx(&pb, i, j, 1);
                const double dcprev = du[uc];
                rhs[up] = -(rhs[up] + dcn[up] * dcprev);
                rhs[uc] = -(rhs[uc] + dcn[uc] * dcprev);
            }
        if (factor_at(&w, ps, cs, cprev)) { rc = -3; break; }
        band_solve(w.B, w.n2, w.kl, w.ku, w.piv, rhs, 0);
        memcpy(du, rhs, sizeof(double) * w.n2);
    }
    if (rc == 0) {
        const double h2 = pb.h * pb.h;
        const double* cN = ct + (size_t)nsteps * n;
        double d = 0.0;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx / 2; ++i) {
                const int f = j * nx + i;
                const double rho = ph->rho0 + (ph->rho1 - ph->rho0) * cN[f];
                d += h2 * rho * cN[f] * v_phi[f];
                d += h2 * phi[f] * (ph->rho0 + 2.0 * (ph->rho1 - ph->rho0) * cN[f]) * du[uidx(&pb, i, j, 1)];
            }
        *dqoi = d;
    }
    free(du); free(rhs); free(dcn); free(scratchR);
    work_free(&w);
    free(pt); free(ct); free(pf); free(cf);
    return rc;
}
