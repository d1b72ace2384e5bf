/*
 * henry.h -- C ABI of the MI355X (gfx950) library for batched Henry
 * saltwater-intrusion solves, the deterministic kernel that the multilevel
 * Monte Carlo method of Litvinenko, Logashenko, Tempone, Vasilyeva and
 * Wittum (arXiv 2302.07804) runs once per random sample and per level.
 *
 * Problem (Sec. 2.1 of the paper): on D = [0,2] x [-1,0] m, fluid mass
 * conservation (e_cont_eq) and salt transport (e_tran_eq) with Darcy's law
 * (e_Darcy_vel), rho(c) = rho0 + (rho1 - rho0) c (e_lin_density), diffusion
 * phi D I (e_mol_diff); c = 0 at t = 0; right side x = 2: c = 1 and
 * p = -rho1 g y; left side x = 0: fresh-water inflow rho q . e_x = rho0 q;
 * top and bottom impermeable.  Porosity phi, permeability K and recharge q
 * are the uncertain inputs (Sec. 2.2).  Discretisation: cell-centred finite
 * volumes with donor-cell upwinding, harmonic face K and phi, arithmetic
 * face density, implicit Euler with fixed tau = T / nsteps (Sec. 2.3).
 *
 * Conventions for every call:
 *   - All array arguments marked "device" are device pointers on the
 *     context's GPU, owned and allocated by the caller; nothing here frees
 *     them.  Calls are asynchronous on `stream` (a hipStream_t; NULL = the
 *     null stream) and validate every host-side argument before anything is
 *     enqueued: on an error return nothing has been launched.
 *   - A cell field is [ny][nx] row-major (x fastest), row 0 at the bottom
 *     (y = -1 + h/2).  "Packed" per-solve fields are concatenated in solve
 *     order: solve k starts at element sum_{m<k} nx_m * ny_m.
 *   - Grids must satisfy nx == 2 * ny (square cells, h = 1/ny), ny a power
 *     of two with 1 <= ny <= 512 (the line solver keeps at most 16 rows of
 *     a line per lane, 64 lanes per line), nsteps >= 1.  One workgroup owns
 *     a solve, or a cluster of workgroups for grids above 2048 cells
 *     (henry_opts_t.cluster).
 *   - Return codes are the HENRY_* values below; no exception crosses the
 *     ABI.  A context is not thread-safe; use one per host thread.
 */
#ifndef HENRY_H
#define HENRY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HENRY_OK 0
#define HENRY_EINVAL (-1)      /* invalid argument; nothing launched          */
#define HENRY_ENOMEM (-2)      /* workspace too small / host allocation failed */
#define HENRY_EHIP (-3)        /* a HIP runtime call failed                    */
#define HENRY_ENOCONV (-4)     /* reported through status[]: see below         */
#define HENRY_ENONFINITE (-5)  /* reported through status[]                    */

/* Per-solve status values written to the device status[] array. */
#define HENRY_STATUS_OK 0
#define HENRY_STATUS_NOCONV 1      /* some step hit max_outer; integration went on */
#define HENRY_STATUS_NONFINITE 2   /* a residual became NaN/Inf; the solve stopped */
#define HENRY_STATUS_SYNC 3        /* the workgroups of a cluster did not meet at a
                                      barrier within opts.cluster_wait_us (10 s by
                                      default); the solve stopped                 */

/* Physical constants, SI units (Table 1 of the paper lists rho0, mu, D,
 * E[phi]; the workload fixes rho1, g, k0, q_in and T). */
typedef struct {
    double rho0, rho1, mu, g, D, phi0, k0, q_in, T;
} henry_phys_t;

/* One deterministic solve: grid and number of implicit Euler steps. */
typedef struct {
    int32_t nx, ny, nsteps, reserved; /* reserved must be 0 */
} henry_grid_t;

/* How the random inputs reach a solve (Sec. 2.2: porosity, permeability
 * and recharge are uncertain).
 *   CLOSED3:  xi[k][3] ~ U[-1,1]^3 per solve,
 *             phi = phi0 (1 + 0.2 xi1 cos(pi x/2) cos(pi y)),
 *             K = k0 exp(0.5 xi2 sin(pi x/2)), q = q_in (1 + 0.2 xi3),
 *             evaluated at cell centres.
 *   KL41:     xi[k][41]: truncated Karhunen-Loeve expansions (20 modes of a
 *             separable squared-exponential covariance, henry_ctx_set_kl)
 *             phi = phi0 (1 + s_phi Z_phi), log K = log k0 + s_K Z_K,
 *             Z_phi = sum_{k<20} sqrt(lam_k) e_k xi_k, Z_K with xi_{20+k},
 *             q = q_in (1 + 0.2 xi_41); every grid of the call needs a basis.
 *   EXPLICIT: the caller passes packed per-cell phi and log K and a
 *             per-solve recharge q[k] (m/s).
 *   TWOLAYER3: xi[k][3], the paper's own model (Sec. 4, eq:poro_2levels,
 *             eq:poro_2levels_C, e_perm_Kozeny_Carman):
 *             phi = phi0 (1 + 0.15 (xi2 cos(pi x/2) + xi2 sin(2 pi y)
 *                   + xi1 cos(2 pi x))) C0, C0 = 1 + 0.2 xi1 below
 *                   y = -0.75 and 1 - 0.2 xi1 above (a cell face for
 *                   ny >= 4; the cell centre decides),
 *             K = kappa phi^3 / (1 - phi^2), kappa = k0 (1 - phi0^2) / phi0^3
 *                   so that K(phi0) = k0,
 *             q = q_in (1 + 0.5 xi3).  phi stays within [0.44, 1.74] phi0,
 *             so the call needs phi0 < 1/1.74 (HENRY_EINVAL otherwise). */
#define HENRY_FIELD_CLOSED3 0
#define HENRY_FIELD_KL41 1
#define HENRY_FIELD_EXPLICIT 2
#define HENRY_FIELD_TWOLAYER3 3

/* Inner precision of the multigrid / line-relaxation preconditioner.  The
 * outer nonlinear residual, the state, the buoyancy term and every
 * reduction are FP64 in both modes. */
#define HENRY_PREC_FP64 0
#define HENRY_PREC_MIXED 1

typedef struct {
    int32_t prec;             /* HENRY_PREC_*                                   */
    int32_t max_outer;        /* defect-correction iterations per step (>= 1)   */
    double tol;               /* stop a step when max_P |R_P| tau/(h^2 phi_P rho0)
                                 <= tol for both the fluid and the salt equation */
    int32_t threads;          /* threads per solve-workgroup, a power of two:
                                 64..1024 with PREC_MIXED, 64..512 with
                                 PREC_FP64 and in henry_adjoint_batch (a tuned
                                 choice above 512 is clamped there); 0 = tuned
                                 choice                                          */
    int32_t steps_per_launch; /* 0 = whole time loop in one launch per grid
                                 group; k > 0 = launches of k global steps, all
                                 captured into one hipGraph and replayed        */
    int32_t profile;          /* 1 = time each grid group's launches with HIP
                                 events on the stream they run on; read with
                                 henry_profile_last                              */
    int32_t serial_groups;    /* 1 = run grid groups one after another on one
                                 stream instead of concurrently                  */
    int32_t cluster;          /* workgroups (CUs) sharing one solve of
                                 henry_solve_batch or henry_adjoint_batch: 1, 2,
                                 4 or 8; 0 = built-in choice (one per 8192 fine
                                 cells, at most 8, and at most 256 workgroups
                                 per grid group).  Grids of 2048 cells or fewer
                                 always use 1.  The fine levels are split over
                                 the cluster, the coarse ones run on its first
                                 workgroup; results are bitwise the same for
                                 every value.  The members synchronise through
                                 the solve's workspace; grid groups with
                                 clusters run one after another.                 */
    int32_t cluster_wait_us;  /* bound of one wait at a cluster barrier, in
                                 microseconds; 0 = 10 s.  A member that waits
                                 longer stops its cluster: the solve reports
                                 HENRY_STATUS_SYNC.                              */
    int32_t predictor;        /* start of each step's iteration, extrapolated
                                 through the last converged states: 1 = the
                                 interpolating polynomial through up to four;
                                 2 = the same, then the least-squares cubic
                                 through five once five are there (it
                                 amplifies the states' own errors, of the size
                                 of tol, less); 0 = built-in: 2 for solves of
                                 200 steps or more at tol >= 1e-8, else 1.
                                 The choice changes only the iteration count,
                                 not what a step converges to (within tol).      */
} henry_opts_t;

/* Timing of one grid group of the last henry_solve_batch call made with
 * opts.profile = 1 (complete once that call's work has finished). */
typedef struct {
    int32_t nx, ny, nsolves, launches;
    int64_t cell_steps;      /* sum over the group's solves of nx*ny*nsteps */
    double ms;               /* HIP-event time of the group's solve launches */
    int32_t threads, cluster; /* workgroup size and workgroups per solve used
                                 (0 in the one entry of a graph replay)      */
} henry_group_time_t;

typedef struct henry_ctx henry_ctx;

const char* henry_strerror(int code);

/* Create a context bound to HIP device `device` (the current device is
 * restored on return).  `phys` is copied. */
int henry_ctx_create(henry_ctx** out, const henry_phys_t* phys, int device);
void henry_ctx_destroy(henry_ctx* ctx);

/* Default options: mixed precision, max_outer 40, tol 1e-10, tuned threads,
 * one launch per grid group. */
void henry_opts_default(henry_opts_t* opts);

/* Counter-based sample generator (Philox4x32-10, Salmon et al. SC'11).
 * Host-side, writes count*dim doubles to out_host: component d of sample
 * `first + s` of stream (seed, level) is built from Philox block
 * counter = (d/2, level, index lo, index hi), key = (seed lo, seed hi):
 * words (2e, 2e+1), e = d mod 2, form a 64-bit integer whose top 53 bits x
 * give x * 2^-52 - 1 in [-1, 1).  Fine and coarse solves of one MLMC pair
 * share the key, so they see the same xi (eq:A, Sec. 3). */
int henry_sample_xi(uint64_t seed, int32_t level, int64_t first, int64_t count, int32_t dim,
                    double* out_host);

/* KL basis of the separable squared-exponential covariance
 * C = exp(-|x-x'|^2 / (2 corr_len^2)) on [0,2] x [-1,0] at the cell centres
 * of an nx x ny grid (host-only).  1D eigenpairs by the Nystrom method with
 * an nquad-point Gauss-Legendre rule, eigenfunctions of unit L2 norm signed
 * positive at the first node, interpolated by the Nystrom formula; 2D modes
 * are products ordered by decreasing eigenvalue (ties by (a+b, a)).
 * lambda_out [nmodes], modes_out [nmodes][ny][nx] (host). */
int henry_kl_basis(int32_t nx, int32_t ny, int32_t nmodes, double corr_len, int32_t nquad, double* lambda_out,
                   double* modes_out);

/* Build (200-point rule, 20 modes) and upload the KL basis used by
 * HENRY_FIELD_KL41 for nx x ny grids; sigma_phi is the relative standard
 * deviation of porosity, sigma_logk that of log K.  The context owns the
 * device copy. */
int henry_ctx_set_kl(henry_ctx* ctx, int32_t nx, int32_t ny, double corr_len, double sigma_phi,
                     double sigma_logk);

/* 41 coefficients per sample for HENRY_FIELD_KL41 (host-side): components
 * 2g, 2g+1 (g < 20) are Box-Muller normals from Philox block
 * counter = (100 + g, level, index lo, index hi), key = (seed lo, seed hi):
 * 53-bit integers x1 (words 0,1) and x2 (words 2,3), u1 = (x1 + 1) 2^-53,
 * u2 = x2 2^-53, r = sqrt(-2 ln u1), (r cos 2 pi u2, r sin 2 pi u2);
 * component 40 is uniform on [-1,1) from block (200, level, ...), words
 * (0,1), as in henry_sample_xi.  out_host [count][41]. */
int henry_sample_xi_kl(uint64_t seed, int32_t level, int64_t first, int64_t count, double* out_host);

/* The FP64 residual of each solve's discrete equations at a given state:
 * the cell-centred finite-volume form of the fluid and salt balances
 * (e_cont_eq, e_tran_eq with Darcy's law e_Darcy_vel, Sec. 2.1) after one
 * implicit Euler step of tau = T / nsteps (Sec. 2.3), per cell
 *   R^p = (h^2/tau) phi (rho(c) - rho(c^n)) + sum of the face mass fluxes out,
 *   R^c = (h^2/tau) phi (rho(c) c - rho(c^n) c^n) + sum of the face salt fluxes out
 * (kg/s per m of depth), the residual whose scaled max norm ends a step of
 * henry_solve_batch.
 *   solves, field, xi, phi, logk, qin: as henry_solve_batch
 *   p, c, cn  device packed FP64 [ny][nx] per solve: the state (p, c) and
 *             the previous time level c^n
 *   rp_out, rc_out  device packed FP64 residuals
 *   workspace, ws_bytes: at least henry_workspace_bytes(ctx, solves, nsolves,
 *             NULL, ...); its content is overwritten.
 * Errors: HENRY_EINVAL (bad grid, NULL pointer, missing KL basis),
 * HENRY_ENOMEM (ws_bytes too small), HENRY_EHIP. */
int henry_residual_batch(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field,
                         const double* xi, const double* phi, const double* logk, const double* qin,
                         const double* p, const double* c, const double* cn, double* rp_out, double* rc_out,
                         void* workspace, size_t ws_bytes, void* stream);

/* Workspace (device bytes) that henry_solve_batch needs for these solves. */
int henry_workspace_bytes(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves,
                          const henry_opts_t* opts, size_t* bytes_out);

/* Batched forward solves.  Every solve k integrates its own grid for
 * solves[k].nsteps implicit Euler steps to T; solves of different grids
 * and step counts share one call.
 *   solves   host [nsolves]
 *   field    HENRY_FIELD_*
 *   xi       device [nsolves][3] (CLOSED3, TWOLAYER3), [nsolves][41] (KL41),
 *            else ignored
 *   phi,logk device packed per-cell fields (EXPLICIT) else ignored
 *   qin      device [nsolves] recharge in m/s (EXPLICIT) else ignored
 *   c0       device packed initial salt mass fraction, or NULL for c = 0
 *   c_out    device packed c at T (FP64)
 *   p_out    device packed p at T (FP64), or NULL
 *   qoi_out  device [nsolves]: salt mass in x < 1 at T,
 *            Q = h^2 sum_{x_i < 1} phi rho(c) c  (kg per m of depth)
 *   status   device [nsolves] HENRY_STATUS_*
 *   iters    device [nsolves] total outer iterations over all steps, or NULL
 *   workspace, ws_bytes: device scratch of at least henry_workspace_bytes.
 * Errors: HENRY_EINVAL (bad grid, NULL required pointer, opts out of range),
 * HENRY_ENOMEM (ws_bytes too small), HENRY_EHIP. */
int henry_solve_batch(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field,
                      const double* xi, const double* phi, const double* logk, const double* qin,
                      const double* c0, const henry_opts_t* opts, double* c_out, double* p_out,
                      double* qoi_out, int32_t* status, int32_t* iters, void* workspace, size_t ws_bytes,
                      void* stream);

/* Allocation-free variant of henry_solve_batch, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, results and
 * kernels as henry_solve_batch, without the workspace: the solves' state
 * (the workspace henry_workspace_bytes sizes) lives in a library-owned
 * static device buffer of HENRY_STATIC_SCRATCH_BYTES (128 MiB), one per
 * GPU, held by every GPU the library runs on until the process ends.  The
 * call allocates nothing (no hipMalloc, hipFree, hipHostMalloc, graph or
 * event): the descriptor table reaches the device as kernel arguments.
 * Limits and errors, besides those of henry_solve_batch:
 *   - henry_workspace_bytes(solves, opts) > HENRY_STATIC_SCRATCH_BYTES:
 *     HENRY_ENOMEM, nothing launched (split the batch);
 *   - opts->steps_per_launch != 0 or opts->profile != 0: HENRY_EINVAL;
 *   - the buffer's address could not be looked up at context creation:
 *     HENRY_EHIP.
 * Every call on one GPU uses that GPU's one buffer, and the buffer keeps
 * the last call's contents (each call re-initialises what it reads).
 * Calls that overlap in time on one GPU (on two streams, from two contexts
 * or host threads) race on it and corrupt each other's solves: order them,
 * e.g. on one stream. */
#define HENRY_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
int henry_solve_batch_static(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field,
                             const double* xi, const double* phi, const double* logk, const double* qin,
                             const double* c0, const henry_opts_t* opts, double* c_out, double* p_out,
                             double* qoi_out, int32_t* status, int32_t* iters, void* stream);

/* Batched forward solves that also record a time series of each solve
 * (Sec. 4: the fresh-water integral eq:integral_fw and c at the points of
 * eq:12points over time, the inputs of the paper's Figs. 4-7).  Every
 * argument of henry_solve_batch keeps its meaning; in addition:
 *   nrec     records per solve, 1 <= nrec <= every solve's nsteps: record k
 *            (k = 1..nrec) holds the state after step ceil(k nsteps / nrec),
 *            the first step at or after t = k T / nrec
 *   npts     0..16 points; points: host [npts][2] (x, y) in the closed
 *            domain [0,2] x [-1,0]
 *   c_fresh  threshold of the fresh-water indicator (the paper: 0.012178)
 *   trace_out device [nsolves][nrec][1 + npts]: per record the fresh-water
 *            area Q_FW = h^2 #{cells: c <= c_fresh} (m^2; 2 when all of D is
 *            fresh), then c at each point.  The solution is constant per
 *            cell; a point on a face between two cells takes the mean of
 *            both, on a corner of four the mean of the four (the point's
 *            cell coordinates u = x ny, v = (y + 1) ny decide, in FP64).
 * A solve that stops early (HENRY_STATUS_NONFINITE or _SYNC) gets NaN in
 * the records after the step it stopped at.  Errors: those of
 * henry_solve_batch, and HENRY_EINVAL for nrec, npts, points, c_fresh or
 * trace_out out of range. */
int henry_solve_batch_trace(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field,
                            const double* xi, const double* phi, const double* logk, const double* qin,
                            const double* c0, const henry_opts_t* opts, int32_t nrec, int32_t npts,
                            const double* points, double c_fresh, double* trace_out, double* c_out, double* p_out,
                            double* qoi_out, int32_t* status, int32_t* iters, void* workspace, size_t ws_bytes,
                            void* stream);

/* Sample statistics of nvals quantities over nsamples samples (Sec. 4: the
 * means, variances and quantiles of Figs. 4 and 6; with x_sub the level
 * differences Y_l of paired samples, Sec. 3 eq:A, for MLMC estimates of
 * time series).  x: device [nsamples][nvals]; x_sub: device, the same
 * shape, or NULL; the statistics are of x - x_sub (of x when NULL).
 * Per column v: mean_out[v], the unbiased variance
 * var_out[v] (0 for one sample), and for each probability probs[k] (host,
 * nq <= 16 values in [0, 1]) q_out[k][v] = x_(lo) + (h - lo)(x_(lo+1) - x_(lo)),
 * h = (nsamples - 1) probs[k], lo = floor(h), x_(i) the i-th smallest
 * (Hyndman and Fan's type 7).  NaN sorts after every number and propagates
 * into the mean and variance.  1 <= nsamples, and nsamples <= 8192 when
 * quantiles are asked for (nq > 0; they sort the samples in LDS).  Outputs device,
 * caller-owned.  Deterministic (fixed-order sums, a sort).  Errors:
 * HENRY_EINVAL. */
int henry_sample_stats(henry_ctx* ctx, int32_t nsamples, int32_t nvals, const double* x, const double* x_sub,
                       int32_t nq, const double* probs, double* mean_out, double* var_out, double* q_out,
                       void* stream);

/* First-passage times of sampled series (Sec. 4, Figs. 5 and 7: the first
 * output time at which Q_FW falls below a level, or c at a point crosses
 * one).  trace: device [nsamples][nrec][stride] (as henry_solve_batch_trace
 * writes it); for each sample s, t_out[s] (device) = the first record
 * k = 1..nrec whose value in column col is < threshold (below != 0) or
 * > threshold (below == 0), or 0 if no record is; hist_out (device
 * [nrec + 1], or NULL) = the number of samples with each value of t_out.
 * Errors: HENRY_EINVAL. */
int henry_first_passage(henry_ctx* ctx, int32_t nsamples, int32_t nrec, int32_t stride, int32_t col,
                        const double* trace, double threshold, int32_t below, int32_t* t_out, int32_t* hist_out,
                        void* stream);

/* One multigrid level's smoothing on a caller's linear system A x = b, with
 * the device functions the solves run in every V-cycle (the multigrid
 * preconditioning of Sec. 2.3, redesigned: RB Gauss-Seidel for the
 * pressure, zebra line relaxation for the transport), for checking each on
 * its own.  nx x ny as for a solve; fields [ny][nx] device FP64; x is the
 * start on entry and the result on return (converted to the inner type of
 * prec and back).
 *   kind 0: `sweeps` red-black Gauss-Seidel sweeps, red cells ((i + j) even)
 *           first, on the pressure operator
 *             (A x)_P = sum over P's interior faces f of t_f (x_P - x_Q)
 *                       + te_P x_P on the last column (the seawater face),
 *           coef [2][ny][nx] = te (east face; on the last column the
 *           seawater face), tn (north face; the top row's is ignored).
 *   kind 1 / 2: `sweeps` zebra sweeps of x-lines (rows 0, 2, .. then 1, 3,
 *           ..) or y-lines (columns, likewise), each line solved exactly, on
 *           the transport operator (A x)_P = d_P x_P - sum_Q a_PQ x_Q: a
 *           neighbour couples through the inflow across the shared face plus
 *           diffusion, a_PE = max(-mx_P, 0) + dx_P, a_PW = max(mx_W, 0) + dx_W,
 *           a_PN = max(-my_P, 0) + dy_P, a_PS = max(my_S, 0) + dy_S; d_P =
 *           acc_P + the sum of P's couplings + on the last column
 *           max(-mr_j, 0) + dr_j, on the first dl_j + ml_j.
 *           coef [5][ny][nx] = acc, mx, my, dx, dy (mass flux and diffusion
 *           of the east / north face; the last column's mx and the top row's
 *           my unused), then [4][ny] = mr, dr, dl, ml.
 * workspace: device, 256-byte aligned, >= e (10 nx ny + 4 ny) bytes, e = 4
 * (HENRY_PREC_MIXED) or 8 (HENRY_PREC_FP64).  One workgroup.  Errors:
 * HENRY_EINVAL, HENRY_ENOMEM (workspace too small), HENRY_EHIP. */
int henry_level_smooth(henry_ctx* ctx, int32_t nx, int32_t ny, int32_t kind, int32_t prec, int32_t sweeps,
                       const double* coef, const double* b, double* x, void* workspace, size_t ws_bytes,
                       void* stream);

/* Tuning cache of a context, per grid width nx and precision prec, used
 * by henry_solve_batch, henry_solve_batch_trace and henry_adjoint_batch
 * (the batch plan of the ensemble: how the solves of one grid are packed
 * onto workgroups and streams, priced by their cost n_l r_l, eq:workpl):
 *   threads  workgroup size when opts->threads == 0; 0 = built-in (128
 *            threads up to 128 cells, 256 up to 512, 512 up to 2048, above
 *            that 1024 with PREC_MIXED and 512 with PREC_FP64; 512 for a
 *            PREC_MIXED group whose solves are shared by clusters, which then
 *            runs the kernel's 512-thread build);
 *            <= 1024 for PREC_MIXED and <= 512 for PREC_FP64
 *   cluster  workgroups per solve (1, 2, 4 or 8) when opts->cluster == 0;
 *            0 = built-in (see henry_opts_t.cluster); grids of 2048 cells
 *            or fewer always use 1
 *   stream   stream (0..3) of the grid's group when it runs one workgroup
 *            per solve; -1 = built-in plan.  Groups with clusters always
 *            run on stream 0, one after another.
 * threads = cluster = 0 and stream = -1 clear the entry.  None of the
 * choices changes a result (bitwise).  The measuring driver that fills it
 * times candidates on short runs of the caller's own batch (Python
 * binding: paper_2302_07804_amd.autotune).  henry_tune_get returns the
 * effective workgroup size of a group of one workgroup per solve and the
 * stored cluster and stream (0 / -1 = built-in); cluster and stream may be
 * NULL. */
int henry_tune_set(henry_ctx* ctx, int32_t nx, int32_t prec, int32_t threads, int32_t cluster, int32_t stream);
int henry_tune_get(henry_ctx* ctx, int32_t nx, int32_t prec, int32_t* threads, int32_t* cluster, int32_t* stream);

/* Per-group timings of the last profiled henry_solve_batch call: writes up
 * to `cap` entries, returns the group count through *ngroups.  Synchronises
 * with the recorded events (blocks the host until that work is done). */
int henry_profile_last(henry_ctx* ctx, henry_group_time_t* out, int32_t cap, int32_t* ngroups);

/* Workspace for henry_adjoint_batch: the forward workspace plus, per solve,
 * FP64 adjoint state and checkpoints:
 * 8 (16 n + 8 + ceil(r/k) (10 n + 8) + (k + 1) 2 n) bytes for n cells,
 * r steps, checkpoint interval k. */
int henry_adjoint_workspace_bytes(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves,
                                  const henry_opts_t* opts, int32_t ckpt_every, size_t* bytes_out);

/* Discrete adjoint of the batched solves (not in the paper; gradients of
 * the QoI of henry_solve_batch with respect to the uncertain inputs of
 * Sec. 2.2).  For the implicit steps R^n(u^n, c^{n-1}) = 0 and
 * Q = h^2 sum_{x<1} phi rho(c^N) c^N:
 *   (J^N)^T lam^N = (dQ/du^N)^T,  (J^n)^T lam^n = -(dR^{n+1}/dc^n)^T lam^{n+1},
 *   dQ/dtheta = dQ/dtheta|explicit - sum_n (lam^n)^T dR^n/dtheta,
 * J^n the exact step Jacobian.  Each transposed system is solved by FP64
 * defect correction to max |r|/diag <= adj_tol * max |b|/diag (at most
 * adj_max_it iterations) with the forward V-cycles (opts->prec inner
 * precision) as preconditioner.  The forward pass keeps (p, c) and the
 * four older states of its extrapolated initial guess every ckpt_every
 * steps and recomputes each segment (bitwise the same states) during the
 * reverse sweep.
 *   qoi_out   device [nsolves]
 *   dq_dxi    device [nsolves][3] (CLOSED3, TWOLAYER3) or [nsolves][41]
 *             (KL41); must be NULL for EXPLICIT
 *   dq_dlogk  device packed per cell, dQ/d(log K), or NULL
 *   dq_dphi   device packed per cell, dQ/dphi, or NULL
 *   dq_dq     device [nsolves], dQ/dq (q in m/s), or NULL
 *   status    device [nsolves]: HENRY_STATUS_NOCONV if a forward or an
 *             adjoint step did not converge
 *   iters     device [nsolves] forward + adjoint iterations, or NULL
 * Errors as henry_solve_batch. */
int henry_adjoint_batch(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field,
                        const double* xi, const double* phi, const double* logk, const double* qin,
                        const henry_opts_t* opts, int32_t ckpt_every, double adj_tol, int32_t adj_max_it,
                        double* qoi_out, double* dq_dxi, double* dq_dlogk, double* dq_dphi, double* dq_dq,
                        int32_t* status, int32_t* iters, void* workspace, size_t ws_bytes, void* stream);

/* MLMC level-difference statistics (Sec. 3: eq:EgL / eq:A, Def. eq:Yell).
 * For each level l = 0..L with m[l] samples on grid fine[l]:
 *   Y_l = c_l - I c_{l-1}   (field; I = piecewise-constant injection from
 *                            the coarse grid, which has half the cells per
 *                            direction; Y_0 = c_0)
 *   and Q_l - Q_{l-1} for the scalar QoI.
 * Outputs (device, caller-owned):
 *   mean_Y[l], var_Y[l]: [cells_l] sample mean and unbiased (m-1) variance
 *   qstats: [L+1][2] mean and unbiased variance of the QoI difference
 *   Ec_finest: [cells_L] telescoped E[c] = sum_l I_{l->L} mean_Y[l]
 *   var_est: [2] sum_l V_l/m_l for the QoI, and max over cells of the
 *            same sum for the field.
 * c_fine[l] is [m_l][cells_l], c_coarse[l] is [m_l][cells_l / 4] (NULL at
 * l = 0); q_fine[l], q_coarse[l] are [m_l] (q_coarse[0] NULL).  The pointer
 * arrays themselves are host arrays of device pointers.  Sums run in a
 * fixed order (deterministic); m[l] >= 2. */
int mlmc_level_estimate(henry_ctx* ctx, int32_t L, const henry_grid_t* fine, const int32_t* m,
                        const double* const* c_fine, const double* const* c_coarse,
                        const double* const* q_fine, const double* const* q_coarse,
                        double* const* mean_Y, double* const* var_Y, double* qstats, double* Ec_finest,
                        double* var_est, void* stream);

/* Partial sums of the telescoping MLMC estimator (Sec. 3, eq:A: the
 * estimate of E[g_L] is the sum over levels of the sample means of
 * Y_l = g_l - g_{l-1}) and of its variance sum_l V_l / m_l (the variance
 * half of eq:MSE), for nvals quantities at once, FP64 on the device in a
 * fixed order:
 *   pmean_out[l][v] = sum_{i <= l} mean[i][off[i] + v]
 *   pvar_out[l][v]  = sum_{i <= l} var[i][off[i] + v] / m[i]
 * Row nlevels-1 is the estimate and its variance; row l is the estimate
 * truncated after level l (the partial sums Fig. 11 compares with its
 * reference).
 *   mean, var  host arrays [nlevels] of device pointers to level means and
 *              unbiased variances (henry_sample_stats, mlmc_level_estimate);
 *              var may be NULL, then pvar_out is not written (may be NULL)
 *   m          host [nlevels] sample counts, m[l] >= 1
 *   off        host [nlevels] element offsets into each level's arrays
 *              (e.g. the cell that holds a point on level l's grid), or NULL
 *   pmean_out, pvar_out  device [nlevels][nvals], caller-owned
 * 1 <= nlevels <= 16, nvals >= 0.  Errors: HENRY_EINVAL (NULL pointer,
 * counts or offsets out of range), HENRY_EHIP. */
int henry_mlmc_telescope(henry_ctx* ctx, int32_t nlevels, int32_t nvals, const double* const* mean,
                         const double* const* var, const int32_t* m, const int64_t* off, double* pmean_out,
                         double* pvar_out, void* stream);

/* Sample allocation of an MLMC run (Sec. 3, eq:M_ell): with per-level
 * variances V[l] of Y_l = g_l - g_{l-1} and costs s[l] > 0 per sample
 * (any unit), the counts that minimise sum m_l s_l at estimator variance
 * sum V_l / m_l = eps2:
 *   m_out[l] = ceil(eps2^-1 sqrt(V_l / s_l) sum_i sqrt(V_i s_i)),
 *   cost_out = eps2^-1 (sum_l sqrt(V_l s_l))^2 (or NULL).
 * Host arrays of nlevels >= 1.  A level with V_l = 0 gets 0; callers keep
 * at least their pilot count.  Errors: HENRY_EINVAL (V < 0, s <= 0,
 * eps2 <= 0, non-finite input, a count beyond 9e18). */
int henry_mlmc_allocate(int32_t nlevels, const double* V, const double* s, double eps2, int64_t* m_out,
                        double* cost_out);

/* Convergence rates of an MLMC hierarchy (Sec. 3; the decay the paper fits
 * in its Fig. 10): least-squares slopes over levels l = first .. nlevels-1
 * of log2 |E[Y_l]| and log2 V_l, |E[Y_l]| ~ 2^(-alpha l), V_l ~ 2^(-beta l),
 * and, if bias is not NULL, the bias estimate of the finest level
 * |E[Y_L]| / (2^alpha - 1) (infinite when alpha <= 0) for the MSE split
 * eq:MSE.  Host arrays; at least two levels in the fit, at most 64 levels.
 * Errors: HENRY_EINVAL (fewer than two levels, a zero or non-finite mean or
 * variance in the fit). */
int henry_mlmc_rates(int32_t nlevels, const double* mean, const double* var, int32_t first, double* alpha,
                     double* beta, double* bias);

/* Quasi-Monte Carlo points for a reference mean (abstract and Sec. 4,
 * Fig. 11: the paper checks MLMC against a QMC mean on its finest mesh; its
 * set-up names the Halton sequence).  For k = 0..count-1, d = 0..dim-1:
 *   xi[k][d] = 2 frac(phi_{b_d}(first + k) + shift[d]) - 1   in [-1, 1),
 * phi_b the radical inverse in base b (the base-b digits of the index
 * mirrored about the radix point), b_d the d-th prime (2, 3, 5, ...).
 * shift: host, dim values in [0, 1), or NULL for none -- a Cranley-Patterson
 * rotation; independent uniform shifts give independent unbiased estimates
 * whose spread estimates the QMC error.  xi: host [count][dim] row-major,
 * caller-owned; the points feed HENRY_FIELD_CLOSED3 (dim 3) like
 * henry_sample_xi's.  Index 0 is the origin of the sequence; a rule usually
 * starts at first = 1.  Each phi_b is correctly rounded (exact in base 2).
 * Errors: HENRY_EINVAL (first < 0, count < 0, first + count > 2^31,
 * dim outside 1..16, a shift outside [0, 1), xi NULL with count > 0). */
int henry_qmc_points(int64_t first, int64_t count, int32_t dim, const double* shift, double* xi);

#ifdef __cplusplus
}
#endif
#endif /* HENRY_H */
