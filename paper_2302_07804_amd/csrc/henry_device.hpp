// henry_device.hpp -- gfx950 device code for batched Henry solves.
//
// One workgroup, or for a large grid a cluster of 2-8 workgroups on one XCD,
// owns one solve (one random sample on one grid) and runs its whole
// implicit time loop (Sec. 2.3: implicit Euler, fixed tau).  Each step
// is a defect correction on the FP64 nonlinear residual of the cell-centred
// discretisation of e_cont_eq / e_tran_eq / e_Darcy_vel (Sec. 2.1):
//
//   repeat
//     R = R(p, c)                                   FP64, scaled max norms
//     stop if both norms <= tol
//     unless |R^p| <= tol:
//       (A_pp) dp = -R^p  one V(2,2) cycle, red-black Gauss-Seidel   inner T
//       p += dp                                                       FP64
//     R = R(p, c), S = R^c - c R^p                                    FP64
//     stop if both norms <= tol
//     (A_cc) dc = -S      one V-cycle, zebra x-lines before the coarse
//                         correction, x- (global levels) or y-lines
//                         (LDS levels) after                      inner T
//     c += dc                                                         FP64
//
// Each step starts from an extrapolation through the last converged states
// (interpolating polynomials up to cubic, then on long solves the
// least-squares cubic through five states; see implicit_step).
//
// A_pp = -div(rho K / mu grad .) with the seawater Dirichlet face.  The salt
// block is driven by S = R^c - c R^p, an exact recombination of the two
// equations (same discrete solution): S is the non-conservative upwind form
// of e_tran_eq, in which a mass-flux error of an inexact pressure solve no
// longer appears as a salt source.  A_cc, its frozen-flux derivative, is an
// M-matrix with the stored-mass term (h^2/tau) phi rho(c^n) on the diagonal
// and upwind inflow plus diffusion couplings.  The inner precision T is float (the
// mixed path) or double (the plain FP64 path): one code path, two
// instantiations.  Memory: per-solve FP64 state and per-level inner arrays
// in a caller-provided workspace (L2 / Infinity-Cache resident for the
// grid sizes of an MLMC hierarchy); line systems are solved in registers by
// segmented elimination with a cyclic-reduction interface solve across the
// lanes of a wavefront.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

// The namespace and the FP32 kernel's workgroup bound of this build: the
// library compiles this header twice, as henry with 1024-thread bounds
// (henry_api.hip) and as henry512 with 512-thread bounds (henry_solve512.hip),
// so that each build's device functions get their own register budget.
#ifndef HENRY_NS
#define HENRY_NS henry
#endif
#ifndef HENRY_FP32_THREADS
#define HENRY_FP32_THREADS 1024
#endif
// Grids of at least HENRY_RES_FIELDS_NX columns (0: none): the residual
// pass forms the face coefficients and the norm scale from K and phi (5 FP64
// loads per cell instead of 9, and three FP64 divisions); smaller ones load
// the stored ones.  Both give the same bits.
#ifndef HENRY_RES_FIELDS_NX
#define HENRY_RES_FIELDS_NX 0
#endif
// Cells per thread gathered by the grid transfers of the builds with at most
// 512 threads (the 1024-thread build takes one).
#ifndef HENRY_TRANSFER_BATCH
#define HENRY_TRANSFER_BATCH 1
#endif

namespace HENRY_NS {

// Cells per thread whose operands a transfer between levels (restriction,
// prolongation, coefficient coarsening) from a finer level in global memory
// gathers before it writes any, so that their loads are in flight together;
// the 1024-thread build has no registers to spare for more than one.
constexpr int kTBatch = HENRY_FP32_THREADS <= 512 ? HENRY_TRANSFER_BATCH : 1;

constexpr int kMaxLevels = 12;  // ny <= 512 -> at most 10 multigrid levels
constexpr int kWave = 64;

struct Phys {
    double rho0, rho1, mu, g, D, phi0, k0, q_in, T;
};

// One solve of a batch.  Offsets are in bytes from the workspace base
// (ws_off) or in elements of the packed field arrays (field_off).
struct SolveDesc {
    int32_t nx, ny, nsteps, nlev;
    int32_t reserved;
    int32_t index;       // position in the caller's solve list
    int64_t ws_off;
    int64_t field_off;
    int64_t adj_off;     // adjoint region (adjoint calls only)
};

struct Launch {
    const SolveDesc* descs;
    uint8_t* ws;
    const double* xi;    // [nsolves][3] or null
    const double* phi_in;
    const double* logk_in;
    const double* qin_in;
    const double* c0;
    double* c_out;
    double* p_out;
    double* qoi_out;
    int32_t* status;
    int32_t* iters;
    Phys ph;
    double tol;
    int32_t max_outer;
    int32_t predictor;       // henry_opts_t.predictor
    int32_t field_kind;
    int32_t g_begin, g_end;  // global step range of this launch
    int32_t g_total;         // global steps of the whole batch (max nsteps)
    int32_t lds_cells;       // multigrid levels with at most this many cells live in LDS (wavefront 0)
    int32_t lds_block_cells; // levels 1.. with at most this many cells also live in LDS (whole workgroup)
    int32_t lds_bytes;       // dynamic LDS of the launch (the LDS levels, or the line staging if larger)
    int32_t xi_dim;          // coefficients per solve in xi (3 closed form, 41 KL)
    const double* kl_modes;  // KL: sqrt(lam_k) e_k at the cells of this group's grid, [20][n]
    double kl_sigma_phi, kl_sigma_logk;
    int32_t nsolves;         // solves of this launch (descs[0 .. nsolves-1])
    int32_t cluster;         // workgroups per solve (1, 2, 4 or 8)
    uint64_t cluster_wait;   // bound of one cluster-barrier wait, ticks of the 100 MHz wall clock
    // time series (forward solves only; trace == nullptr: none): record k =
    // 1..trace_nrec after step ceil(k nsteps / trace_nrec), holding the
    // fresh-water area and c at trace_npts points, at
    // trace[index][k-1][0 .. trace_npts]
    double* trace;
    int32_t trace_nrec, trace_npts;
    double trace_fresh;             // c threshold of the fresh-water indicator
    double trace_pts[2 * 16];       // (x, y) of each point
};

constexpr int kMaxTracePoints = 16;

// ------------------------------------------------------------------ layout
__host__ __device__ inline int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

__host__ __device__ inline int num_levels(int ny) {
    int L = 1;
    while (ny > 1) { ny >>= 1; ++L; }
    return L;
}

// Per-level inner arrays, in this order, each nx_l*ny_l elements of T:
//   x, b, r, te, tn, acc, mx, my, dx, dy
// followed by four row arrays of ny_l elements: dl, dr, mr, ml
// (left diffusion, right diffusion, right mass flux, left inflow).
constexpr int kLevelArrays = 10;
constexpr int kRowArrays = 4;

template <typename T>
__host__ __device__ inline int64_t level_bytes(int nx, int ny) {
    return align256((int64_t)(kLevelArrays * nx * ny + kRowArrays * ny) * (int64_t)sizeof(T));
}

// FP64 arrays: p, c, cn, phi, K, pp (previous p), then the face
// coefficients that depend only on the fields, set once per solve:
//   tx, ty  east / north face K_f / mu (harmonic K; 2 K_P / mu on the
//           seawater face; 0 above the top row),
//   wx, wy  east / north face phi_f D (harmonic phi; 2 phi_P D on the
//           seawater face; 0 above the top row),
//   isc     residual scale tau / (h^2 phi_P rho0),
// then the older states c2, p2 (u^{n-2}), c3, p3 (u^{n-3}) and c4, p4
// (u^{n-4}) of the extrapolated initial guess (their roles rotate: bind_history), then kScratch doubles of
// scratch: [0] recharge, [1] status, [2] outer iterations, [3] converged states in a row, [4] the history's
// rotation at the end of a launch, [8..31] phase timers of builds with
// HENRY_PHASE_TIMERS, [32..63] the state of a cluster of workgroups sharing the solve (the members'
// 32-bit arrival counts in [32..35], the error flag in [36], barriers passed [37], the members' XCD
// ids [40..47], their partial residual norms [48..63]).
enum : int { kP, kC, kCn, kPhi, kK, kPp, kTx, kTy, kWx, kWy, kIsc, kC2, kP2, kC3, kP3, kC4, kP4, kF64Arrays };
constexpr int kScratch = 64;
constexpr int kClusterFlags = 32, kClusterErr = 36, kClusterGen = 37, kClusterXcc = 40, kClusterSlots = 48;
constexpr int kMaxCluster = 8;
// the barrier polls the K arrival counts and the error flag in one load:
// the flag sits past the last count, within one wavefront's lanes
static_assert((kClusterErr - kClusterFlags) * 2 >= kMaxCluster && (kClusterErr - kClusterFlags) * 2 < 64,
              "cluster error flag placement");

template <typename T>
__host__ __device__ inline int64_t solve_bytes(int nx, int ny) {
    int64_t b = align256((int64_t)kF64Arrays * nx * ny * 8 + kScratch * 8);
    int lx = nx, ly = ny;
    const int L = num_levels(ny);
    for (int l = 0; l < L; ++l) {
        b += level_bytes<T>(lx, ly);
        lx >>= 1; ly >>= 1;
    }
    return b;
}

template <typename T>
struct Level {
    using value_type = T;
    int nx, ny;
    T *x, *b, *r, *te, *tn, *acc, *mx, *my, *dx, *dy, *dl, *dr, *mr, *ml;
};

// Address-space-typed view of a level for the smoothers and transfers: AS 1
// (global memory) or 3 (LDS) lets the compiler emit global_* / ds_*
// instructions instead of flat ones; AS 0 keeps generic pointers.
template <typename T, int AS> struct AsPtr { using type = T*; };
template <typename T> struct AsPtr<T, 1> { using type = __attribute__((address_space(1))) T*; };
template <typename T> struct AsPtr<T, 3> { using type = __attribute__((address_space(3))) T*; };
template <int AS, typename T>
__device__ inline typename AsPtr<T, AS>::type as_ptr(T* p) { return (typename AsPtr<T, AS>::type)p; }

template <typename T, int AS>
struct LV {
    using value_type = T;
    using P = typename AsPtr<T, AS>::type;
    int nx, ny;
    P x, b, r, te, tn, acc, mx, my, dx, dy, dl, dr, mr, ml;
    __device__ explicit LV(const Level<T>& v)
        : nx(v.nx), ny(v.ny), x(as_ptr<AS>(v.x)), b(as_ptr<AS>(v.b)), r(as_ptr<AS>(v.r)), te(as_ptr<AS>(v.te)),
          tn(as_ptr<AS>(v.tn)), acc(as_ptr<AS>(v.acc)), mx(as_ptr<AS>(v.mx)), my(as_ptr<AS>(v.my)),
          dx(as_ptr<AS>(v.dx)), dy(as_ptr<AS>(v.dy)), dl(as_ptr<AS>(v.dl)), dr(as_ptr<AS>(v.dr)),
          mr(as_ptr<AS>(v.mr)), ml(as_ptr<AS>(v.ml)) {}
};

template <typename T>
struct Solve {
    int nx, ny, n, nsteps, L;
    int lds_from;  // first level whose arrays live in LDS and that wavefront 0 runs alone
    int lb;        // first level whose arrays live in LDS (lb <= lds_from)
    int lc;        // levels 0 .. lc-1 are run by the whole cluster (0 with one workgroup)
    int hand;      // level lc is in LDS and fed by the cluster through its global copy hg
    int hist;      // rotation of the state history (see bind_history)
    double h, tau;
    double q;  // recharge (m/s)
    double *p, *c, *cn, *phi, *K, *pp, *tx, *ty, *wx, *wy, *isc, *c2, *p2, *c3, *p3, *c4, *p4, *scratch;
    Level<T> lv[kMaxLevels];
    Level<T> hg;  // the global-memory arrays of level lb
    double *rout_p, *rout_c;  // residual outputs (henry_residual_kernel)
};

// Levels in LDS: every level of at most `lds_cells` cells (run by
// wavefront 0), and levels 1.. of at most `lds_block_cells` cells (run by
// the whole workgroup; level 0 always stays in global memory, where the
// FP64 residual pass of the whole cluster writes it).
__host__ __device__ inline bool level_in_lds(int l, int cells, int lds_cells, int lds_block_cells) {
    return cells <= lds_cells || (l >= 1 && cells <= lds_block_cells);
}

// Dynamic LDS bytes for the LDS levels of an nx x ny hierarchy.
template <typename T>
__host__ __device__ inline int64_t lds_level_bytes(int nx, int ny, int lds_cells, int lds_block_cells) {
    int64_t b = 0;
    int lx = nx, ly = ny;
    const int L = num_levels(ny);
    for (int l = 0; l < L; ++l) {
        if (level_in_lds(l, lx * ly, lds_cells, lds_block_cells)) b += level_bytes<T>(lx, ly);
        lx >>= 1; ly >>= 1;
    }
    return b;
}

// The state history: five arrays per field hold the iterate and the four
// converged states before it, u^n .. u^{n-3} (the roles c / cn / c2 / c3 /
// c4 and p / pp / p2 / p3 / p4).  A step's extrapolated start overwrites the
// oldest state in place (each cell reads only its own history) and the roles
// then rotate by one: role k is array (k + hist) mod 5 of the field, and a
// step takes hist to hist + 4 mod 5.  One write per cell and field instead of
// five (the older states are never copied).
template <typename T>
__device__ inline void bind_history(Solve<T>& S, uint8_t* base) {
    double* f = reinterpret_cast<double*>(base);
    const int64_t n = (int64_t)S.nx * S.ny;
    const int cs[5] = {kC, kCn, kC2, kC3, kC4}, ps[5] = {kP, kPp, kP2, kP3, kP4};
    double** cr[5] = {&S.c, &S.cn, &S.c2, &S.c3, &S.c4};
    double** pr[5] = {&S.p, &S.pp, &S.p2, &S.p3, &S.p4};
    for (int k = 0; k < 5; ++k) {
        *cr[k] = f + (int64_t)cs[(k + S.hist) % 5] * n;
        *pr[k] = f + (int64_t)ps[(k + S.hist) % 5] * n;
    }
}

// Binds the solve's arrays.  The LDS levels (level_in_lds) get their inner
// arrays in the workgroup's LDS (`lds`): they are rebuilt every iteration,
// so nothing there has to survive a launch.  Every level keeps its region
// in the workspace too (S.hg views that of level lb).  lds_cells >= 2, so
// the coarsest level (2 x 1) is always in LDS and S.lds_from < S.L.
template <typename T>
__device__ inline void bind_solve(Solve<T>& S, uint8_t* base, int nx, int ny, uint8_t* lds, int lds_cells,
                                  int lds_block_cells) {
    S.nx = nx; S.ny = ny; S.n = nx * ny; S.L = num_levels(ny);
    S.h = 1.0 / ny;
    double* f = reinterpret_cast<double*>(base);
    const int n = nx * ny;
    auto arr = [&](int k) { return f + (int64_t)k * n; };
    S.phi = arr(kPhi); S.K = arr(kK);
    S.tx = arr(kTx); S.ty = arr(kTy); S.wx = arr(kWx); S.wy = arr(kWy); S.isc = arr(kIsc);
    S.scratch = arr(kF64Arrays);
    S.hist = 0;
    bind_history(S, base);
    uint8_t* q = base + align256((int64_t)kF64Arrays * n * 8 + kScratch * 8);
    uint8_t* ql = lds;
    int lx = nx, ly = ny;
    S.lds_from = S.L;
    S.lb = S.L;
    S.lc = 0;
    S.hand = 0;
    auto bind_level = [](Level<T>& v, T* a, int lx, int ly) {
        const int m = lx * ly;
        v.nx = lx; v.ny = ly;
        v.x = a; v.b = a + m; v.r = a + 2 * m; v.te = a + 3 * m; v.tn = a + 4 * m; v.acc = a + 5 * m;
        v.mx = a + 6 * m; v.my = a + 7 * m; v.dx = a + 8 * m; v.dy = a + 9 * m;
        v.dl = a + 10 * m; v.dr = a + 10 * m + ly; v.mr = a + 10 * m + 2 * ly; v.ml = a + 10 * m + 3 * ly;
    };
    for (int l = 0; l < S.L; ++l) {
        const bool in_lds = level_in_lds(l, lx * ly, lds_cells, lds_block_cells);
        if (in_lds && S.lb == S.L) {
            S.lb = l;
            bind_level(S.hg, reinterpret_cast<T*>(q), lx, ly);
        }
        if (lx * ly <= lds_cells && S.lds_from == S.L) S.lds_from = l;
        bind_level(S.lv[l], reinterpret_cast<T*>(in_lds ? ql : q), lx, ly);
        if (in_lds) ql += level_bytes<T>(lx, ly);
        q += level_bytes<T>(lx, ly);
        lx >>= 1; ly >>= 1;
    }
}

// ------------------------------------------------------------------ reductions
// max that propagates NaN (fmax would drop it)
__device__ inline double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

__device__ inline double wave_max(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = nanmax(v, __shfl_xor(v, o));
    return v;
}
__device__ inline double wave_sum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-wide max / sum in a fixed order; `red` holds >= nwaves doubles.
// Ends with every thread holding the result.
__device__ inline double block_max(double v, double* red) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int k = 1; k < nw; ++k) r = nanmax(r, red[k]);
    return r;
}
__device__ inline void block_max2(double& a, double& b, double* red) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    a = wave_max(a);
    b = wave_max(b);
    __syncthreads();
    if (lane == 0) { red[2 * w] = a; red[2 * w + 1] = b; }
    __syncthreads();
    double ra = red[0], rb = red[1];
    for (int k = 1; k < nw; ++k) { ra = nanmax(ra, red[2 * k]); rb = nanmax(rb, red[2 * k + 1]); }
    a = ra;
    b = rb;
}
__device__ inline double block_sum(double v, double* red) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int k = 1; k < nw; ++k) r += red[k];
    return r;
}

// Every level's nx and ny are powers of two: cell coordinates come from
// shifts and masks instead of integer division.
__device__ inline int log2i(int v) { return __builtin_ctz((unsigned)v); }

// Division inside the FP32 inner solves uses the hardware reciprocal (about
// 1 ulp; the solves only precondition the FP64 defect correction); the FP64
// path divides exactly.
template <typename T>
__device__ inline T qdiv(T a, T b) {
    if constexpr (sizeof(T) == 4) return a * __builtin_amdgcn_rcpf(b);
    else return a / b;
}

// ------------------------------------------------------------------ teams
// The threads that run one multigrid operation together: the whole
// workgroup (levels in global memory), or wavefront 0 alone (the coarse
// levels in LDS, where barrier latency would dominate the little work).
// Within one wavefront the lanes execute in lockstep and LDS operations of
// the wavefront complete in issue order, so a wavefront-scope fence (which
// keeps the compiler from moving memory operations across it) is the whole
// synchronisation.
struct BlockTeam {
    __device__ static int rank() { return threadIdx.x; }
    __device__ static int size() { return blockDim.x; }
    __device__ static void sync() { __syncthreads(); }
};
struct WaveTeam {
    __device__ static int rank() { return threadIdx.x & (kWave - 1); }
    __device__ static int size() { return kWave; }
    __device__ static void sync() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

// ------------------------------------------------------------------ clusters
// A large grid's solve can be shared by K workgroups (a cluster, K = 2, 4
// or 8), one per CU: the fine levels (0 .. S.lc-1) are split over all
// K x blockDim threads, while member 0 (the leader) runs the coarse levels
// alone.  Every cell and every line is computed by the same arithmetic
// whatever the split, and the residual norms are maxima, so a solve gives
// bitwise the same result for every K.
//
// Members of a cluster are placed on one XCD: the workgroups of a launch
// are dealt to the eight XCDs round robin (block b on XCD b mod 8), so the
// members of cluster c on XCD x are K consecutive blocks of that XCD's
// sequence.  Each launch checks the placement (hardware XCC id, exchanged
// under an agent-scope barrier); the clusters whose members share one XCD,
// and so one L2, synchronise by waiting for their own stores, a relaxed
// store of the member's arrival count and an acquire poll of all members'
// counts in one load (L1 invalidated); any other cluster uses the
// agent-scope release (L2 write-back) instead.  Blocks of one XCD are
// dispatched in order, so the lowest cluster not yet complete always gets
// its members.  Every wait is bounded (Launch::cluster_wait, 10 s by
// default): past it a member raises the cluster's error flag, every later
// barrier of the cluster returns at once, and the solve reports
// HENRY_STATUS_SYNC.
struct ClusterState {
    int K, member, base, size;
    unsigned* flags; // [K] barriers each member has arrived at
    unsigned* err;   // sticky error flag
    double* slots;   // [2K] partial norms
    unsigned gen;    // barriers passed
    int local;       // all members on one XCD
    int failed;
    uint64_t wait;   // bound of one wait (wall-clock ticks)
    uint8_t* stage;  // the dynamic LDS, as line staging buffers on the cluster levels
    int stage_waves; // wavefronts whose staging buffer fits in it
};
__shared__ ClusterState g_cl;

__device__ inline int xcc_id() { return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)); }

// Every workgroup of a cluster waits until all K members have arrived; all
// memory operations before the call are visible to every member after it.
// Wavefront 0 publishes the member's arrival count and polls the K counts
// and the cluster's error flag with one load per lane (lane k < K: member
// k's count; the lane at the error flag's offset: the flag), relaxed, so
// that one poll is one L2 round trip; one acquire fence after the counts
// are all there makes the members' stores visible.  The wall clock is read
// every 16 polls only.
__device__ inline void cluster_barrier() {
    __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have reached L2
    __syncthreads();
    if (threadIdx.x < kWave) {
        const int lane = (int)threadIdx.x;
        const unsigned gen = g_cl.gen + 1u;
        if (!g_cl.failed) {
            if (lane == 0) {
                if (g_cl.local) __hip_atomic_store(g_cl.flags + g_cl.member, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else __hip_atomic_store(g_cl.flags + g_cl.member, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            const int eoff = (int)(g_cl.err - g_cl.flags);  // the error flag's offset (>= K)
            const bool is_err = lane == eoff;
            const unsigned* f = g_cl.flags + (lane < g_cl.K || is_err ? lane : 0);
            const uint64_t t0 = wall_clock64();
            bool failed = false;
            for (unsigned polls = 1;; ++polls) {
                const unsigned v = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (__any(is_err && v != 0u)) {
                    failed = true;
                    break;
                }
                if (__all(is_err || (int)(v - gen) >= 0)) break;
                if ((polls & 15u) == 0u && wall_clock64() - t0 > g_cl.wait) {
                    failed = true;
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (failed && lane == 0) {
                __hip_atomic_store(g_cl.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                g_cl.failed = 1;
            }
        }
        if (lane == 0) g_cl.gen = gen;
    }
    __syncthreads();
}

// All K x blockDim threads of the cluster (the workgroup when K = 1).
struct ClusterTeam {
    __device__ static int rank() { return g_cl.base + (int)threadIdx.x; }
    __device__ static int size() { return g_cl.size; }
    __device__ static void sync() {
        if (g_cl.K == 1) __syncthreads();
        else cluster_barrier();
    }
};

// The launch's dynamic LDS as line staging buffers (thread 0; read after the
// next workgroup barrier).
__device__ inline void cluster_stage(uint8_t* lds, int lds_bytes, int64_t per_wave) {
    g_cl.stage = lds;
    g_cl.stage_waves = (int)(lds_bytes / per_wave);
}

// Cluster of one workgroup (the adjoint kernel, small grids).
__device__ inline void cluster_init_single() {
    if (threadIdx.x == 0) {
        g_cl.K = 1; g_cl.member = 0; g_cl.base = 0; g_cl.size = (int)blockDim.x;
        g_cl.flags = nullptr; g_cl.err = nullptr; g_cl.slots = nullptr;
        g_cl.gen = 0u; g_cl.local = 1; g_cl.failed = 0; g_cl.wait = 0;
        g_cl.stage = nullptr; g_cl.stage_waves = 0;  // no line staging unless cluster_stage says so
    }
    __syncthreads();
}

// Binds member `member` of a K-cluster to the cluster state in the solve's
// scratch `sp` and checks the members' placement.
__device__ inline void cluster_init(int K, int member, double* sp, uint64_t wait) {
    if (threadIdx.x == 0) {
        g_cl.wait = wait;
        g_cl.K = K; g_cl.member = member; g_cl.base = member * (int)blockDim.x; g_cl.size = K * (int)blockDim.x;
        g_cl.flags = reinterpret_cast<unsigned*>(sp + kClusterFlags);
        g_cl.err = reinterpret_cast<unsigned*>(sp + kClusterErr);
        g_cl.slots = sp + kClusterSlots;
        g_cl.gen = (unsigned)sp[kClusterGen];
        g_cl.local = 0;  // the placement check itself uses the agent-scope protocol
        g_cl.failed = 0;
        g_cl.stage = nullptr; g_cl.stage_waves = 0;  // no line staging unless cluster_stage says so
        sp[kClusterXcc + member] = (double)xcc_id();
    }
    cluster_barrier();
    if (threadIdx.x == 0) {
        // a cluster that failed in an earlier launch stays failed
        if (__hip_atomic_load(g_cl.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) g_cl.failed = 1;
        int same = 1;
        const double x0 = sp[kClusterXcc];
        for (int k = 1; k < K; ++k) same &= sp[kClusterXcc + k] == x0 ? 1 : 0;
        g_cl.local = same;
    }
    __syncthreads();
}

// Maxima of two per-thread values over the whole cluster, in a fixed order
// (NaN propagates); every thread of every member gets the same pair.
__device__ inline void cluster_max2(double a, double b, double* red, double& ra, double& rb) {
    double pa = a, pb = b;
    block_max2(pa, pb, red);
    if (g_cl.K == 1) {
        ra = pa; rb = pb;
        return;
    }
    if (threadIdx.x == 0) {
        g_cl.slots[2 * g_cl.member] = pa;
        g_cl.slots[2 * g_cl.member + 1] = pb;
    }
    cluster_barrier();
    ra = g_cl.slots[0];
    rb = g_cl.slots[1];
    for (int k = 1; k < g_cl.K; ++k) {
        ra = nanmax(ra, g_cl.slots[2 * k]);
        rb = nanmax(rb, g_cl.slots[2 * k + 1]);
    }
}

// Neighbour indices of (i, j), clamped to the cell itself at the boundary.
struct Nb {
    int idx, w, e, s, n;
    bool hw, he, hs, hn;
    __device__ Nb(int i, int j, int nx, int ny) {
        idx = j * nx + i;
        hw = i > 0; he = i + 1 < nx; hs = j > 0; hn = j + 1 < ny;
        w = hw ? idx - 1 : idx; e = he ? idx + 1 : idx;
        s = hs ? idx - nx : idx; n = hn ? idx + nx : idx;
    }
};

// Layout of the pressure cycle's level arrays (x, b, r, te, tn while the
// pressure V-cycle runs): every row stores its red cells ((i + j) even)
// first and its black cells after them, each in order of i, so that a
// red-black half-sweep reads and writes whole cache lines.  The transport
// cycle keeps the natural row-major order.
__device__ inline int pidx(int i, int j, int nx) { return j * nx + (((i + j) & 1) ? (nx >> 1) : 0) + (i >> 1); }

// Cell (i, j) at storage position s of the colour-split layout (nx = 2^sx).
__device__ inline void pcell(int s, int nx, int sx, int& i, int& j) {
    j = s >> sx;
    const int r = s & (nx - 1), half = nx >> 1;
    const int col = r >= half ? 1 : 0;
    i = 2 * (r - col * half) + ((j + col) & 1);
}

// Neighbour storage positions of (i, j) in the colour-split layout,
// clamped to the cell itself at the boundary.
struct NbS {
    int idx, w, e, s, n;
    bool hw, he, hs, hn;
    __device__ NbS(int i, int j, int nx, int ny) {
        hw = i > 0; he = i + 1 < nx; hs = j > 0; hn = j + 1 < ny;
        idx = pidx(i, j, nx);
        w = hw ? pidx(i - 1, j, nx) : idx; e = he ? pidx(i + 1, j, nx) : idx;
        s = hs ? pidx(i, j - 1, nx) : idx; n = hn ? pidx(i, j + 1, nx) : idx;
    }
};

// ------------------------------------------------------------------ physics (FP64)
__device__ inline double rho_of(const Phys& ph, double c) { return ph.rho0 + (ph.rho1 - ph.rho0) * c; }

// Mass and salt flux from cell a to its east neighbour b, per metre of
// depth: harmonic K and phi on the face (precomputed: tx = K_f/mu,
// wx = phi_f D), arithmetic rho; donor cell.
struct FaceFlux { double M, F, lam, dif; };

// Interior face a|b (b east or north of a); on a north face Darcy's law
// with gravity (0,-g) adds rho_f g h to the pressure difference.
template <bool kNorth>
__device__ inline FaceFlux flux_face(const Phys& ph, double h, double pa, double pb, double ca, double cb, double kf,
                                     double wf) {
    FaceFlux f;
    const double rf = 0.5 * (rho_of(ph, ca) + rho_of(ph, cb));
    f.lam = rf * kf;
    f.dif = rf * wf;
    f.M = kNorth ? -f.lam * ((pb - pa) + rf * ph.g * h) : -f.lam * (pb - pa);
    f.F = f.M * (f.M >= 0.0 ? ca : cb) - f.dif * (cb - ca);
    return f;
}

// Seawater face at x = 2 (half-cell distance): p_B = -rho1 g y, c_B = 1;
// kf = 2 K_P / mu, wf = 2 phi_P D.
__device__ inline FaceFlux flux_right(const Phys& ph, double y, double pP, double cP, double kf, double wf) {
    FaceFlux f;
    const double rB = 0.5 * (rho_of(ph, cP) + ph.rho1);
    f.lam = rB * kf;
    f.dif = rB * wf;
    f.M = -f.lam * (-ph.rho1 * ph.g * y - pP);
    f.F = f.M * (f.M >= 0.0 ? cP : 1.0) - f.dif * (1.0 - cP);
    return f;
}

// Recharge face at x = 0: inflow rho0 q h of fresh water (c_B = 0).
__device__ inline FaceFlux flux_left(const Phys& ph, double h, double q, double cP, double phiP) {
    FaceFlux f;
    const double rB = 0.5 * (rho_of(ph, cP) + ph.rho0);
    f.lam = 0.0;
    f.dif = 2.0 * rB * phiP * ph.D;
    f.M = -ph.rho0 * q * h;
    f.F = f.dif * cP;
    return f;
}

// Wall-clock accumulators of the phases of one step (builds with
// HENRY_PHASE_TIMERS only; wall_clock64 runs at a constant 100 MHz).
// Slots 0..7, 13, 15, 21, 23: phases of the outer iteration (the residual
// passes split into the pass and its reduction or barrier); 8..12, 14 and
// 16..20, 22: parts of the pressure and of the transport V-cycle.
struct PhaseClock {
#ifdef HENRY_PHASE_TIMERS
    uint64_t acc[24];
    uint64_t last;
    __device__ void init() {
        for (int k = 0; k < 24; ++k) acc[k] = 0;
        last = wall_clock64();
    }
    __device__ void tick(int k) {
        const uint64_t t = wall_clock64();
        acc[k] += t - last;
        last = t;
    }
#else
    __device__ void init() {}
    __device__ void tick(int) {}
#endif
};

// ------------------------------------------------------------------ FP64 residual
// Face coefficients between cells a and b: t = K_f / mu and w = phi_f D with
// the harmonic means K_f = 2 Ka Kb / (Ka + Kb) and phi_f = 2 fa fb / (fa + fb),
// both from one division.  At the seawater boundary (half a cell from the
// centre) the coefficients are 2 K / mu and 2 phi D: twice the pair of the
// cell with itself.  With the scale of a cell's residual in the norms, the
// fields kernel stores them; the residual pass may form them again from K and
// phi with the same operations.
struct FacePair { double t, w; };
__device__ inline FacePair face_pair(const Phys& ph, double Ka, double Kb, double fa, double fb) {
    const double sK = (Ka + Kb) * ph.mu, sf = fa + fb;
    const double r = 1.0 / (sK * sf);
    return {2.0 * Ka * Kb * sf * r, 2.0 * fa * fb * ph.D * sK * r};
}
__device__ inline double res_scale(const Phys& ph, double tau, double h, double f) { return tau / (h * h * f * ph.rho0); }

// Operands of one cell's residual, loaded from clamped indices before any
// arithmetic (no loads under boundary branches).
struct ResIn {
    double cP, cnP, phiP, pP, cE, pE, cW, pW, cN, pN;
    double txP, wxP, txW, wxW, tyP, wyP, sc;
};

// The residual of one cell from its operands; both the interior and the
// boundary flux of a face are formed and the applicable one selected.  The
// south face's flux fs comes in from the cell below (its north face, the same
// operation on the same operands); the north face's goes out through fn.
// Writes the level-0 inner arrays of `mode` and returns the scaled |R^p|,
// |R^c| through mp, mc.
template <typename T>
__device__ inline void res_cell(const Phys& ph, Solve<T>& S, int mode, int idx, int j, const Nb& q, const ResIn& a,
                                const FaceFlux& fs, FaceFlux& fn_out, double& mp, double& mc) {
    const double h = S.h, h2t = h * h / S.tau;
    Level<T>& L0 = S.lv[0];
    const double rP = rho_of(ph, a.cP), rN = rho_of(ph, a.cnP);
    double Rp = h2t * a.phiP * (rP - rN);
    double Rc = h2t * a.phiP * (rP * a.cP - rN * a.cnP);
    // east face: interior, or the seawater boundary
    const FaceFlux fe = flux_face<false>(ph, h, a.pP, a.pE, a.cP, a.cE, a.txP, a.wxP);
    const FaceFlux fr = flux_right(ph, -1.0 + (j + 0.5) * h, a.pP, a.cP, a.txP, a.wxP);
    Rp += q.he ? fe.M : fr.M;
    Rc += q.he ? fe.F : fr.F;
    // west face: interior (flux out of the west neighbour), or recharge
    const FaceFlux fw = flux_face<false>(ph, h, a.pW, a.pP, a.cW, a.cP, a.txW, a.wxW);
    const FaceFlux fl = flux_left(ph, h, S.q, a.cP, a.phiP);
    Rp += q.hw ? -fw.M : fl.M;
    Rc += q.hw ? -fw.F : fl.F;
    // north face (the top is impermeable)
    const FaceFlux fn = flux_face<true>(ph, h, a.pP, a.pN, a.cP, a.cN, a.tyP, a.wyP);
    fn_out = fn;
    Rp += q.hn ? fn.M : 0.0;
    Rc += q.hn ? fn.F : 0.0;
    // south face (the bottom is impermeable)
    Rp -= q.hs ? fs.M : 0.0;
    Rc -= q.hs ? fs.F : 0.0;
    if (mode == 0) {
        const int ps = pidx(idx - j * S.nx, j, S.nx);  // pressure cycle: colour-split
        L0.te[ps] = (T)(q.he ? fe.lam : fr.lam);
        L0.tn[ps] = (T)(q.hn ? fn.lam : 0.0);
        L0.b[ps] = (T)(-Rp);
        L0.x[ps] = (T)0;
        mp = nanmax(mp, fabs(Rp * a.sc));
    } else if (mode == 2) {
        S.rout_p[idx] = Rp;
        S.rout_c[idx] = Rc;
    } else {
        mp = nanmax(mp, fabs(Rp * a.sc));
        L0.mx[idx] = (T)(q.he ? fe.M : 0.0);
        L0.dx[idx] = (T)(q.he ? fe.dif : 0.0);
        L0.my[idx] = (T)(q.hn ? fn.M : 0.0);
        L0.dy[idx] = (T)(q.hn ? fn.dif : 0.0);
        if (!q.he) { L0.dr[j] = (T)fr.dif; L0.mr[j] = (T)fr.M; }
        if (!q.hw) { L0.dl[j] = (T)fl.dif; L0.ml[j] = (T)(-fl.M); }
        L0.acc[idx] = (T)(h2t * a.phiP * rN);
        L0.b[idx] = (T)(-(Rc - a.cP * Rp));
        L0.x[idx] = (T)0;
    }
    mc = nanmax(mc, fabs(Rc * a.sc));
}

// The rows of one residual pass (see residual_pass).  kFields: the face
// coefficients and the norm scale formed from K and phi (5 FP64 loads per
// cell instead of 9, and three FP64 divisions), with the same operations as
// the fields kernel's stored ones, so both variants give the same bits.
template <bool kFields, typename T>
__device__ inline void residual_rows(const Phys& ph, Solve<T>& S, int mode, double& mp, double& mc) {
    const int nx = S.nx, ny = S.ny;
    const int bs = ClusterTeam::size(), rk = ClusterTeam::rank();
    const int cw = nx < bs ? nx : bs;  // both powers of two
    const int G = bs / cw;
    const int band = (ny + G - 1) / G;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = rk / cw, ci = rk - g * cw;
    const int j0 = g * band;
    for (int cx = 0; cx < nx; cx += cw) {
        const int i = cx + ci;
        // rows below and at the start of the band (clamped into the grid)
        const int jb = j0 < ny ? j0 : ny - 1;
        const int js = jb > 0 ? jb - 1 : jb;
        double pS = S.p[js * nx + i], cS = S.c[js * nx + i];
        double pP = S.p[jb * nx + i], cP = S.c[jb * nx + i];
        double KP = 0.0, fP = 0.0, tyS = 0.0, wyS = 0.0;
        if constexpr (kFields) {
            KP = S.K[jb * nx + i];
            fP = S.phi[jb * nx + i];
            if (jb > 0) {  // the first row's south face (none at j = 0)
                const double Ks = S.K[js * nx + i], phs = S.phi[js * nx + i];
                const FacePair fy = face_pair(ph, Ks, KP, phs, fP);
                tyS = fy.t;
                wyS = fy.w;
            }
        } else {
            tyS = S.ty[js * nx + i];
            wyS = S.wy[js * nx + i];
        }
        // the flux through the south face of the band's first row; every
        // later row takes it from the row below
        FaceFlux fs = flux_face<true>(ph, S.h, pS, pP, cS, cP, tyS, wyS);
        for (int t = 0; t < band; ++t) {  // the same trip count in every lane (shuffles)
            const int j = j0 + t;
            const bool active = j < ny;
            const int jc = active ? j : ny - 1;
            const Nb q(i, jc, nx, ny);
            const int idx = q.idx;
            ResIn a;
            a.pP = pP; a.cP = cP;
            a.pN = S.p[q.n]; a.cN = S.c[q.n];
            a.cnP = S.cn[idx];
            // neighbours in x: adjacent lanes, or memory at the wavefront's ends
            double pEm = 0.0, cEm = 0.0, pWm = 0.0, cWm = 0.0, txWm = 0.0, wxWm = 0.0;
            double KN = 0.0, fN = 0.0;
            if constexpr (kFields) {
                KN = S.K[q.n];
                fN = S.phi[q.n];
                double KEm = 0.0, fEm = 0.0;
                if (lane == kWave - 1) { pEm = S.p[q.e]; cEm = S.c[q.e]; KEm = S.K[q.e]; fEm = S.phi[q.e]; }
                if (lane == 0) { pWm = S.p[q.w]; cWm = S.c[q.w]; txWm = S.tx[q.w]; wxWm = S.wx[q.w]; }
                const double KEs = __shfl_down(KP, 1, kWave), fEs = __shfl_down(fP, 1, kWave);
                const double KE = lane == kWave - 1 ? KEm : KEs, fE = lane == kWave - 1 ? fEm : fEs;
                a.phiP = fP;
                const FacePair fx = face_pair(ph, KP, q.he ? KE : KP, fP, q.he ? fE : fP);
                const FacePair fy = face_pair(ph, KP, KN, fP, fN);
                a.txP = q.he ? fx.t : 2.0 * fx.t;
                a.wxP = q.he ? fx.w : 2.0 * fx.w;
                a.tyP = q.hn ? fy.t : 0.0;
                a.wyP = q.hn ? fy.w : 0.0;
                a.sc = res_scale(ph, S.tau, S.h, fP);
            } else {
                a.phiP = S.phi[idx];
                a.txP = S.tx[idx]; a.wxP = S.wx[idx]; a.tyP = S.ty[idx]; a.wyP = S.wy[idx];
                a.sc = S.isc[idx];
                if (lane == kWave - 1) { pEm = S.p[q.e]; cEm = S.c[q.e]; }
                if (lane == 0) { pWm = S.p[q.w]; cWm = S.c[q.w]; txWm = S.tx[q.w]; wxWm = S.wx[q.w]; }
            }
            const double pEs = __shfl_down(pP, 1, kWave), cEs = __shfl_down(cP, 1, kWave);
            const double pWs = __shfl_up(pP, 1, kWave), cWs = __shfl_up(cP, 1, kWave);
            const double txWs = __shfl_up(a.txP, 1, kWave), wxWs = __shfl_up(a.wxP, 1, kWave);
            a.pE = lane == kWave - 1 ? pEm : pEs;
            a.cE = lane == kWave - 1 ? cEm : cEs;
            a.pW = lane == 0 ? pWm : pWs;
            a.cW = lane == 0 ? cWm : cWs;
            a.txW = lane == 0 ? txWm : txWs;
            a.wxW = lane == 0 ? wxWm : wxWs;
            FaceFlux fn = fs;
            if (active) res_cell(ph, S, mode, idx, j, q, a, fs, fn, mp, mc);
            // carry up one row
            fs = fn;
            pP = a.pN; cP = a.cN;
            KP = KN; fP = fN;
        }
    }
}

// mode 0: R^p and R^c, pressure coefficients te/tn at level 0, and the
//         scaled max norms (block max).
// mode 1: the salt defect S = R^c - c R^p with the transport coefficients
//         at level 0.
// mode 2: R^p and R^c into S.rout_p, S.rout_c (the residual entry point).
// Thread layout: lanes along x (cw = min(nx, blockDim) columns), the
// blockDim / cw row groups each march up their own band of rows.  A cell
// takes p and c of the rows below and above from the registers of the
// previous row and a load of the next one, and its east and west
// neighbours' values from the adjacent lanes (one-lane loads only at the
// ends of a wavefront): 9 full loads per cell instead of 21.  Grids of at
// least HENRY_RES_FIELDS_NX columns form the face coefficients from K and
// phi instead (their passes are bound by bandwidth); on smaller ones, whose
// passes wait on load latency, the divisions would lengthen the wait.
// The row bands are spread over all threads of the cluster; mode 0 ends
// with the cluster-wide norms, mode 1 with a cluster barrier only.
template <typename T>
__device__ void residual_pass(const Phys& ph, Solve<T>& S, int mode, double* red, double& np_out, double& nc_out,
                              PhaseClock* pcx = nullptr) {
    double mp = 0.0, mc = 0.0;
    if (HENRY_RES_FIELDS_NX > 0 && S.nx >= HENRY_RES_FIELDS_NX) residual_rows<true>(ph, S, mode, mp, mc);
    else residual_rows<false>(ph, S, mode, mp, mc);
    if (pcx) pcx->tick(mode == 0 ? 23 : 21);
    cluster_max2(mp, mc, red, np_out, nc_out);
    __syncthreads();
}

// ------------------------------------------------------------------ coefficient coarsening
// One level of each hierarchy from the level below it (Team loops; the
// caller synchronises the team before the level is read).
template <typename T, class Team, int ASF, int ASC, int KB>
__device__ inline void coarsen_pressure_level_kb(const LV<T, ASF>& F, const LV<T, ASC>& C) {
    const int nc = C.nx * C.ny;
    const int sx = log2i(C.nx);
    const int ts = Team::size();
    for (int k0 = Team::rank(); k0 < nc; k0 += KB * ts) {
        T e0[KB], e1[KB], n0[KB], n1[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int k = k0 + u * ts;
            const int idx = k < nc ? k : 0;
            int I, J;  // colour-split layout on both levels
            pcell(idx, C.nx, sx, I, J);
            e0[u] = F.te[pidx(2 * I + 1, 2 * J, F.nx)];
            e1[u] = F.te[pidx(2 * I + 1, 2 * J + 1, F.nx)];
            n0[u] = F.tn[pidx(2 * I, 2 * J + 1, F.nx)];
            n1[u] = F.tn[pidx(2 * I + 1, 2 * J + 1, F.nx)];
        }
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int k = k0 + u * ts;
            if (k < nc) {
                C.te[k] = (T)0.5 * (e0[u] + e1[u]);
                C.tn[k] = (T)0.5 * (n0[u] + n1[u]);
            }
        }
    }
}

template <typename T, class Team, int ASF, int ASC>
__device__ void coarsen_pressure_level(const Level<T>& F0, Level<T>& C0) {
    const LV<T, ASF> F(F0);
    const LV<T, ASC> C(C0);
    if (kTBatch > 1 && ASF == 1 && C.nx * C.ny > Team::size())
        coarsen_pressure_level_kb<T, Team, ASF, ASC, kTBatch>(F, C);
    else coarsen_pressure_level_kb<T, Team, ASF, ASC, 1>(F, C);
}

template <typename T, class Team, int ASF, int ASC, int KB>
__device__ inline void coarsen_transport_level_kb(const LV<T, ASF>& F, const LV<T, ASC>& C) {
    const int nc = C.nx * C.ny;
    const int sx = log2i(C.nx);
    const int ts = Team::size();
    for (int k0 = Team::rank(); k0 < nc; k0 += KB * ts) {
        T a00[KB], a01[KB], a10[KB], a11[KB], mx0[KB], mx1[KB], dx0[KB], dx1[KB], my0[KB], my1[KB], dy0[KB],
            dy1[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int k = k0 + u * ts;
            const int idx = k < nc ? k : 0;
            const int I = idx & (C.nx - 1), J = idx >> sx;
            const int f0 = (2 * J) * F.nx + 2 * I, f1 = f0 + F.nx;
            a00[u] = F.acc[f0]; a01[u] = F.acc[f0 + 1]; a10[u] = F.acc[f1]; a11[u] = F.acc[f1 + 1];
            mx0[u] = F.mx[f0 + 1]; mx1[u] = F.mx[f1 + 1]; dx0[u] = F.dx[f0 + 1]; dx1[u] = F.dx[f1 + 1];
            my0[u] = F.my[f1]; my1[u] = F.my[f1 + 1]; dy0[u] = F.dy[f1]; dy1[u] = F.dy[f1 + 1];
        }
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int k = k0 + u * ts;
            if (k < nc) {
                const int I = k & (C.nx - 1), J = k >> sx;
                C.acc[k] = (a00[u] + a01[u]) + (a10[u] + a11[u]);
                // mass fluxes through the two fine faces add; diffusion
                // transmissibilities (length/distance = 1 on every level) average
                C.mx[k] = (I + 1 < C.nx) ? mx0[u] + mx1[u] : (T)0;
                C.dx[k] = (I + 1 < C.nx) ? (T)0.5 * (dx0[u] + dx1[u]) : (T)0;
                C.my[k] = (J + 1 < C.ny) ? my0[u] + my1[u] : (T)0;
                C.dy[k] = (J + 1 < C.ny) ? (T)0.5 * (dy0[u] + dy1[u]) : (T)0;
            }
        }
    }
    for (int J = Team::rank(); J < C.ny; J += ts) {
        C.dl[J] = (T)0.5 * (F.dl[2 * J] + F.dl[2 * J + 1]);
        C.dr[J] = (T)0.5 * (F.dr[2 * J] + F.dr[2 * J + 1]);
        C.mr[J] = F.mr[2 * J] + F.mr[2 * J + 1];
        C.ml[J] = F.ml[2 * J] + F.ml[2 * J + 1];
    }
}

template <typename T, class Team, int ASF, int ASC>
__device__ void coarsen_transport_level(const Level<T>& F0, Level<T>& C0) {
    const LV<T, ASF> F(F0);
    const LV<T, ASC> C(C0);
    if (kTBatch > 1 && ASF == 1 && C.nx * C.ny > Team::size())
        coarsen_transport_level_kb<T, Team, ASF, ASC, kTBatch>(F, C);
    else coarsen_transport_level_kb<T, Team, ASF, ASC, 1>(F, C);
}

template <typename T, bool kTransport, class Team, int ASF, int ASC>
__device__ void coarsen_level(const Level<T>& F, Level<T>& C) {
    if constexpr (kTransport) coarsen_transport_level<T, Team, ASF, ASC>(F, C);
    else coarsen_pressure_level<T, Team, ASF, ASC>(F, C);
}

// Re-discretised coarse coefficients.  The cluster forms levels 1 .. lc
// (from cluster levels; level lc into its global copy when the leader runs
// it in LDS; no barrier after the last, whose next reader, the leader's
// part of the V-cycle, comes after the restriction's barrier).
template <typename T, bool kTransport>
__device__ void coarsen_cluster(Solve<T>& S) {
    for (int l = 1; l <= S.lc; ++l) {
        if (l > 1) ClusterTeam::sync();
        coarsen_level<T, kTransport, ClusterTeam, 1, 1>(S.lv[l - 1], (S.hand && l == S.lc) ? S.hg : S.lv[l]);
    }
}

// Levels `from` .. L-1, run by the leader alone: its workgroup forms the
// levels whose finer neighbour is in global memory or in the workgroup's
// part of LDS, wavefront 0 the rest (LDS levels, from LDS levels).
template <typename T, bool kTransport>
__device__ void coarsen_leader(Solve<T>& S, int from) {
    const int lw = S.lds_from, lb = S.lb;
    for (int l = from > 1 ? from : 1; l < S.L && l <= lw; ++l) {
        if (l < lb) coarsen_level<T, kTransport, BlockTeam, 1, 1>(S.lv[l - 1], S.lv[l]);
        else if (l == lb) coarsen_level<T, kTransport, BlockTeam, 1, 3>(S.lv[l - 1], S.lv[l]);
        else coarsen_level<T, kTransport, BlockTeam, 3, 3>(S.lv[l - 1], S.lv[l]);
        __syncthreads();
    }
    if (threadIdx.x < kWave) {
        for (int l = (from > lw + 1 ? from : lw + 1); l < S.L; ++l) {
            coarsen_level<T, kTransport, WaveTeam, 3, 3>(S.lv[l - 1], S.lv[l]);
            WaveTeam::sync();
        }
    }
    __syncthreads();
}

template <typename T, bool kTransport>
__device__ void handoff_in(Solve<T>& S);

// Every level, complete on return (the adjoint's transposed solves reuse
// the coefficients over several cycles; a level handed from the cluster to
// the leader's LDS is copied there first).
template <typename T, bool kTransport>
__device__ void coarsen(Solve<T>& S) {
    coarsen_cluster<T, kTransport>(S);
    if (S.lc > 0) ClusterTeam::sync();
    if (g_cl.member == 0) {
        if (S.hand) {
            handoff_in<T, kTransport>(S);
            __syncthreads();
        }
        coarsen_leader<T, kTransport>(S, S.lc + 1);
    }
    ClusterTeam::sync();
}

template <typename T>
__device__ void coarsen_pressure(Solve<T>& S) { coarsen<T, false>(S); }

template <typename T>
__device__ void coarsen_transport(Solve<T>& S) { coarsen<T, true>(S); }

// ------------------------------------------------------------------ stencils
// Pressure: (A x)_P = diag x_P - sum_nb t_nb x_nb; te of the last column is
// the seawater Dirichlet coefficient (diagonal only); tn of the top row is 0.
// The operations below load every operand from a clamped (always valid)
// index and zero the missing neighbours afterwards: loads under boundary
// branches would each wait for their own round trip.
template <typename T>
struct Stencil { T d, w, e, s, n; };


template <class V, class Q, typename T = typename V::value_type>
__device__ inline Stencil<T> pstencil(const V& v, const Q& q) {
    Stencil<T> st;
    const T te = v.te[q.idx], tw = v.te[q.w], tn = v.tn[q.idx], ts = v.tn[q.s];
    st.e = q.he ? te : (T)0;
    st.w = q.hw ? tw : (T)0;
    st.n = tn;
    st.s = q.hs ? ts : (T)0;
    st.d = te + st.w + st.n + st.s;
    return st;
}

// Transport (non-conservative upwind form): a neighbour couples only
// through inflow across the shared face plus diffusion; the diagonal is
// the stored mass plus the sum of the couplings and the boundary inflow /
// diffusion terms.  mx/my are the mass fluxes leaving (i,j) east/north.
template <typename T>
__device__ inline T pos(T a) { return a > (T)0 ? a : (T)0; }

template <class V, typename T = typename V::value_type>
__device__ inline Stencil<T> cstencil(const V& v, const Nb& q, int j) {
    Stencil<T> st;
    const T a = v.acc[q.idx];
    const T mE = v.mx[q.idx], dE = v.dx[q.idx], mW = v.mx[q.w], dW = v.dx[q.w];
    const T mN = v.my[q.idx], dN = v.dy[q.idx], mS = v.my[q.s], dS = v.dy[q.s];
    const T bE = pos(-v.mr[j]) + v.dr[j], bW = v.dl[j] + v.ml[j];
    T d = a;
    st.e = q.he ? pos(-mE) + dE : (T)0;
    d += q.he ? st.e : bE;
    st.w = q.hw ? pos(mW) + dW : (T)0;
    d += q.hw ? st.w : bW;
    st.n = q.hn ? pos(-mN) + dN : (T)0;
    d += st.n;
    st.s = q.hs ? pos(mS) + dS : (T)0;
    d += st.s;
    st.d = d;
    return st;
}

// Transpose of the transport operator (adjoint solves): a cell couples to
// a neighbour with that neighbour's coupling to it; the diagonal is the same.
template <class V, typename T = typename V::value_type>
__device__ inline Stencil<T> cstencil_t(const V& v, const Nb& q, int j) {
    Stencil<T> st;
    const T a = v.acc[q.idx];
    const T mE = v.mx[q.idx], dE = v.dx[q.idx], mW = v.mx[q.w], dW = v.dx[q.w];
    const T mN = v.my[q.idx], dN = v.dy[q.idx], mS = v.my[q.s], dS = v.dy[q.s];
    const T bE = pos(-v.mr[j]) + v.dr[j], bW = v.dl[j] + v.ml[j];
    T d = a;
    d += q.he ? pos(-mE) + dE : bE;
    st.e = q.he ? pos(mE) + dE : (T)0;
    d += q.hw ? pos(mW) + dW : bW;
    st.w = q.hw ? pos(-mW) + dW : (T)0;
    d += q.hn ? pos(-mN) + dN : (T)0;
    st.n = q.hn ? pos(mN) + dN : (T)0;
    d += q.hs ? pos(mS) + dS : (T)0;
    st.s = q.hs ? pos(-mS) + dS : (T)0;
    st.d = d;
    return st;
}

template <typename T, bool kTransport, bool kTrans = false, class V, class Q>
__device__ inline Stencil<T> stencil(const V& v, const Q& q, int j) {
    if constexpr (kTransport) {
        if constexpr (kTrans) return cstencil_t(v, q, j);
        else return cstencil(v, q, j);
    } else {
        return pstencil(v, q);
    }
}

// ------------------------------------------------------------------ grid transfer
// Prolongation: bilinear with constant extrapolation at the boundary,
// x_f += P x_c.  Restriction is its exact transpose (full weighting with
// weights (1,3,3,1)/4 per direction, boundary weights folded in).
// kSplit: both levels in the colour-split layout (pressure cycle).
template <typename T, class Team, int ASC, int ASF, bool kSplit, int KB>
__device__ inline void prolong_add_kb(const LV<T, ASC>& C, const LV<T, ASF>& F) {
    const int n = F.nx * F.ny;
    const int sx = log2i(F.nx);
    const int ts = Team::size();
    auto cat = [&](int I, int J) { return kSplit ? pidx(I, J, C.nx) : J * C.nx + I; };
    for (int k0 = Team::rank(); k0 < n; k0 += KB * ts) {
        T v[KB], xf[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int k = k0 + u * ts;
            const int idx = k < n ? k : 0;
            int i, j;
            if constexpr (kSplit) pcell(idx, F.nx, sx, i, j);
            else { i = idx & (F.nx - 1); j = idx >> sx; }
            const int I = i >> 1, J = j >> 1;
            const int In = (i & 1) ? min(I + 1, C.nx - 1) : max(I - 1, 0);
            const int Jn = (j & 1) ? min(J + 1, C.ny - 1) : max(J - 1, 0);
            v[u] = (T)0.5625 * C.x[cat(I, J)] + (T)0.1875 * (C.x[cat(In, J)] + C.x[cat(I, Jn)]) +
                   (T)0.0625 * C.x[cat(In, Jn)];
            xf[u] = F.x[idx];
        }
#pragma unroll
        for (int u = 0; u < KB; ++u)
            if (k0 + u * ts < n) F.x[k0 + u * ts] = xf[u] + v[u];
    }
}

// Prolongation: bilinear with constant extrapolation at the boundary,
// x_f += P x_c.  Restriction is its exact transpose (full weighting with
// weights (1,3,3,1)/4 per direction, boundary weights folded in).
// kSplit: both levels in the colour-split layout (pressure cycle).
template <typename T, class Team = BlockTeam, int ASC = 0, int ASF = 0, bool kSplit = false>
__device__ void prolong_add(const Level<T>& C0, Level<T>& F0) {
    const LV<T, ASC> C(C0);
    const LV<T, ASF> F(F0);
    if (kTBatch > 1 && ASF == 1 && F.nx * F.ny > Team::size())
        prolong_add_kb<T, Team, ASC, ASF, kSplit, kTBatch>(C, F);
    else prolong_add_kb<T, Team, ASC, ASF, kSplit, 1>(C, F);
}

// 1D restriction weight of fine index I2 = 2I - 1 + a (a = 0..3) for coarse
// index I of n: (1,3,3,1)/4, with the boundary ghost weight folded in.
__device__ inline float rweight(int I, int n, int a) {
    float w = (a == 0 || a == 3) ? 0.25f : 0.75f;
    if (a == 1 && I == 0) w += 0.25f;
    if (a == 2 && I == n - 1) w += 0.25f;
    return w;
}

template <typename T, class Team, int ASF, int ASC, bool kSplit, int KB>
__device__ inline void restrict_residual_kb(const LV<T, ASF>& F, const LV<T, ASC>& C) {
    const int n = C.nx * C.ny;
    const int sx = log2i(C.nx);
    const int ts = Team::size();
    // fine cells whose residual the level residual left out (zero): black
    // cells (aq + bq odd) in the pressure cycle, odd rows (bq even) in the
    // transport cycle
    auto live = [](int aq, int bq) { return kSplit ? ((aq + bq) & 1) == 0 : (bq & 1) == 1; };
    for (int k0 = Team::rank(); k0 < n; k0 += KB * ts) {
        T rv[KB][4][4];
        int cI[KB], cJ[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int k = k0 + u * ts;
            const int idx = k < n ? k : 0;
            int I, J;
            if constexpr (kSplit) pcell(idx, C.nx, sx, I, J);
            else { I = idx & (C.nx - 1); J = idx >> sx; }
            cI[u] = I; cJ[u] = J;
            // fine rows / columns outside the level get weight 0 (their load
            // is clamped to a valid cell)
#pragma unroll
            for (int bq = 0; bq < 4; ++bq) {
                const int jf = min(max(2 * J - 1 + bq, 0), F.ny - 1);
#pragma unroll
                for (int aq = 0; aq < 4; ++aq) {
                    const int ifn = min(max(2 * I - 1 + aq, 0), F.nx - 1);
                    rv[u][bq][aq] = live(aq, bq) ? F.r[kSplit ? pidx(ifn, jf, F.nx) : jf * F.nx + ifn] : (T)0;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int I = cI[u], J = cJ[u];
            // terms outside the level are selected away, not weighted by
            // zero: their clamped load may land on a cell whose residual was
            // never written
            T s = (T)0;
#pragma unroll
            for (int bq = 0; bq < 4; ++bq) {
                const int jf = 2 * J - 1 + bq;
                const bool jin = jf >= 0 && jf < F.ny;
                T row = (T)0;
#pragma unroll
                for (int aq = 0; aq < 4; ++aq) {
                    const int ifn = 2 * I - 1 + aq;
                    const bool iin = ifn >= 0 && ifn < F.nx;
                    row += iin ? (T)rweight(I, C.nx, aq) * rv[u][bq][aq] : (T)0;
                }
                s += jin ? (T)rweight(J, C.ny, bq) * row : (T)0;
            }
            const int k = k0 + u * ts;
            if (k < n) {
                C.b[k] = s;
                C.x[k] = (T)0;
            }
        }
    }
}

template <typename T, class Team = BlockTeam, int ASF = 0, int ASC = 0, bool kSplit = false>
__device__ void restrict_residual(const Level<T>& F0, Level<T>& C0) {
    const LV<T, ASF> F(F0);
    const LV<T, ASC> C(C0);
    if (kTBatch > 1 && ASF == 1 && C.nx * C.ny > Team::size())
        restrict_residual_kb<T, Team, ASF, ASC, kSplit, kTBatch>(F, C);
    else restrict_residual_kb<T, Team, ASF, ASC, kSplit, 1>(F, C);
}

// r = b - A x on one level after the pre-smoothing (operands of kRBatch
// cells gathered first), on the cells smoothed first only: the cells the
// smoother updated last (black cells of the red-black sweep, odd rows of the
// zebra x-line sweep) satisfy their equations with the current neighbours,
// so their residual is zero to rounding, and the restriction skips them.
// Pressure: red cells, the first half of each row of the colour-split
// layout; transport: the even rows.
constexpr int kRBatch = 2;
template <typename T, bool kTransport, bool kTrans, class Team, int AS, int KB>
__device__ inline void level_residual_kb(const LV<T, AS>& v) {
    const int half = v.nx >> 1;
    const int n = kTransport ? v.nx * ((v.ny + 1) >> 1) : half * v.ny;  // live cells
    const int ts = Team::size();
    const int sx = log2i(v.nx);
    for (int k0 = Team::rank(); k0 < n; k0 += KB * ts) {
        T res[KB];
        int at[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int k = k0 + u * ts;
            const int kk = k < n ? k : 0;
            int i, j, idx;
            if constexpr (kTransport) {
                i = kk & (v.nx - 1); j = 2 * (kk >> sx);
                idx = j * v.nx + i;
            } else {
                j = kk >> (sx - 1);
                const int kr = kk & (half - 1);
                i = 2 * kr + (j & 1);
                idx = j * v.nx + kr;
            }
            at[u] = idx;
            using Q = typename std::conditional<kTransport, Nb, NbS>::type;
            const Q q(i, j, v.nx, v.ny);
            const Stencil<T> st = stencil<T, kTransport, kTrans>(v, q, j);
            const T xP = v.x[idx], xW = v.x[q.w], xE = v.x[q.e], xS = v.x[q.s], xN = v.x[q.n];
            const T bP = v.b[idx];
            // missing neighbours have zero couplings
            T ax = st.d * xP;
            ax -= st.w * xW;
            ax -= st.e * xE;
            ax -= st.s * xS;
            ax -= st.n * xN;
            res[u] = bP - ax;
        }
#pragma unroll
        for (int u = 0; u < KB; ++u)
            if (k0 + u * ts < n) v.r[at[u]] = res[u];
    }
}

// One cell per thread when one pass of the team covers the live cells.
template <typename T, bool kTransport, bool kTrans = false, class Team = BlockTeam, int AS = 0>
__device__ void level_residual(Level<T>& v0) {
    const LV<T, AS> v(v0);
    const int n = kTransport ? v.nx * ((v.ny + 1) >> 1) : (v.nx >> 1) * v.ny;
    if (n <= Team::size()) level_residual_kb<T, kTransport, kTrans, Team, AS, 1>(v);
    else level_residual_kb<T, kTransport, kTrans, Team, AS, kRBatch>(v);
}

// ------------------------------------------------------------------ smoothers
// Red-black Gauss-Seidel (pressure): colour (i + j) & 1.  Cells of one
// colour are independent; each thread gathers the operands of kBatch cells
// before it writes any of them, so their loads are in flight together.
constexpr int kBatch = 4;

// One half-sweep (colour col) with KB cells gathered per thread.
template <typename T, class Team, int AS, int KB>
__device__ inline void rbgs_colour(const LV<T, AS>& v, int col) {
    const int nx = v.nx, ny = v.ny;
    const int half = nx >> 1;  // nx is even on every level
    const int sh = log2i(half);
    const int m = half * ny;
    const auto te = v.te;
    const auto tn = v.tn;
    const auto b = v.b;
    const auto x = v.x;
    for (int k0 = Team::rank(); k0 < m; k0 += KB * Team::size()) {
        T num[KB], den[KB];
        int at[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int k = k0 + u * Team::size();
            const int kk = k < m ? k : 0;
            const int j = kk >> sh;
            const int i = 2 * (kk & (half - 1)) + ((j + col) & 1);
            const NbS q(i, j, nx, ny);  // q.idx = j nx + col half + (kk mod half)
            at[u] = k < m ? q.idx : -1;
            const T tE = te[q.idx], tWl = te[q.w], tN = tn[q.idx], tSl = tn[q.s];
            const T xW = x[q.w], xE = x[q.e], xS = x[q.s], xN = x[q.n];
            const T bP = b[q.idx];
            const T tW = q.hw ? tWl : (T)0, tS = q.hs ? tSl : (T)0;
            const T tEc = q.he ? tE : (T)0;  // the seawater coefficient is diagonal only
            T a = bP;
            a += tW * xW;
            a += tEc * xE;
            a += tS * xS;
            a += tN * xN;
            num[u] = a;
            den[u] = tE + tW + tN + tS;
        }
#pragma unroll
        for (int u = 0; u < KB; ++u)
            if (at[u] >= 0) x[at[u]] = qdiv(num[u], den[u]);
    }
}

// A colour that one pass of the team covers takes one cell per thread
// (the coarse levels: a fixed batch would issue the loads and arithmetic of
// kBatch cells per lane for one useful cell or none); larger ones take
// kBatch.  The cells and their arithmetic are the same either way.
template <typename T, class Team = BlockTeam, int AS = 0>
__device__ void rbgs(Level<T>& v0, int sweeps) {
    const LV<T, AS> v(v0);
    const bool one = (v.nx >> 1) * v.ny <= Team::size();
    for (int s = 0; s < sweeps; ++s)
        for (int col = 0; col < 2; ++col) {
            if (one) rbgs_colour<T, Team, AS, 1>(v, col);
            else rbgs_colour<T, Team, AS, kBatch>(v, col);
            Team::sync();
        }
}

// Segmented line solve.  Every line of one colour is split over T lanes of
// one wavefront (T a power of two dividing 64), lane t owning the m = len/T
// consecutive rows t*m .. t*m+m-1 of the line.  The lane's last row is an
// interface unknown iota_t; its m-1 interior rows are eliminated locally
// (Thomas, three right-hand sides: the line rhs and the unit couplings to
// iota_{t-1} and iota_t), which leaves a tridiagonal system in the T
// interface unknowns.  That reduced system is solved by parallel cyclic
// reduction across the T lanes with wavefront shuffles, then every lane
// back-substitutes its interior rows.  All coefficients live in registers;
// a colour of lines is one block-wide phase.
// MS = rows per lane (a power of two, 2 to 16, chosen by line_sweep); line
// lengths are powers of two, so TL = len/MS <= 64 lanes per line.
// Each instantiation is its own function, so the register budget of the
// long-line variants does not weigh on the short ones.
template <typename T, bool kXLine, bool kTrans, int MS, class Team, int AS>
__device__ __attribute__((noinline)) void line_sweep_m(Level<T>& v0, int col) {
    const LV<T, AS> v(v0);
    const int len = kXLine ? v.nx : v.ny;
    const int other = kXLine ? v.ny : v.nx;
    const int nlines = (other - col + 1) >> 1;
    const int m = MS;                   // rows per lane
    const int TL = len / m;             // lanes per line
    const int stl = log2i(TL);
    const int lane = threadIdx.x & (kWave - 1);
    const int t = lane & (TL - 1);
    const int need = nlines * TL;
    for (int base = 0; base < need; base += Team::size()) {
        const int g = base + Team::rank();
        const int li = g >> stl;
        const bool active = li < nlines;
        const int fixed = col + 2 * (active ? li : 0);
        // w (the response to iota_t) is zero above row m-2 before the back
        // substitution, so afterwards w[q] = w[m-2] * prod_{k=q}^{m-3} (-cp[k]):
        // it is carried as a running product instead of an array
        T cp[MS], y[MS], u[MS];
        T wlast = (T)0;
        T ar = (T)0, br = (T)1, cr = (T)0, dr = (T)0;
        // forward elimination of the interior rows, interface row kept aside
#pragma unroll
        for (int q = 0; q < MS; ++q) {
            if (q < m) {
                const int k = t * m + q;
                const int i = kXLine ? k : fixed, j = kXLine ? fixed : k;
                const Nb nb(i, j, v.nx, v.ny);
                const Stencil<T> st = stencil<T, true, kTrans>(v, nb, j);
                T rhs = v.b[nb.idx];
                T a, c;
                // off-line neighbours; missing ones have zero couplings
                if (kXLine) {
                    const T xS = v.x[nb.s], xN = v.x[nb.n];
                    rhs += st.s * xS;
                    rhs += st.n * xN;
                    a = -st.w; c = -st.e;
                } else {
                    const T xW = v.x[nb.w], xE = v.x[nb.e];
                    rhs += st.w * xW;
                    rhs += st.e * xE;
                    a = -st.s; c = -st.n;
                }
                if (q < m - 1) {
                    const T den = (q > 0) ? st.d - a * cp[q > 0 ? q - 1 : 0] : st.d;
                    const T inv = qdiv((T)1, den);
                    const T yprev = (q > 0) ? y[q > 0 ? q - 1 : 0] : (T)0;
                    const T uprev = (q > 0) ? u[q > 0 ? q - 1 : 0] : (T)0;
                    cp[q] = c * inv;
                    y[q] = (rhs - a * yprev) * inv;
                    u[q] = ((q == 0 ? -a : (T)0) - a * uprev) * inv;
                    if (q == m - 2) wlast = (-c - a * (T)0) * inv;
                } else {
                    ar = a; br = st.d; cr = c; dr = rhs;
                }
            }
        }
        // back substitution of the interior rows (coupling to iota_t: the
        // running product wrun, w[q] = 0 - cp[q] w[q + 1])
        T wrun = wlast;
#pragma unroll
        for (int q = MS - 2; q >= 0; --q) {
            if (q < m - 2) {
                y[q] -= cp[q] * y[q + 1];
                u[q] -= cp[q] * u[q + 1];
                wrun = (T)0 - cp[q] * wrun;
            }
        }
        // interior rows next to the interfaces
        T yL = (T)0, uL = (T)1, wL = (T)0;  // row before the interface (m == 1: iota_{t-1} itself)
        T yF = (T)0, uF = (T)0, wF = (T)1;  // first row of this lane (m == 1: iota_t itself)
#pragma unroll
        for (int q = 0; q < MS; ++q) {
            if (q == m - 2) { yL = y[q]; uL = u[q]; wL = wlast; }
        }
        if (m >= 2) { yF = y[0]; uF = u[0]; wF = m >= 2 ? wrun : (T)1; }
        // first row of the next lane of the same line
        const bool last = (t == TL - 1);
        const int src = last ? lane : lane + 1;
        T yN = __shfl(yF, src, kWave), uN = __shfl(uF, src, kWave), wN = __shfl(wF, src, kWave);
        if (last) { yN = (T)0; uN = (T)0; wN = (T)0; cr = (T)0; }
        T A = ar * uL;
        T B = br + ar * wL + cr * uN;
        T C = cr * wN;
        T D = dr - ar * yL - cr * yN;
        // parallel cyclic reduction over the TL interface equations
        for (int sft = 1; sft < TL; sft <<= 1) {
            const bool hasL = t >= sft, hasR = t + sft < TL;
            const int l = hasL ? lane - sft : lane, r = hasR ? lane + sft : lane;
            const T Al = __shfl(A, l, kWave), Bl = __shfl(B, l, kWave), Cl = __shfl(C, l, kWave),
                    Dl = __shfl(D, l, kWave);
            const T Ar = __shfl(A, r, kWave), Br = __shfl(B, r, kWave), Cr = __shfl(C, r, kWave),
                    Dr = __shfl(D, r, kWave);
            T nA = (T)0, nB = B, nC = (T)0, nD = D;
            if (hasL) {
                const T k1 = qdiv(A, Bl);
                nA = -Al * k1;
                nB -= Cl * k1;
                nD -= Dl * k1;
            }
            if (hasR) {
                const T k2 = qdiv(C, Br);
                nC = -Cr * k2;
                nB -= Ar * k2;
                nD -= Dr * k2;
            }
            A = nA; B = nB; C = nC; D = nD;
        }
        const T iota = qdiv(D, B);
        const T left0 = __shfl(iota, t > 0 ? lane - 1 : lane, kWave);
        const T left = t > 0 ? left0 : (T)0;
        if (active) {
            // rows from the bottom up, rebuilding w[q] as in the back substitution
            T wq = wlast;
#pragma unroll
            for (int q = MS - 1; q >= 0; --q) {
                if (q < m) {
                    const int k = t * m + q;
                    const int i = kXLine ? k : fixed, j = kXLine ? fixed : k;
                    if (q < m - 2) wq = (T)0 - cp[q] * wq;
                    v.x[j * v.nx + i] = (q < m - 1) ? y[q] + u[q] * left + wq * iota : iota;
                }
            }
        }
    }
    Team::sync();
}

// Rows per lane: x-lines take the fewest rows (at least two) that fit a
// line in one wavefront; y-lines of 64 to 256 rows take four, so that a
// wavefront holds two or more neighbouring columns and each of its loads
// touches half as many (or fewer) cache lines as with one column of strided
// rows.  The wavefront-team levels (at most 512 cells) have lines of at most
// 32 cells: two rows per lane.
// x-lines of 512 and 1024 cells on the cluster levels (one wavefront per
// line, MS = 8 or 16 rows per lane).  line_sweep_m gathers a lane's MS
// consecutive cells, so each of its load instructions touches 32 cache lines
// at 8 bytes each, and the lines are gone from L1 and L2 before the lane
// comes back for the rest of them.  Here the wavefront forms each row's
// coefficients (the same stencil arithmetic) from coalesced loads, 64
// consecutive cells per instruction, into its own LDS buffer, and each lane
// reads its segment back from there for the same elimination (results are
// bitwise those of line_sweep_m).  A 1024-cell row is staged in two halves
// of 512 (lanes 0-31 eliminate the first, 32-63 the second).  The buffers
// overlay the LDS levels, which are dead while the cluster runs its levels
// in the forward solve: every cycle's leader rebuilds them (coarse_coeffs)
// after the cluster's downward leg and is done with them before its upward
// leg.  The adjoint's transposed cycles keep them from cycle to cycle, so
// its kernel turns the staging off (g_cl.stage_waves = 0).  Padding of one
// element per segment keeps the segment reads free of bank conflicts (lane
// stride MS + 1).
constexpr int kStageCells = 512;
constexpr int kStageElems = kStageCells + kStageCells / 8;  // one pad per segment of >= 8 cells
template <typename T>
__host__ __device__ constexpr int64_t line_stage_bytes_per_wave() { return 4 * (int64_t)kStageElems * (int64_t)sizeof(T); }

template <typename T, bool kTrans, int MS>
__device__ __attribute__((noinline)) void line_sweep_x_staged(Level<T>& v0, int col) {
    static_assert(MS == 8 || MS == 16, "staged x-lines are 512 or 1024 cells");
    constexpr int NH = kWave * MS / kStageCells;  // halves of a row
    const LV<T, 1> v(v0);
    const int nlines = (v.ny - col + 1) >> 1;
    const int lane = threadIdx.x & (kWave - 1);
    T* buf = reinterpret_cast<T*>(g_cl.stage) + (int64_t)(threadIdx.x / kWave) * 4 * kStageElems;
    auto As = as_ptr<3>(buf);
    auto Cs = as_ptr<3>(buf + kStageElems);
    auto Ds = as_ptr<3>(buf + 2 * kStageElems);
    auto Rs = as_ptr<3>(buf + 3 * kStageElems);
    const int waves = ClusterTeam::size() / kWave, wrank = ClusterTeam::rank() / kWave;
    const int t = lane;
    for (int l0 = 0; l0 < nlines; l0 += waves) {  // the same trip count in every lane
        const int li = l0 + wrank;
        const bool active = li < nlines;
        const int j = col + 2 * (active ? li : 0);
        T cp[MS], y[MS], u[MS];
        T wlast = (T)0;
        T ar = (T)0, br = (T)1, cr = (T)0, dr = (T)0;
        for (int hh = 0; hh < NH; ++hh) {
            // coefficients of cells hh * 512 + r * 64 + lane, coalesced
#pragma unroll 2
            for (int r = 0; r < kStageCells / kWave; ++r) {
                const int kl = r * kWave + lane;
                const Nb nb(hh * kStageCells + kl, j, v.nx, v.ny);
                const Stencil<T> st = stencil<T, true, kTrans>(v, nb, j);
                T rhs = v.b[nb.idx];
                const T xS = v.x[nb.s], xN = v.x[nb.n];
                rhs += st.s * xS;
                rhs += st.n * xN;
                const int si = kl + kl / MS;
                As[si] = -st.w;
                Cs[si] = -st.e;
                Ds[si] = st.d;
                Rs[si] = rhs;
            }
            WaveTeam::sync();
            // forward elimination of the lanes whose segment lies in this half
            if (t * MS / kStageCells == hh) {
                const int s0 = (t * MS - hh * kStageCells) / MS * (MS + 1);
#pragma unroll
                for (int q = 0; q < MS; ++q) {
                    const T a = As[s0 + q], c = Cs[s0 + q], d = Ds[s0 + q], rhs = Rs[s0 + q];
                    if (q < MS - 1) {
                        const T den = (q > 0) ? d - a * cp[q > 0 ? q - 1 : 0] : d;
                        const T inv = qdiv((T)1, den);
                        const T yprev = (q > 0) ? y[q > 0 ? q - 1 : 0] : (T)0;
                        const T uprev = (q > 0) ? u[q > 0 ? q - 1 : 0] : (T)0;
                        cp[q] = c * inv;
                        y[q] = (rhs - a * yprev) * inv;
                        u[q] = ((q == 0 ? -a : (T)0) - a * uprev) * inv;
                        if (q == MS - 2) wlast = (-c - a * (T)0) * inv;
                    } else {
                        ar = a; br = d; cr = c; dr = rhs;
                    }
                }
            }
            WaveTeam::sync();  // the buffer is refilled by the next half or line
        }
        // back substitution of the interior rows (coupling to iota_t: the
        // running product wrun, w[q] = 0 - cp[q] w[q + 1])
        T wrun = wlast;
#pragma unroll
        for (int q = MS - 2; q >= 0; --q) {
            if (q < MS - 2) {
                y[q] -= cp[q] * y[q + 1];
                u[q] -= cp[q] * u[q + 1];
                wrun = (T)0 - cp[q] * wrun;
            }
        }
        const T yL = y[MS - 2], uL = u[MS - 2], wL = wlast;
        const T yF = y[0], uF = u[0], wF = wrun;
        // first row of the next lane of the same line
        const bool last = (t == kWave - 1);
        const int src = last ? lane : lane + 1;
        T yN = __shfl(yF, src, kWave), uN = __shfl(uF, src, kWave), wN = __shfl(wF, src, kWave);
        if (last) { yN = (T)0; uN = (T)0; wN = (T)0; cr = (T)0; }
        T A = ar * uL;
        T B = br + ar * wL + cr * uN;
        T C = cr * wN;
        T D = dr - ar * yL - cr * yN;
        // parallel cyclic reduction over the 64 interface equations
        for (int sft = 1; sft < kWave; sft <<= 1) {
            const bool hasL = t >= sft, hasR = t + sft < kWave;
            const int l = hasL ? lane - sft : lane, r = hasR ? lane + sft : lane;
            const T Al = __shfl(A, l, kWave), Bl = __shfl(B, l, kWave), Cl = __shfl(C, l, kWave),
                    Dl = __shfl(D, l, kWave);
            const T Ar = __shfl(A, r, kWave), Br = __shfl(B, r, kWave), Cr = __shfl(C, r, kWave),
                    Dr = __shfl(D, r, kWave);
            T nA = (T)0, nB = B, nC = (T)0, nD = D;
            if (hasL) {
                const T k1 = qdiv(A, Bl);
                nA = -Al * k1;
                nB -= Cl * k1;
                nD -= Dl * k1;
            }
            if (hasR) {
                const T k2 = qdiv(C, Br);
                nC = -Cr * k2;
                nB -= Ar * k2;
                nD -= Dr * k2;
            }
            A = nA; B = nB; C = nC; D = nD;
        }
        const T iota = qdiv(D, B);
        const T left0 = __shfl(iota, t > 0 ? lane - 1 : lane, kWave);
        const T left = t > 0 ? left0 : (T)0;
        if (active) {
            // rows from the bottom up, rebuilding w[q] as in the back substitution
            T wq = wlast;
#pragma unroll
            for (int q = MS - 1; q >= 0; --q) {
                if (q < MS - 2) wq = (T)0 - cp[q] * wq;
                v.x[j * v.nx + t * MS + q] = (q < MS - 1) ? y[q] + u[q] * left + wq * iota : iota;
            }
        }
    }
    ClusterTeam::sync();
}

template <typename T, bool kXLine, bool kTrans = false, class Team = BlockTeam, int AS = 0>
__device__ void line_sweep(Level<T>& v, int col) {
    const int len = kXLine ? v.nx : v.ny;  // 2 .. 1024, a power of two
    if constexpr (kXLine && AS == 1 && std::is_same<Team, ClusterTeam>::value) {
        if (len >= 512 && g_cl.K > 1 && (int)(blockDim.x / kWave) <= g_cl.stage_waves) {
            if (len == 512) line_sweep_x_staged<T, kTrans, 8>(v, col);
            else line_sweep_x_staged<T, kTrans, 16>(v, col);
            return;
        }
    }
    if constexpr (std::is_same<Team, WaveTeam>::value) {
        line_sweep_m<T, kXLine, kTrans, 2, Team, AS>(v, col);
    } else if constexpr (kXLine) {
        // rows of 64 and 128 cells: 16 or 32 lanes per line, so that a
        // wavefront solves two or four lines at once with fewer reduction
        // steps (128x64 group 188 -> 179 ms, 64x32 86 -> 80 ms)
        if (len < 64) line_sweep_m<T, kXLine, kTrans, 2, Team, AS>(v, col);
        else if (len <= 256) line_sweep_m<T, kXLine, kTrans, 4, Team, AS>(v, col);
        else if (len == 512) line_sweep_m<T, kXLine, kTrans, 8, Team, AS>(v, col);
        else line_sweep_m<T, kXLine, kTrans, 16, Team, AS>(v, col);
    } else {
        if (len < 64) line_sweep_m<T, kXLine, kTrans, 2, Team, AS>(v, col);
        else if (len <= 256) line_sweep_m<T, kXLine, kTrans, 4, Team, AS>(v, col);
        else line_sweep_m<T, kXLine, kTrans, 8, Team, AS>(v, col);
    }
}

// One zebra sweep in one direction: x-lines (even rows, then odd rows) or
// y-lines (even columns, then odd columns; a one-row level has only its
// x-line).  The transport V-cycle pre-smooths with x-lines; it post-smooths
// with y-lines on the coarse (LDS) levels, so every cycle relaxes along
// both directions.
template <typename T, bool kTrans = false, class Team = BlockTeam, int AS = 0>
__device__ void line_smooth(Level<T>& v, bool ylines) {
    if (ylines && v.ny > 1) {
        line_sweep<T, false, kTrans, Team, AS>(v, 0);
        line_sweep<T, false, kTrans, Team, AS>(v, 1);
    } else {
        line_sweep<T, true, kTrans, Team, AS>(v, 0);
        line_sweep<T, true, kTrans, Team, AS>(v, 1);
    }
}

// ------------------------------------------------------------------ V-cycles
// Downward leg on level l (address space AS; level l+1 in ASN): smooth,
// residual, restriction to level l+1.
template <typename T, bool kTransport, bool kTrans, class Team, int AS, int ASN>
__device__ void vdown(Solve<T>& S, int l) {
    Level<T>& v = S.lv[l];
    Level<T>& c = (S.hand && l + 1 == S.lc) ? S.hg : S.lv[l + 1];
    if constexpr (kTransport) line_smooth<T, kTrans, Team, AS>(v, false);
    else rbgs<T, Team, AS>(v, 2);
    level_residual<T, kTransport, kTrans, Team, AS>(v);
    Team::sync();
    restrict_residual<T, Team, AS, ASN, !kTransport>(v, c);
    Team::sync();
}

// Upward leg on level l: prolongation from level l+1, smooth.  The
// transport post-smoothing takes y-lines on the levels wavefront 0 runs and
// x-lines on the larger ones: in global memory a y-line sweep costs about
// three x-line sweeps (the rows of a column are a cache line apart), and
// the outer iteration counts stay the same (1.69 per step on 256x128/800
// either way); the cycle still relaxes along y on every level of 512 cells
// or fewer.
template <typename T, bool kTransport, bool kTrans, class Team, int AS, int ASN>
__device__ void vup(Solve<T>& S, int l) {
    Level<T>& v = S.lv[l];
    const Level<T>& c = (S.hand && l + 1 == S.lc) ? S.hg : S.lv[l + 1];
    prolong_add<T, Team, ASN, AS, !kTransport>(c, v);
    Team::sync();
    if constexpr (kTransport) line_smooth<T, kTrans, Team, AS>(v, std::is_same<Team, WaveTeam>::value);
    else rbgs<T, Team, AS>(v, 2);
}

// Level lc between the cluster and the leader's LDS (S.hand): the leader
// copies what the cluster formed in the level's global copy (coefficients,
// restricted right-hand side) into LDS before its part of the cycle, and
// the correction x back afterwards.
template <typename T, bool kTransport>
__device__ void handoff_in(Solve<T>& S) {
    const Level<T>& G = S.hg;
    const LV<T, 3> D(S.lv[S.lc]);
    const int n = G.nx * G.ny;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        D.b[i] = G.b[i];
        D.x[i] = (T)0;
        if constexpr (kTransport) {
            D.acc[i] = G.acc[i]; D.mx[i] = G.mx[i]; D.my[i] = G.my[i]; D.dx[i] = G.dx[i]; D.dy[i] = G.dy[i];
        } else {
            D.te[i] = G.te[i]; D.tn[i] = G.tn[i];
        }
    }
    if constexpr (kTransport) {
        for (int j = threadIdx.x; j < G.ny; j += blockDim.x) {
            D.dl[j] = G.dl[j]; D.dr[j] = G.dr[j]; D.mr[j] = G.mr[j]; D.ml[j] = G.ml[j];
        }
    }
}

template <typename T>
__device__ void handoff_out(Solve<T>& S) {
    const LV<T, 3> D(S.lv[S.lc]);
    Level<T>& G = S.hg;
    const int n = G.nx * G.ny;
    for (int i = threadIdx.x; i < n; i += blockDim.x) G.x[i] = D.x[i];
}

// The coarsest level of every hierarchy has one row (ny = 1, nx = 2): the
// system is a single x-line, solved exactly.
template <typename T, bool kTransport, bool kTrans, class Team, int AS>
__device__ void vcoarsest(Solve<T>& S) {
    if constexpr (kTransport) line_sweep<T, true, kTrans, Team, AS>(S.lv[S.L - 1], 0);
    else {
        const LV<T, AS> v(S.lv[S.L - 1]);
        // pressure coarsest (2 x 1 cells): direct solve of the 2 x 2 system
        if (Team::rank() == 0) {
            const Stencil<T> s0 = pstencil(v, NbS(0, 0, 2, 1)), s1 = pstencil(v, NbS(1, 0, 2, 1));
            const T det = s0.d * s1.d - s0.e * s1.w;
            v.x[0] = (v.b[0] * s1.d + s0.e * v.b[1]) / det;
            v.x[1] = (s0.d * v.b[1] + s1.w * v.b[0]) / det;
        }
        Team::sync();
    }
}

// One V-cycle.  The cluster levels (0 .. lc-1) are run by the whole
// cluster; the leader alone runs the rest: its workgroup the levels in
// global memory, and from the first level in LDS (S.lds_from; the coarsest
// level always is) down to the coarsest and back, its wavefront 0 alone
// while the other wavefronts wait at one barrier.  With coarse_coeffs the
// leader first forms the coefficients of levels lc+1 .. L-1 (the cluster
// formed levels 1 .. lc before the cycle).
template <typename T, bool kTransport, bool kTrans = false>
__device__ void vcycle(Solve<T>& S, PhaseClock* pc = nullptr, bool coarse_coeffs = false) {
    const int L = S.L;
    const int lw = S.lds_from;
    const int lc = S.lc;
    const int t0 = kTransport ? 16 : 8;
    if (pc) pc->tick(kTransport ? 4 : 1);
    for (int l = 0; l < lc; ++l) {
        vdown<T, kTransport, kTrans, ClusterTeam, 1, 1>(S, l);
        if (pc) pc->tick(t0 + (l == 0 ? 1 : 2));
    }
    const int lb = S.lb;
    if (g_cl.member == 0) {
        if (S.hand) {
            handoff_in<T, kTransport>(S);
            __syncthreads();
        }
        if (coarse_coeffs) coarsen_leader<T, kTransport>(S, lc + 1);
        for (int l = lc; l < lw; ++l) {
            if (l + 1 < lb) vdown<T, kTransport, kTrans, BlockTeam, 1, 1>(S, l);
            else if (l < lb) vdown<T, kTransport, kTrans, BlockTeam, 1, 3>(S, l);
            else vdown<T, kTransport, kTrans, BlockTeam, 3, 3>(S, l);
            if (pc) pc->tick(t0 + (l == 0 ? 1 : 2));
        }
        if (threadIdx.x < kWave) {
            for (int l = lw; l < L - 1; ++l) vdown<T, kTransport, kTrans, WaveTeam, 3, 3>(S, l);
            vcoarsest<T, kTransport, kTrans, WaveTeam, 3>(S);
            for (int l = L - 2; l >= lw; --l) vup<T, kTransport, kTrans, WaveTeam, 3, 3>(S, l);
        }
        __syncthreads();
        if (pc) pc->tick(t0 + 3);
        for (int l = lw - 1; l >= lc; --l) {
            if (l + 1 < lb) vup<T, kTransport, kTrans, BlockTeam, 1, 1>(S, l);
            else if (l < lb) vup<T, kTransport, kTrans, BlockTeam, 1, 3>(S, l);
            else vup<T, kTransport, kTrans, BlockTeam, 3, 3>(S, l);
            if (pc) pc->tick(t0 + (l == 0 ? 6 : 4));
        }
        if (S.hand) handoff_out(S);
    }
    if (lc > 0) {
        ClusterTeam::sync();
        for (int l = lc - 1; l >= 0; --l) {
            vup<T, kTransport, kTrans, ClusterTeam, 1, 1>(S, l);
            if (pc) pc->tick(t0 + (l == 0 ? 6 : 4));
        }
    }
}

// Batched per-cell loops of the step: every thread first loads its kB cells
// (kB round trips in flight at once), then stores; one cell per loop trip
// would wait out a full memory latency per cell.
template <int kB>
__device__ inline void extrapolate_field(const double* u0, const double* u1, const double* u2, const double* u3,
                                         double* u4, int order, int n, int rk, int ts) {
    for (int base = rk; base < n; base += kB * ts) {
        double a0[kB], a1[kB], a2[kB], a3[kB], a4[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            const int idx = base + k * ts;
            if (idx < n) {
                a0[k] = u0[idx]; a1[k] = u1[idx]; a2[k] = u2[idx]; a3[k] = u3[idx];
                a4[k] = order == 4 ? u4[idx] : 0.0;
            }
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            const int idx = base + k * ts;
            if (idx < n) {
                double e = a0[k];
                if (order == 1) e = 2.0 * a0[k] - a1[k];
                else if (order == 2) e = 3.0 * a0[k] - 3.0 * a1[k] + a2[k];
                else if (order == 3) e = 4.0 * a0[k] - 6.0 * a1[k] + 4.0 * a2[k] - a3[k];
                else if (order == 4) e = (16.0 * a0[k] - 14.0 * a1[k] - 4.0 * a2[k] + 11.0 * a3[k] - 4.0 * a4[k]) * 0.2;
                u4[idx] = e;  // the oldest state's array becomes the iterate
            }
        }
    }
}

template <int kB, typename T, class XI>
__device__ inline void add_correction(double* u, const T* x, int n, int rk, int ts, XI xi) {
    for (int base = rk; base < n; base += kB * ts) {
        double uv[kB];
        T xv[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            const int idx = base + k * ts;
            if (idx < n) { uv[k] = u[idx]; xv[k] = x[xi(idx)]; }
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            const int idx = base + k * ts;
            if (idx < n) u[idx] = uv[k] + (double)xv[k];
        }
    }
}

// One implicit Euler step (Sec. 2.3) from the state u^n = (S.p, S.c):
// u^n becomes S.cn / S.pp (c^n is the previous time level of the
// residual) and the older states move down one role (bind_history), and the
// defect correction runs until
// both scaled residual max norms are <= tol.  The iteration starts from an
// extrapolation through the last states, by `order`: 0..3 the polynomial
// through the last order + 1 states (u^n; 2u^n - u^{n-1};
// 3u^n - 3u^{n-1} + u^{n-2}; 4u^n - 6u^{n-1} + 4u^{n-2} - u^{n-3}), 4 the
// least-squares cubic through the last five, (16u^n - 14u^{n-1} - 4u^{n-2}
// + 11u^{n-3} - 4u^{n-4}) / 5, which amplifies the states' own errors (of
// the size of the tolerance) less than the interpolating cubic does; on
// entry S.cn/pp, c2/p2, c3/p3, c4/p4 hold u^{n-1} .. u^{n-4}.  The start
// only changes how many iterations a step takes, not what it converges to.
// Returns 0 converged, 1 max_outer reached, 2 non-finite residual; adds the
// iterations used to `iters`.
template <typename T>
__device__ int implicit_step(const Phys& ph, Solve<T>& S, double* red, int max_outer, double tol, double& iters,
                             PhaseClock& pc, int order = 0) {
    const int n = S.n;
    const int rk = ClusterTeam::rank(), ts = ClusterTeam::size();
    extrapolate_field<4>(S.c, S.cn, S.c2, S.c3, S.c4, order, n, rk, ts);
    extrapolate_field<4>(S.p, S.pp, S.p2, S.p3, S.p4, order, n, rk, ts);
    ClusterTeam::sync();
    if (threadIdx.x == 0) {
        S.hist = (S.hist + 4) % 5;
        bind_history(S, reinterpret_cast<uint8_t*>(S.scratch - (int64_t)kF64Arrays * n));
    }
    __syncthreads();
    pc.tick(7);
    for (int it = 0; it < max_outer; ++it) {
        double np, nc;
        pc.tick(13);
        residual_pass(ph, S, 0, red, np, nc, &pc);
        pc.tick(0);
        if (!(np == np) || !(nc == nc) || np > 1e300 || nc > 1e300) return 2;
        if (np <= tol && nc <= tol) return 0;
        iters += 1.0;
        if (np > tol) {  // a pressure residual within the tolerance needs no correction
            coarsen_cluster<T, false>(S);
            pc.tick(1);
            vcycle<T, false>(S, &pc, true);
            pc.tick(2);
            const int nx = S.nx, sx = log2i(S.nx);
            add_correction<8>(S.p, S.lv[0].x, n, rk, ts, [=](int idx) {
                const int j = idx >> sx;
                return pidx(idx - j * nx, j, nx);
            });
            ClusterTeam::sync();
        }
        pc.tick(15);
        // the salt system's pass evaluates both residuals at the updated
        // state: the step may end here, before the salt cycle
        residual_pass(ph, S, 1, red, np, nc, &pc);
        if (!(np == np) || !(nc == nc) || np > 1e300 || nc > 1e300) return 2;
        if (np <= tol && nc <= tol) return 0;
        pc.tick(3);
        coarsen_cluster<T, true>(S);
        pc.tick(4);
        vcycle<T, true>(S, &pc, true);
        pc.tick(5);
        add_correction<8>(S.c, S.lv[0].x, n, rk, ts, [](int idx) { return idx; });
        ClusterTeam::sync();
        pc.tick(6);
    }
    return 1;
}

// Initial state: c = c0 (or 0, Sec. 2.1); p only seeds the iteration: the
// cell's own hydrostatic value -rho(c) g y.
template <typename T>
__device__ void initial_state(const Phys& ph, Solve<T>& S, const double* c0) {
    for (int idx = ClusterTeam::rank(); idx < S.n; idx += ClusterTeam::size()) {
        const int j = idx / S.nx;
        const double c = c0 ? c0[idx] : 0.0;
        S.c[idx] = c;
        S.p[idx] = -rho_of(ph, c) * ph.g * (-1.0 + (j + 0.5) * S.h);
    }
}

// Q = h^2 sum_{x<1} phi rho(c) c (FP64) in an order fixed by the grid
// alone: wavefront 0 keeps 64 partial sums (lane l adds the cells of index
// l mod 64 in increasing order), then a fixed butterfly over the lanes, so
// every workgroup size, cluster size and build gives the same bits.  Once
// per solve; the other wavefronts wait.
template <typename T>
__device__ double qoi_of(const Phys& ph, Solve<T>& S, double* red) {
    if (threadIdx.x < kWave) {
        double part = 0.0;
        for (int idx = threadIdx.x; idx < S.n; idx += kWave)
            if ((idx % S.nx) < S.nx / 2) part += S.phi[idx] * rho_of(ph, S.c[idx]) * S.c[idx];
        part = wave_sum(part);
        if (threadIdx.x == 0) red[0] = part;
    }
    __syncthreads();
    const double q = red[0] * S.h * S.h;
    __syncthreads();  // red is reused
    return q;
}

// Start of a step after `good` converged states in a row (the initial state
// counts as one): the extrapolation order grows with the history, up to the
// interpolating cubic (predictor 1) or the least-squares cubic through five
// states (predictor 2).  Predictor 0 takes 2 where the states' own errors,
// of the size of tol, outweigh the cubic's interpolation error: solves of
// 200 steps or more at tol >= 1e-8; 1 elsewhere.
__device__ inline int max_order(int predictor, int nsteps, double tol) {
    return predictor == 2 || (predictor == 0 && nsteps >= 200 && tol >= 1e-8) ? 4 : 3;
}
__device__ inline int start_order(int good, int top) { return min(max(good - 1, 0), top); }
__device__ inline int next_good(int good, int st) { return st == 0 ? min(good + 1, 5) : 0; }

// ------------------------------------------------------------------ time series
// Value of the piecewise-constant solution at (x, y): the cell that holds
// the point; on a face between two cells the mean of both, at a corner of
// four the mean of the four (the mean of the one-sided limits).
__device__ inline double point_value(const double* c, int nx, int ny, double x, double y) {
    const double u = x * ny, v = (y + 1.0) * ny;
    int i0 = (int)floor(u), j0 = (int)floor(v);
    int i1 = i0, j1 = j0;
    if (u == (double)i0) i0 -= 1;  // a vertical face: the cells on both sides
    if (v == (double)j0) j0 -= 1;
    i0 = min(max(i0, 0), nx - 1); i1 = min(max(i1, 0), nx - 1);
    j0 = min(max(j0, 0), ny - 1); j1 = min(max(j1, 0), ny - 1);
    return 0.25 * ((c[j0 * nx + i0] + c[j0 * nx + i1]) + (c[j1 * nx + i0] + c[j1 * nx + i1]));
}

// One record of a solve's time series (eq:integral_fw, eq:12points), by the
// whole workgroup of the leader: the fresh-water area h^2 #{c <= c_fresh}
// (an integer count, so the sum is exact in any order) and c at the points.
template <typename T>
__device__ void record_trace(const Launch& lp, Solve<T>& S, int index, int k, double* red) {
    double* out = lp.trace + ((int64_t)index * lp.trace_nrec + (k - 1)) * (1 + lp.trace_npts);
    double cnt = 0.0;
    for (int idx = threadIdx.x; idx < S.n; idx += blockDim.x) cnt += S.c[idx] <= lp.trace_fresh ? 1.0 : 0.0;
    cnt = block_sum(cnt, red);
    if (threadIdx.x == 0) out[0] = cnt * S.h * S.h;
    if (threadIdx.x < lp.trace_npts)
        out[1 + threadIdx.x] =
            point_value(S.c, S.nx, S.ny, lp.trace_pts[2 * threadIdx.x], lp.trace_pts[2 * threadIdx.x + 1]);
}

// ------------------------------------------------------------------ the solve kernel
// Cluster levels of a solve shared by K workgroups: level 0, then every
// level of >= 1024 K cells (>= 1024 per member) whose coarser neighbour is
// not run by wavefront 0; the level after them is handed to the leader's
// LDS when it lives there (cluster levels, of 8192 cells or more, never
// do).  At K = 8 the 128x64 level of a 256x128 solve is split (1024 cells
// per member): 383 -> 367 ms for the 16 such solves of the L = 4 batch,
// against its leader running it alone.
template <typename T>
__device__ inline void set_cluster_levels(Solve<T>& S, int K) {
    int lc = 0;
    if (K > 1) {
        lc = 1;
        while (lc + 1 < S.lds_from && (S.lv[lc].nx * S.lv[lc].ny) >= 1024 * K) ++lc;
    }
    S.lc = lc;
    S.hand = lc > 0 && lc == S.lb;
}

// Blocks of a launch: one per solve, or with clusters of K > 1 the blocks
// x + 8 (K c + r), r = 0 .. K-1, for cluster (solve) x + 8 c, so that the
// K members of a solve share an XCD; the launch has ceil(nsolves / 8) 8 K
// blocks and those of clusters past the last solve return at once.
__device__ inline void cluster_of_block(int K, int& cid, int& member) {
    const int b = (int)blockIdx.x;
    if (K == 1) { cid = b; member = 0; return; }
    const int x = b & 7, s = b >> 3;
    cid = x + 8 * (s / K);
    member = s % K;
}

template <typename T>
__global__ void __launch_bounds__(sizeof(T) == 4 ? HENRY_FP32_THREADS : 512) henry_solve_kernel(Launch lp) {
    extern __shared__ __align__(256) uint8_t lds_levels[];
    __shared__ Solve<T> S;
    __shared__ double red[32];
    int cid, member;
    cluster_of_block(lp.cluster, cid, member);
    if (cid >= lp.nsolves) return;
    const SolveDesc d = lp.descs[cid];
    const Phys& ph = lp.ph;
    // local steps of this launch: a solve with r steps advances r/g_total
    // local steps per global step (lockstep schedule across grids)
    const int s_begin = (int)(((int64_t)lp.g_begin * d.nsteps) / lp.g_total);
    const int s_end = (int)(((int64_t)lp.g_end * d.nsteps) / lp.g_total);
    if (s_begin >= s_end) return;
    if (threadIdx.x == 0) {
        bind_solve(S, lp.ws + d.ws_off, d.nx, d.ny, lds_levels, lp.lds_cells, lp.lds_block_cells);
        S.nsteps = d.nsteps;
        S.tau = ph.T / d.nsteps;
        set_cluster_levels(S, lp.cluster);
    }
    __syncthreads();
    double* sp = S.scratch;
    if (lp.cluster > 1) cluster_init(lp.cluster, member, sp, lp.cluster_wait);
    else cluster_init_single();
    if (threadIdx.x == 0) cluster_stage(lds_levels, lp.lds_bytes, line_stage_bytes_per_wave<T>());
    const int n = S.n;
    // scratch: [0] = q, [1] = status, [2] = iterations, [3] = converged
    // states in a row (the initial state counts as one), [4] = the history's
    // rotation; written by the leader at the end of a launch, read by every
    // member at the next
    int status = 0, good = 1;
    double iters = 0.0;
    if (s_begin == 0) {
        initial_state(ph, S, lp.c0 ? lp.c0 + d.field_off : nullptr);
    } else {
        status = (int)sp[1];
        iters = sp[2];
        good = (int)sp[3];
    }
    if (threadIdx.x == 0) {
        S.q = sp[0];
        if (s_begin > 0) {
            S.hist = (int)sp[4];
            bind_history(S, lp.ws + d.ws_off);
        }
    }
    ClusterTeam::sync();
    PhaseClock pc;
    pc.init();
    const int64_t N = d.nsteps, nrec = lp.trace ? lp.trace_nrec : 0;
    const int top = max_order(lp.predictor, d.nsteps, lp.tol);
    int s = s_begin;
    for (; s < s_end && status != 2 && !g_cl.failed; ++s) {
        // extrapolate only through converged states: a step that stopped at
        // max_outer restarts the history
        const int st = implicit_step(ph, S, red, lp.max_outer, lp.tol, iters, pc, start_order(good, top));
        if (st == 2) status = 2;
        else if (st == 1 && status == 0) status = 1;
        good = next_good(good, st);
        if (nrec && st != 2) {
            // the record whose step is s + 1, if any (nrec <= N: at most one)
            const int64_t k = (int64_t)(s + 1) * nrec / N;
            if (k >= 1 && (k * N + nrec - 1) / nrec == s + 1) {
                if (member == 0) record_trace(lp, S, d.index, (int)k, red);
                ClusterTeam::sync();  // the others keep c until the leader has read it
            }
        }
    }
    ClusterTeam::sync();
    if (g_cl.failed) status = 3;
    if (member != 0) return;
    if (nrec && (status == 2 || status == 3)) {
        // NaN in the records of step s (the step the solve stopped in, or
        // the first step of this launch) and later: the first such record is
        // k0 = floor((s - 1) nrec / N) + 1
        const int rw = 1 + lp.trace_npts;
        const int64_t k0 = s > 0 ? (int64_t)(s - 1) * nrec / N + 1 : 1;
        for (int64_t k = k0; k <= nrec; ++k)
            for (int v = threadIdx.x; v < rw; v += blockDim.x)
                lp.trace[((int64_t)d.index * nrec + (k - 1)) * rw + v] = __builtin_nan("");
    }
    if (threadIdx.x == 0) {
        sp[3] = (double)good;
        sp[1] = (double)status;
        sp[2] = iters;
        sp[4] = (double)S.hist;
        sp[kClusterGen] = (double)g_cl.gen;
#ifdef HENRY_PHASE_TIMERS
        for (int k = 0; k < 24; ++k) sp[8 + k] = (double)pc.acc[k];
#endif
    }
    if (s_end == d.nsteps) {
        // outputs: c, p at T and the QoI
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
            lp.c_out[d.field_off + idx] = S.c[idx];
            if (lp.p_out) lp.p_out[d.field_off + idx] = S.p[idx];
        }
        const double Q = qoi_of(ph, S, red);
        if (threadIdx.x == 0) {
            lp.qoi_out[d.index] = Q;
            lp.status[d.index] = status;
            if (lp.iters) lp.iters[d.index] = (int32_t)iters;
        }
    }
}

// The kernels below run from the main build only (a build of the solve
// kernel alone defines HENRY_SOLVE_KERNEL_ONLY).
#ifndef HENRY_SOLVE_KERNEL_ONLY

// The FP64 residual of one solve's discrete equations at a given state
// (p, c; previous time level cn): the same residual pass as the solver's,
// writing R^p and R^c instead of the inner-solve arrays.  One workgroup per
// solve, after henry_fields_kernel.
__global__ void __launch_bounds__(1024) henry_residual_kernel(Launch lp, const double* p, const double* c,
                                                              const double* cn, double* rp, double* rc) {
    extern __shared__ __align__(256) uint8_t lds_levels[];  // launched with none: no level in LDS
    __shared__ Solve<float> S;
    __shared__ double red[32];
    const SolveDesc d = lp.descs[blockIdx.x];
    const Phys& ph = lp.ph;
    if (threadIdx.x == 0) {
        bind_solve(S, lp.ws + d.ws_off, d.nx, d.ny, lds_levels, 0, 0);
        S.nsteps = d.nsteps;
        S.tau = ph.T / d.nsteps;
        S.q = S.scratch[0];
        S.rout_p = rp + d.field_off;
        S.rout_c = rc + d.field_off;
    }
    cluster_init_single();
    for (int idx = threadIdx.x; idx < S.n; idx += blockDim.x) {
        S.p[idx] = p[d.field_off + idx];
        S.c[idx] = c[d.field_off + idx];
        S.cn[idx] = cn[d.field_off + idx];
    }
    __syncthreads();
    double np, nc;
    residual_pass(ph, S, 2, red, np, nc);
}

// ------------------------------------------------------------------ random fields
// Point values at cell centres of the closed-form fields, of the KL
// expansions, of the two-layer porosity model, or the caller's explicit
// fields; FP64.  One block per solve.
__global__ void henry_fields_kernel(Launch lp) {
    const SolveDesc d = lp.descs[blockIdx.x];
    const Phys& ph = lp.ph;
    uint8_t* base = lp.ws + d.ws_off;
    double* f = reinterpret_cast<double*>(base);
    const int nx = d.nx, ny = d.ny, n = nx * ny;
    double* phi = f + (int64_t)kPhi * n;
    double* K = f + (int64_t)kK * n;
    double* sp = f + (int64_t)kF64Arrays * n;
    const double h = 1.0 / ny;
    if (lp.field_kind == 2) {
        // truncated KL expansions: phi = phi0 (1 + s_phi Z_phi), log K = log k0 + s_K Z_K,
        // Z = sum_k sqrt(lam_k) e_k xi_k; recharge factor (1 + 0.2 xi_41)
        const double* xi = lp.xi + (size_t)41 * d.index;
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
            double zp = 0.0, zk = 0.0;
            for (int k = 0; k < 20; ++k) {
                const double m = lp.kl_modes[(size_t)k * n + idx];
                zp += m * xi[k];
                zk += m * xi[20 + k];
            }
            phi[idx] = ph.phi0 * (1.0 + lp.kl_sigma_phi * zp);
            K[idx] = exp(log(ph.k0) + lp.kl_sigma_logk * zk);
        }
        if (threadIdx.x == 0) sp[0] = ph.q_in * (1.0 + 0.2 * xi[40]);
    } else if (lp.field_kind == 0) {
        const double x1 = lp.xi[3 * d.index], x2 = lp.xi[3 * d.index + 1], x3 = lp.xi[3 * d.index + 2];
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
            const int i = idx % nx, j = idx / nx;
            const double x = (i + 0.5) * h, y = -1.0 + (j + 0.5) * h;
            phi[idx] = ph.phi0 * (1.0 + 0.2 * x1 * cos(M_PI * x / 2.0) * cos(M_PI * y));
            K[idx] = ph.k0 * exp(0.5 * x2 * sin(M_PI * x / 2.0));
        }
        if (threadIdx.x == 0) sp[0] = ph.q_in * (1.0 + 0.2 * x3);
    } else if (lp.field_kind == 3) {
        // two porosity layers split at y = -0.75 (eq:poro_2levels, eq:poro_2levels_C),
        // Kozeny-Carman permeability (e_perm_Kozeny_Carman) scaled so that
        // K(phi0) = k0, recharge q_in (1 + 0.5 xi3)
        const double x1 = lp.xi[3 * d.index], x2 = lp.xi[3 * d.index + 1], x3 = lp.xi[3 * d.index + 2];
        const double kappa = ph.k0 * (1.0 - ph.phi0 * ph.phi0) / (ph.phi0 * ph.phi0 * ph.phi0);
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
            const int i = idx % nx, j = idx / nx;
            const double x = (i + 0.5) * h, y = -1.0 + (j + 0.5) * h;
            const double layer = y < -0.75 ? 1.0 + 0.2 * x1 : 1.0 - 0.2 * x1;
            const double fP =
                ph.phi0 * (1.0 + 0.15 * (x2 * cos(M_PI * x / 2.0) + x2 * sin(2.0 * M_PI * y) + x1 * cos(2.0 * M_PI * x))) *
                layer;
            phi[idx] = fP;
            K[idx] = kappa * fP * fP * fP / (1.0 - fP * fP);
        }
        if (threadIdx.x == 0) sp[0] = ph.q_in * (1.0 + 0.5 * x3);
    } else {
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
            phi[idx] = lp.phi_in[d.field_off + idx];
            K[idx] = exp(lp.logk_in[d.field_off + idx]);
        }
        if (threadIdx.x == 0) sp[0] = lp.qin_in[d.index];
    }
    // a fresh cluster state for the solve's first launch
    if (threadIdx.x == 0) {
        for (int k = kClusterFlags; k <= kClusterGen; ++k) sp[k] = 0.0;
    }
    __syncthreads();
    // face coefficients (harmonic means) and the residual scale
    double* tx = f + (int64_t)kTx * n;
    double* ty = f + (int64_t)kTy * n;
    double* wx = f + (int64_t)kWx * n;
    double* wy = f + (int64_t)kWy * n;
    double* isc = f + (int64_t)kIsc * n;
    const double tau = ph.T / d.nsteps;
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
        const int i = idx % nx, j = idx / nx;
        const double KP = K[idx], fP = phi[idx];
        if (i + 1 < nx) {
            const FacePair fx = face_pair(ph, KP, K[idx + 1], fP, phi[idx + 1]);
            tx[idx] = fx.t;
            wx[idx] = fx.w;
        } else {
            const FacePair fx = face_pair(ph, KP, KP, fP, fP);
            tx[idx] = 2.0 * fx.t;
            wx[idx] = 2.0 * fx.w;
        }
        if (j + 1 < ny) {
            const FacePair fy = face_pair(ph, KP, K[idx + nx], fP, phi[idx + nx]);
            ty[idx] = fy.t;
            wy[idx] = fy.w;
        } else {
            ty[idx] = 0.0;
            wy[idx] = 0.0;
        }
        isc[idx] = res_scale(ph, tau, h, fP);
    }
}

#endif  // HENRY_SOLVE_KERNEL_ONLY

}  // namespace HENRY_NS
