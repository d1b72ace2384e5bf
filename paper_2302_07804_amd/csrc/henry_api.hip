// henry_api.hip -- host side of the C ABI declared in include/henry.h.
//
// Validates every host argument before anything is enqueued, plans the
// batch (groups of solves sharing a grid, largest work first), places each
// solve's state in the caller's workspace, and launches the field and
// solve kernels.  Groups run concurrently on the context's internal
// streams, forked from and joined back into the caller's stream with
// events; with steps_per_launch > 0 the whole lockstep time loop is
// captured once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "henry.h"
#include "henry_adjoint.hpp"
#include "henry_check.hpp"
#include "henry_stats.hpp"
#include "henry_device.hpp"
#include "henry_kl.hpp"
#include "henry_mlmc.hpp"

// The 512-thread FP32 build (henry_solve512.hip).
size_t henry512_launch_bytes();
hipError_t henry512_launch_solve(dim3 grid, dim3 block, size_t lds, hipStream_t stream, const void* launch);

namespace {

constexpr int kStreams = 4;
// Multigrid levels of at most this many cells (32 x 16 and coarser) are kept
// in LDS: 28 KB per workgroup at FP32, 56 KB at FP64.
constexpr int kLdsCells = 512;  // levels of at most this many cells live in LDS (run by wavefront 0)
static_assert(kLdsCells >= 2, "the coarsest level (2 x 1) must be in LDS");
// With FP32 inner arrays, levels 1.. of up to 2048 cells also live in LDS
// (run by the whole workgroup): 82 KB for the 2048-cell level, ~110 KB in
// all, within the 160 KB of one CU.  The FP64 arrays would not fit.
constexpr int kLdsBlockCellsF32 = 2048;
int lds_block_cells(int prec) { return prec == HENRY_PREC_MIXED ? kLdsBlockCellsF32 : 0; }

// HENRY_FIELD_* to the fields kernel's branch: 0 closed form, 1 explicit,
// 2 KL, 3 two-layer porosity
int field_kind_of(int field) {
    switch (field) {
        case HENRY_FIELD_CLOSED3: return 0;
        case HENRY_FIELD_KL41: return 2;
        case HENRY_FIELD_TWOLAYER3: return 3;
        default: return 1;
    }
}
size_t lds_bytes(int nx, int ny, int prec) {
    return (size_t)(prec == HENRY_PREC_MIXED
                        ? henry::lds_level_bytes<float>(nx, ny, kLdsCells, lds_block_cells(prec))
                        : henry::lds_level_bytes<double>(nx, ny, kLdsCells, lds_block_cells(prec)));
}

// Dynamic LDS of a solve or adjoint launch: the LDS levels, or, for grids
// of 512 or 1024 cells per row shared by clusters, the line staging buffers
// of every wavefront if they take more (they overlay the levels; see
// henry::line_sweep_x_staged), as long as the workgroup's LDS holds them
// beside the kernel's static LDS (a few KB).
constexpr size_t kLdsStageCap = 150 * 1024;
size_t launch_lds_bytes(int nx, int ny, int prec, int threads, int cluster) {
    size_t b = lds_bytes(nx, ny, prec);
    if (cluster > 1 && nx >= 512) {
        const size_t per_wave = (size_t)(prec == HENRY_PREC_MIXED ? henry::line_stage_bytes_per_wave<float>()
                                                                  : henry::line_stage_bytes_per_wave<double>());
        const size_t st = (size_t)(threads / 64) * per_wave;
        if (st <= kLdsStageCap) b = std::max(b, st);
    }
    return b;
}

// Device memory of the allocation-free entry point (henry_solve_batch_static):
// every GPU the library runs on holds one copy of this array until the
// process ends.  Host code never uses the array's name as an address: each
// device's copy is looked up once with hipGetSymbolAddress (scratch_of) and
// only that pointer reaches kernels.
constexpr size_t kStaticScratchBytes = HENRY_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_rc[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// The static scratch of `device` (which must be current), looked up on the
// first call for that device; nullptr if the lookup failed.
void* scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void* ptr = nullptr;
        g_scratch_rc[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[device] = g_scratch_rc[device] == hipSuccess ? ptr : nullptr;
        g_scratch_done[device] = true;
    }
    return g_scratch_ptr[device];
}

// Descriptors of the allocation-free path reach the device as kernel
// arguments, kDescChunk at a time (no staging buffer, no copy from host memory).
constexpr int kDescChunk = 32;
struct DescChunk {
    henry::SolveDesc d[kDescChunk];
    int32_t first, count;
};

__global__ void desc_fill_kernel(DescChunk ch, henry::SolveDesc* table) {
    const int k = threadIdx.x;
    if (k < ch.count) table[ch.first + k] = ch.d[k];
}

struct Group {
    int nx, ny, threads, cluster;
    int stream = -1;           // tuned stream of a one-workgroup group, -1 = built-in plan
    std::vector<int> members;  // indices into the solve list
    double cost;
};

// Choices of the tuning cache for one grid width and precision (0 / -1 =
// the built-in choice).
struct Tuned {
    int threads = 0, cluster = 0, stream = -1;
};

struct PlanKey {
    std::vector<int64_t> words;
    bool operator==(const PlanKey& o) const { return words == o.words; }
};

constexpr int kKlModes = 20;

// KL basis of one grid in device memory: sqrt(lam_k) e_k at the cells.
struct KlGrid {
    double* modes = nullptr;  // [kKlModes][nx*ny]
    double sigma_phi = 0.1, sigma_logk = 0.5;
};

}  // namespace

struct henry_ctx {
    int device = 0;
    henry::Phys ph{};
    hipStream_t streams[kStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t joins[kStreams] = {};
    void* pinned = nullptr;      // host staging for descriptor tables
    size_t pinned_bytes = 0;
    hipEvent_t staging_done = nullptr;
    std::map<long, Tuned> tuned;  // (nx, prec) -> tuned launch choices
    // profiling of the last batch
    std::vector<henry_group_time_t> prof;
    std::vector<hipEvent_t> prof_ev;  // 2 per group
    // cached executable graph of the last chunked (lockstep) batch
    hipGraphExec_t graph_exec = nullptr;
    PlanKey graph_key;
    // graphs are captured and launched on this stream (the caller's stream
    // may be the legacy null stream, which cannot be captured)
    hipStream_t cap_stream = nullptr;
    hipEvent_t cap_in = nullptr, cap_out = nullptr;
    // KL bases by grid width
    std::map<int, KlGrid> kl;
    // this device's copy of the static scratch (allocation-free entry point)
    void* scratch = nullptr;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Largest workgroup of the solve kernel: the FP32-inner kernel has a build
// for 1024 threads (<= 128 VGPRs) and one for 512 (henry_solve512.hip, no
// register spills); the FP64 kernel is built for 512.
int max_threads(int prec) { return prec == HENRY_PREC_MIXED ? 1024 : 512; }

// Groups whose solves are shared by clusters run the 512-thread FP32 build
// when their workgroups allow it (their phases stream whole levels, and the
// spills of the 1024-thread build cost them: 1024x512 KL batch 4 % faster);
// the groups of one workgroup per solve keep the 1024-thread build, of which
// two 512-thread workgroups fit on one CU.  Results are the same bits.
bool use_build512(int prec, int threads, int cluster) {
    return prec == HENRY_PREC_MIXED && cluster > 1 && threads <= 512;
}
constexpr int kAdjMaxThreads = 512;

int check_grid(const henry_grid_t& g) {
    if (g.reserved != 0) return HENRY_EINVAL;
    if (g.ny < 1 || g.ny > 512 || !pow2(g.ny) || g.nx != 2 * g.ny) return HENRY_EINVAL;
    if (g.nsteps < 1) return HENRY_EINVAL;
    return HENRY_OK;
}

int check_opts(const henry_opts_t* o) {
    if (!o) return HENRY_EINVAL;
    if (o->prec != HENRY_PREC_FP64 && o->prec != HENRY_PREC_MIXED) return HENRY_EINVAL;
    if (o->max_outer < 1 || o->max_outer > 100000) return HENRY_EINVAL;
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return HENRY_EINVAL;
    if (o->threads != 0 && (o->threads < 64 || o->threads > max_threads(o->prec) || !pow2(o->threads)))
        return HENRY_EINVAL;
    if (o->steps_per_launch < 0) return HENRY_EINVAL;
    if (o->profile != 0 && o->profile != 1) return HENRY_EINVAL;
    if (o->serial_groups != 0 && o->serial_groups != 1) return HENRY_EINVAL;
    if (o->cluster != 0 && (o->cluster > henry::kMaxCluster || !pow2(o->cluster))) return HENRY_EINVAL;
    if (o->cluster_wait_us < 0) return HENRY_EINVAL;
    if (o->predictor < 0 || o->predictor > 2) return HENRY_EINVAL;
    return HENRY_OK;
}

// Workgroups per solve.  A cluster needs the level below the finest in
// global memory (more than 4 x kLdsCells cells).  Built-in choice: one
// workgroup per 8192 fine cells, at most 8, and at most as many as keep the
// group's clusters within the 256 CUs (one 1024-thread workgroup each).
int cluster_size(int nx, int ny, int nsolves, int requested) {
    const int cells = nx * ny;
    if (cells <= 4 * kLdsCells) return 1;
    if (requested > 0) return requested;
    int k = 1;
    while (2 * k <= henry::kMaxCluster && cells >= 2 * k * 8192 && 2 * k * nsolves <= 256) k *= 2;
    return k;
}

int64_t solve_bytes(int nx, int ny, int prec) {
    return prec == HENRY_PREC_MIXED ? henry::solve_bytes<float>(nx, ny) : henry::solve_bytes<double>(nx, ny);
}

// Built-in workgroup size (the choices the measuring autotuner makes on the
// MLMC hierarchy): twice the cells up to 512 threads, then the largest size
// the precision's kernel is built for.
int default_threads(int nx, int ny, int prec) {
    const int cells = nx * ny;
    if (cells <= 128) return 128;
    if (cells <= 512) return 256;
    if (cells <= 2048) return 512;
    return max_threads(prec);
}

int64_t desc_bytes(int nsolves) { return henry::align256((int64_t)nsolves * (int64_t)sizeof(henry::SolveDesc)); }


// Stream of each group (see enqueue_groups).
// A one-workgroup group with a tuned stream takes it; groups with clusters
// always take stream 0 (see enqueue_groups).
std::vector<int> stream_plan(const std::vector<Group>& order, int nstreams) {
    bool any_cluster = false;
    for (const Group& G : order) any_cluster |= G.cluster > 1;
    std::vector<int> si(order.size(), 0);
    int next = 0;
    for (size_t gi = 0; gi < order.size(); ++gi) {
        if (nstreams <= 0 || order[gi].cluster != 1) continue;
        if (order[gi].stream >= 0)
            si[gi] = order[gi].stream % nstreams;
        else
            si[gi] = any_cluster ? (nstreams > 1 ? 1 : 0) : next++ % nstreams;
    }
    return si;
}

// Fork from `s0`, launch every group (fields kernel, then the solve kernel
// over lockstep chunks of `steps_per_launch` global steps, or one launch),
// join back into `s0`.  Groups run concurrently on the context's streams
// unless `serial`.  Groups whose solves are shared by clusters all take
// stream 0, one after another: two cluster launches side by side could each
// hold CUs for partly dispatched clusters and wait on each other (the waits
// are bounded, but the solves would report HENRY_STATUS_SYNC).  Beside them
// the groups of one workgroup per solve run one after another on stream 1:
// run side by side they slow each other and the cluster group, which is
// the batch's critical path (L = 4 MLMC batch: 567 ms with the small
// groups on three streams, 482 ms on one).  Without a cluster group the
// groups take all streams in turn (there, side by side is faster).
int enqueue_groups(henry_ctx* ctx, const std::vector<Group>& order, const std::vector<int>& gstart,
                   const henry_grid_t* solves, const henry_opts_t* o, const henry::Launch& lp,
                   henry::SolveDesc* dtable, int rmax, hipStream_t s0, bool serial, bool profile) {
    const int ng = (int)order.size();
    const int nstreams = serial ? 0 : std::min(kStreams, ng);
    const int prec = o->prec;
    const int spl = o->steps_per_launch;
    if (hipEventRecord(ctx->fork, s0) != hipSuccess) return HENRY_EHIP;
    for (int k = 0; k < nstreams; ++k)
        if (hipStreamWaitEvent(ctx->streams[k], ctx->fork, 0) != hipSuccess) return HENRY_EHIP;
    const std::vector<int> si = stream_plan(order, nstreams);
    for (int gi = 0; gi < ng; ++gi) {
        const Group& G = order[gi];
        const int K = G.cluster;
        hipStream_t st = serial ? s0 : ctx->streams[si[gi]];
        henry::Launch l = lp;
        l.descs = dtable + gstart[gi];
        const int nb = (int)G.members.size();
        const int nblk = K == 1 ? nb : (nb + 7) / 8 * 8 * K;  // see henry::cluster_of_block
        l.nsolves = nb;
        l.cluster = K;
        l.cluster_wait = (uint64_t)(o->cluster_wait_us > 0 ? o->cluster_wait_us : 10000000) * 100u;  // 100 MHz
        if (l.field_kind == 2) {
            const KlGrid& kg = ctx->kl.at(G.nx);
            l.kl_modes = kg.modes;
            l.kl_sigma_phi = kg.sigma_phi;
            l.kl_sigma_logk = kg.sigma_logk;
        }
        hipLaunchKernelGGL(henry::henry_fields_kernel, dim3(nb), dim3(256), 0, st, l);
        // lockstep time chunks: local step s of a solve with r steps runs in
        // global step s * rmax / r; one chunk when steps_per_launch == 0
        l.lds_cells = kLdsCells;
        l.lds_block_cells = lds_block_cells(prec);
        const size_t lds = launch_lds_bytes(G.nx, G.ny, prec, G.threads, K);
        l.lds_bytes = (int32_t)lds;
        const int chunk = spl > 0 ? spl : rmax;
        if (profile) {
            henry_group_time_t& pt = ctx->prof[gi];
            pt.nx = G.nx; pt.ny = G.ny; pt.nsolves = nb; pt.launches = 0; pt.cell_steps = 0;
            pt.threads = G.threads; pt.cluster = K;
            for (int k : G.members) pt.cell_steps += (int64_t)solves[k].nx * solves[k].ny * solves[k].nsteps;
            if (hipEventRecord(ctx->prof_ev[2 * gi], st) != hipSuccess) return HENRY_EHIP;
        }
        for (int g0 = 0; g0 < rmax; g0 += chunk) {
            if (profile) ctx->prof[gi].launches++;
            l.g_begin = g0;
            l.g_end = std::min(rmax, g0 + chunk);
            l.g_total = rmax;
            if (use_build512(prec, G.threads, K)) {
                if (henry512_launch_bytes() != sizeof(l)) return HENRY_EHIP;  // one header, one layout
                if (henry512_launch_solve(dim3(nblk), dim3(G.threads), lds, st, &l) != hipSuccess) return HENRY_EHIP;
            } else if (prec == HENRY_PREC_MIXED) {
                hipLaunchKernelGGL(henry::henry_solve_kernel<float>, dim3(nblk), dim3(G.threads), lds, st, l);
            } else {
                hipLaunchKernelGGL(henry::henry_solve_kernel<double>, dim3(nblk), dim3(G.threads), lds, st, l);
            }
        }
        if (hipGetLastError() != hipSuccess) return HENRY_EHIP;
        if (profile && hipEventRecord(ctx->prof_ev[2 * gi + 1], st) != hipSuccess) return HENRY_EHIP;
    }
    for (int k = 0; k < nstreams; ++k) {
        if (hipEventRecord(ctx->joins[k], ctx->streams[k]) != hipSuccess) return HENRY_EHIP;
        if (hipStreamWaitEvent(s0, ctx->joins[k], 0) != hipSuccess) return HENRY_EHIP;
    }
    return HENRY_OK;
}

}  // namespace

extern "C" {

const char* henry_strerror(int code) {
    switch (code) {
        case HENRY_OK: return "ok";
        case HENRY_EINVAL: return "invalid argument";
        case HENRY_ENOMEM: return "workspace too small or out of host memory";
        case HENRY_EHIP: return "HIP runtime error";
        case HENRY_ENOCONV: return "a solve did not converge";
        case HENRY_ENONFINITE: return "non-finite residual";
        default: return "unknown error";
    }
}

void henry_opts_default(henry_opts_t* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->prec = HENRY_PREC_MIXED;
    o->max_outer = 40;
    o->tol = 1e-10;
    o->threads = 0;
    o->steps_per_launch = 0;
}

int henry_ctx_create(henry_ctx** out, const henry_phys_t* phys, int device) {
    if (!out || !phys) return HENRY_EINVAL;
    *out = nullptr;
    const double* v = &phys->rho0;
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(v[k])) return HENRY_EINVAL;
    if (!(phys->rho0 > 0) || !(phys->rho1 > 0) || !(phys->mu > 0) || phys->D < 0 || !(phys->T > 0))
        return HENRY_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HENRY_EINVAL;
    henry_ctx* c = new (std::nothrow) henry_ctx();
    if (!c) return HENRY_ENOMEM;
    c->device = device;
    std::memcpy(&c->ph, phys, sizeof(c->ph));
    DeviceGuard g(device);
    bool ok = true;
    for (int k = 0; k < kStreams; ++k) {
        ok &= hipStreamCreateWithFlags(&c->streams[k], hipStreamNonBlocking) == hipSuccess;
        ok &= hipEventCreateWithFlags(&c->joins[k], hipEventDisableTiming) == hipSuccess;
    }
    ok &= hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) == hipSuccess;
    ok &= hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess;
    ok &= hipEventCreateWithFlags(&c->cap_in, hipEventDisableTiming) == hipSuccess;
    ok &= hipEventCreateWithFlags(&c->cap_out, hipEventDisableTiming) == hipSuccess;
    ok &= hipEventCreateWithFlags(&c->staging_done, hipEventDisableTiming) == hipSuccess;
    // set-up of the allocation-free entry point: this device's scratch address
    // (a failed lookup only disables henry_solve_batch_static, which then
    // returns HENRY_EHIP)
    c->scratch = scratch_of(device);
    if (!ok) {
        henry_ctx_destroy(c);
        return HENRY_EHIP;
    }
    *out = c;
    return HENRY_OK;
}

void henry_ctx_destroy(henry_ctx* c) {
    if (!c) return;
    DeviceGuard g(c->device);
    for (int k = 0; k < kStreams; ++k) {
        if (c->streams[k]) (void)hipStreamSynchronize(c->streams[k]);
        if (c->streams[k]) (void)hipStreamDestroy(c->streams[k]);
        if (c->joins[k]) (void)hipEventDestroy(c->joins[k]);
    }
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->staging_done) {
        (void)hipEventSynchronize(c->staging_done);
        (void)hipEventDestroy(c->staging_done);
    }
    if (c->pinned) (void)hipHostFree(c->pinned);
    for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->cap_stream) {
        (void)hipStreamSynchronize(c->cap_stream);
        (void)hipStreamDestroy(c->cap_stream);
    }
    if (c->cap_in) (void)hipEventDestroy(c->cap_in);
    for (auto& kv : c->kl)
        if (kv.second.modes) (void)hipFree(kv.second.modes);
    if (c->cap_out) (void)hipEventDestroy(c->cap_out);
    delete c;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with Weyl-sequence key increments.
static void philox10(uint32_t x[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x[2];
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x[1] ^ k0;
        const uint32_t y1 = (uint32_t)p1;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x[3] ^ k1;
        const uint32_t y3 = (uint32_t)p0;
        x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

int henry_sample_xi(uint64_t seed, int32_t level, int64_t first, int64_t count, int32_t dim, double* out) {
    if (!out || count < 0 || first < 0 || dim < 1 || level < 0) return HENRY_EINVAL;
    for (int64_t s = 0; s < count; ++s) {
        const uint64_t index = (uint64_t)(first + s);
        for (int32_t blk = 0; 2 * blk < dim; ++blk) {
            uint32_t x[4] = {(uint32_t)blk, (uint32_t)level, (uint32_t)(index & 0xffffffffu), (uint32_t)(index >> 32)};
            philox10(x, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
            for (int half = 0; half < 2; ++half) {
                const int d = 2 * blk + half;
                if (d >= dim) break;
                const uint64_t bits = ((uint64_t)x[2 * half + 1] << 32) | x[2 * half];
                out[s * dim + d] = std::ldexp((double)(bits >> 11), -52) - 1.0;
            }
        }
    }
    return HENRY_OK;
}

int henry_kl_basis(int32_t nx, int32_t ny, int32_t nmodes, double corr_len, int32_t nquad, double* lambda_out,
                   double* modes_out) {
    if (nx < 2 || ny < 1 || nx != 2 * ny || nmodes < 1 || nmodes > 64 || !(corr_len > 0.0) || nquad < 8 ||
        nquad > 1024 || !lambda_out || !modes_out)
        return HENRY_EINVAL;
    std::vector<double> lam, modes;
    henry::kl::basis_2d(nx, ny, nmodes, corr_len, nquad, lam, modes);
    std::memcpy(lambda_out, lam.data(), sizeof(double) * nmodes);
    std::memcpy(modes_out, modes.data(), sizeof(double) * modes.size());
    return HENRY_OK;
}

int henry_ctx_set_kl(henry_ctx* ctx, int32_t nx, int32_t ny, double corr_len, double sigma_phi,
                     double sigma_logk) {
    if (!ctx) return HENRY_EINVAL;
    henry_grid_t g{nx, ny, 1, 0};
    if (check_grid(g) != HENRY_OK || !(corr_len > 0.0) || !std::isfinite(sigma_phi) || !std::isfinite(sigma_logk))
        return HENRY_EINVAL;
    std::vector<double> lam, modes;
    henry::kl::basis_2d(nx, ny, kKlModes, corr_len, 200, lam, modes);
    const size_t n = (size_t)nx * ny;
    for (int k = 0; k < kKlModes; ++k) {
        const double s = std::sqrt(std::max(lam[k], 0.0));
        for (size_t i = 0; i < n; ++i) modes[(size_t)k * n + i] *= s;
    }
    DeviceGuard dg(ctx->device);
    KlGrid& kg = ctx->kl[nx];
    if (!kg.modes && hipMalloc(&kg.modes, sizeof(double) * modes.size()) != hipSuccess) {
        ctx->kl.erase(nx);
        return HENRY_ENOMEM;
    }
    if (hipMemcpy(kg.modes, modes.data(), sizeof(double) * modes.size(), hipMemcpyHostToDevice) != hipSuccess)
        return HENRY_EHIP;
    kg.sigma_phi = sigma_phi;
    kg.sigma_logk = sigma_logk;
    if (ctx->graph_exec) {  // a cached graph may refer to the old basis
        (void)hipGraphExecDestroy(ctx->graph_exec);
        ctx->graph_exec = nullptr;
    }
    return HENRY_OK;
}

int henry_sample_xi_kl(uint64_t seed, int32_t level, int64_t first, int64_t count, double* out) {
    if (!out || count < 0 || first < 0 || level < 0) return HENRY_EINVAL;
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    for (int64_t s = 0; s < count; ++s) {
        const uint64_t index = (uint64_t)(first + s);
        const uint32_t ilo = (uint32_t)(index & 0xffffffffu), ihi = (uint32_t)(index >> 32);
        for (int g = 0; g < 20; ++g) {
            uint32_t x[4] = {(uint32_t)(100 + g), (uint32_t)level, ilo, ihi};
            philox10(x, k0, k1);
            const uint64_t b1 = (((uint64_t)x[1] << 32) | x[0]) >> 11;
            const uint64_t b2 = (((uint64_t)x[3] << 32) | x[2]) >> 11;
            const double u1 = std::ldexp((double)(b1 + 1), -53), u2 = std::ldexp((double)b2, -53);
            const double r = std::sqrt(-2.0 * std::log(u1));
            out[s * 41 + 2 * g] = r * std::cos(2.0 * M_PI * u2);
            out[s * 41 + 2 * g + 1] = r * std::sin(2.0 * M_PI * u2);
        }
        uint32_t x[4] = {200u, (uint32_t)level, ilo, ihi};
        philox10(x, k0, k1);
        out[s * 41 + 40] = std::ldexp((double)((((uint64_t)x[1] << 32) | x[0]) >> 11), -52) - 1.0;
    }
    return HENRY_OK;
}

int henry_workspace_bytes(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, const henry_opts_t* opts,
                          size_t* bytes_out) {
    (void)ctx;  // host-only computation; a context is not needed
    if (!bytes_out || nsolves < 0 || (nsolves > 0 && !solves)) return HENRY_EINVAL;
    henry_opts_t def;
    henry_opts_default(&def);
    const henry_opts_t* o = opts ? opts : &def;
    if (int rc = check_opts(o)) return rc;
    int64_t total = desc_bytes(nsolves);
    for (int k = 0; k < nsolves; ++k) {
        if (int rc = check_grid(solves[k])) return rc;
        total += solve_bytes(solves[k].nx, solves[k].ny, o->prec);
    }
    *bytes_out = (size_t)total;
    return HENRY_OK;
}

namespace {

// Time-series request of a forward batch (none: nrec == 0).
struct TraceArgs {
    int32_t nrec = 0, npts = 0;
    const double* pts = nullptr;  // host (x, y) pairs
    double fresh = 0.0;
    double* out = nullptr;        // device
};

int solve_batch_impl(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field, const double* xi,
                     const double* phi, const double* logk, const double* qin, const double* c0,
                     const henry_opts_t* opts, const TraceArgs& tr, double* c_out, double* p_out, double* qoi_out,
                     int32_t* status, int32_t* iters, void* workspace, size_t ws_bytes, void* stream,
                     bool static_scratch = false);

}  // namespace

int henry_solve_batch(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field, const double* xi,
                      const double* phi, const double* logk, const double* qin, const double* c0,
                      const henry_opts_t* opts, double* c_out, double* p_out, double* qoi_out, int32_t* status,
                      int32_t* iters, void* workspace, size_t ws_bytes, void* stream) {
    return solve_batch_impl(ctx, solves, nsolves, field, xi, phi, logk, qin, c0, opts, TraceArgs{}, c_out, p_out,
                            qoi_out, status, iters, workspace, ws_bytes, stream);
}

int henry_solve_batch_static(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field,
                             const double* xi, const double* phi, const double* logk, const double* qin,
                             const double* c0, const henry_opts_t* opts, double* c_out, double* p_out,
                             double* qoi_out, int32_t* status, int32_t* iters, void* stream) {
    return solve_batch_impl(ctx, solves, nsolves, field, xi, phi, logk, qin, c0, opts, TraceArgs{}, c_out, p_out,
                            qoi_out, status, iters, nullptr, 0, stream, true);
}

int henry_solve_batch_trace(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field,
                            const double* xi, const double* phi, const double* logk, const double* qin,
                            const double* c0, const henry_opts_t* opts, int32_t nrec, int32_t npts,
                            const double* points, double c_fresh, double* trace_out, double* c_out, double* p_out,
                            double* qoi_out, int32_t* status, int32_t* iters, void* workspace, size_t ws_bytes,
                            void* stream) {
    if (nrec < 1 || npts < 0 || npts > henry::kMaxTracePoints || (npts > 0 && !points) || !trace_out ||
        !std::isfinite(c_fresh))
        return HENRY_EINVAL;
    for (int k = 0; k < npts; ++k) {
        const double x = points[2 * k], y = points[2 * k + 1];
        if (!(x >= 0.0 && x <= 2.0 && y >= -1.0 && y <= 0.0)) return HENRY_EINVAL;
    }
    if (solves)
        for (int k = 0; k < nsolves; ++k)
            if (solves[k].nsteps < nrec) return HENRY_EINVAL;
    TraceArgs tr;
    tr.nrec = nrec; tr.npts = npts; tr.pts = points; tr.fresh = c_fresh; tr.out = trace_out;
    return solve_batch_impl(ctx, solves, nsolves, field, xi, phi, logk, qin, c0, opts, tr, c_out, p_out, qoi_out,
                            status, iters, workspace, ws_bytes, stream);
}

namespace {

int solve_batch_impl(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field, const double* xi,
                     const double* phi, const double* logk, const double* qin, const double* c0,
                     const henry_opts_t* opts, const TraceArgs& tr, double* c_out, double* p_out, double* qoi_out,
                     int32_t* status, int32_t* iters, void* workspace, size_t ws_bytes, void* stream,
                     bool static_scratch) {
    if (!ctx || nsolves < 0) return HENRY_EINVAL;
    if (nsolves == 0) return HENRY_OK;
    if (!solves) return HENRY_EINVAL;
    henry_opts_t def;
    henry_opts_default(&def);
    const henry_opts_t* o = opts ? opts : &def;
    if (int rc = check_opts(o)) return rc;
    if (field == HENRY_FIELD_CLOSED3 || field == HENRY_FIELD_TWOLAYER3) {
        if (!xi) return HENRY_EINVAL;
        if (field == HENRY_FIELD_TWOLAYER3 && !(1.74 * ctx->ph.phi0 < 1.0)) return HENRY_EINVAL;
    } else if (field == HENRY_FIELD_KL41) {
        if (!xi) return HENRY_EINVAL;
        for (int k = 0; k < nsolves; ++k)
            if (ctx->kl.find(solves[k].nx) == ctx->kl.end()) return HENRY_EINVAL;
    } else if (field == HENRY_FIELD_EXPLICIT) {
        if (!phi || !logk || !qin) return HENRY_EINVAL;
    } else {
        return HENRY_EINVAL;
    }
    if (static_scratch) {
        // nothing that allocates: no graph, no profiling events
        if (o->steps_per_launch != 0 || o->profile != 0) return HENRY_EINVAL;
        workspace = ctx->scratch;
        ws_bytes = kStaticScratchBytes;
    }
    if (!c_out || !qoi_out || !status) return HENRY_EINVAL;
    size_t need = 0;
    if (int rc = henry_workspace_bytes(ctx, solves, nsolves, o, &need)) return rc;
    if (static_scratch && !workspace) return HENRY_EHIP;
    if (!workspace) return HENRY_EINVAL;
    if (ws_bytes < need) return HENRY_ENOMEM;
    if (((uintptr_t)workspace & 255) != 0) return HENRY_EINVAL;

    // ---- plan: descriptors, groups by grid, largest work first
    const int prec = o->prec;
    std::vector<henry::SolveDesc> desc(nsolves);
    int64_t off = desc_bytes(nsolves), foff = 0;
    int32_t rmax = 0;
    for (int k = 0; k < nsolves; ++k) rmax = std::max(rmax, solves[k].nsteps);
    std::map<long, Group> groups;
    for (int k = 0; k < nsolves; ++k) {
        const henry_grid_t& g = solves[k];
        henry::SolveDesc& d = desc[k];
        d.nx = g.nx; d.ny = g.ny; d.nsteps = g.nsteps; d.nlev = henry::num_levels(g.ny);
        d.reserved = 0; d.index = k; d.ws_off = off; d.field_off = foff; d.adj_off = 0;
        off += solve_bytes(g.nx, g.ny, prec);
        foff += (int64_t)g.nx * g.ny;
        Group& G = groups[(long)g.nx];
        G.nx = g.nx; G.ny = g.ny;
        G.members.push_back(k);
        G.cost += (double)g.nx * g.ny * g.nsteps;
    }
    std::vector<Group> order;
    for (auto& kv : groups) order.push_back(kv.second);
    std::sort(order.begin(), order.end(), [](const Group& a, const Group& b) { return a.cost > b.cost; });
    // the table is laid out group by group so each launch sees a contiguous slice
    std::vector<henry::SolveDesc> table;
    table.reserve(nsolves);
    std::vector<int> gstart;
    for (auto& G : order) {
        gstart.push_back((int)table.size());
        for (int k : G.members) table.push_back(desc[k]);
        const auto it = ctx->tuned.find((long)G.nx * 4 + prec);
        const Tuned tu = it != ctx->tuned.end() ? it->second : Tuned{};
        int t = o->threads;
        G.cluster = cluster_size(G.nx, G.ny, (int)G.members.size(), o->cluster > 0 ? o->cluster : tu.cluster);
        if (t == 0 && tu.threads > 0) t = tu.threads;
        if (t == 0) t = (prec == HENRY_PREC_MIXED && G.cluster > 1) ? 512 : default_threads(G.nx, G.ny, prec);
        G.threads = t;
        G.stream = tu.stream;
    }

    DeviceGuard dg(ctx->device);
    hipStream_t s0 = reinterpret_cast<hipStream_t>(stream);
    const size_t tbytes = sizeof(henry::SolveDesc) * (size_t)nsolves;
    uint8_t* ws = reinterpret_cast<uint8_t*>(workspace);
    henry::SolveDesc* dtable = reinterpret_cast<henry::SolveDesc*>(ws);
    if (static_scratch) {
        for (int first = 0; first < nsolves; first += kDescChunk) {
            DescChunk ch{};
            ch.first = first;
            ch.count = std::min(kDescChunk, nsolves - first);
            for (int k = 0; k < ch.count; ++k) ch.d[k] = table[first + k];
            hipLaunchKernelGGL(desc_fill_kernel, dim3(1), dim3(kDescChunk), 0, s0, ch, dtable);
        }
        if (hipGetLastError() != hipSuccess) return HENRY_EHIP;
    } else {
        if (ctx->pinned) {
            if (hipEventSynchronize(ctx->staging_done) != hipSuccess) return HENRY_EHIP;
        }
        if (ctx->pinned_bytes < tbytes) {
            if (ctx->pinned) (void)hipHostFree(ctx->pinned);
            ctx->pinned = nullptr;
            ctx->pinned_bytes = 0;
            if (hipHostMalloc(&ctx->pinned, tbytes, hipHostMallocDefault) != hipSuccess) return HENRY_ENOMEM;
            ctx->pinned_bytes = tbytes;
        }
        std::memcpy(ctx->pinned, table.data(), tbytes);
        if (hipMemcpyAsync(dtable, ctx->pinned, tbytes, hipMemcpyHostToDevice, s0) != hipSuccess) return HENRY_EHIP;
        if (hipEventRecord(ctx->staging_done, s0) != hipSuccess) return HENRY_EHIP;
    }

    henry::Launch lp{};
    lp.ws = ws;
    lp.xi = xi; lp.phi_in = phi; lp.logk_in = logk; lp.qin_in = qin; lp.c0 = c0;
    lp.c_out = c_out; lp.p_out = p_out; lp.qoi_out = qoi_out; lp.status = status; lp.iters = iters;
    std::memcpy(&lp.ph, &ctx->ph, sizeof(lp.ph));
    lp.tol = o->tol;
    lp.max_outer = o->max_outer;
    lp.predictor = o->predictor;
    lp.field_kind = field_kind_of(field);
    lp.xi_dim = field == HENRY_FIELD_KL41 ? 41 : 3;
    if (tr.nrec > 0) {
        lp.trace = tr.out;
        lp.trace_nrec = tr.nrec;
        lp.trace_npts = tr.npts;
        lp.trace_fresh = tr.fresh;
        for (int k = 0; k < 2 * tr.npts; ++k) lp.trace_pts[k] = tr.pts[k];
    }

    const int ng = (int)order.size();
    const bool serial = o->serial_groups != 0;
    const int spl = o->steps_per_launch;
    const bool graph = spl > 0;
    // per-group event timing only outside graph capture; a replayed graph is
    // timed as one unit (entry 0)
    if (o->profile) {
        while ((int)ctx->prof_ev.size() < 2 * std::max(ng, 1)) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return HENRY_EHIP;
            ctx->prof_ev.push_back(e);
        }
        ctx->prof.assign(graph ? 1 : ng, henry_group_time_t{});
    } else {
        ctx->prof.clear();
    }
    if (!graph) return enqueue_groups(ctx, order, gstart, solves, o, lp, dtable, rmax, s0, serial, o->profile != 0);

    // Lockstep chunks of `spl` global steps: capture the whole sequence once
    // and replay it; the cached executable is reused while the plan and every
    // pointer argument are unchanged.
    PlanKey key;
    key.words.reserve(4 * nsolves + 32);
    for (int k = 0; k < nsolves; ++k) {
        key.words.push_back(solves[k].nx);
        key.words.push_back(solves[k].nsteps);
    }
    const uintptr_t ptrs[] = {(uintptr_t)xi, (uintptr_t)phi, (uintptr_t)logk, (uintptr_t)qin, (uintptr_t)c0,
                              (uintptr_t)c_out, (uintptr_t)p_out, (uintptr_t)qoi_out, (uintptr_t)status,
                              (uintptr_t)iters, (uintptr_t)workspace, (uintptr_t)s0};
    for (uintptr_t v : ptrs) { key.words.push_back((int64_t)v); }
    int64_t tolbits;
    std::memcpy(&tolbits, &o->tol, 8);
    for (int64_t v : {(int64_t)o->prec, (int64_t)o->max_outer, tolbits, (int64_t)o->threads, (int64_t)spl,
                      (int64_t)o->serial_groups, (int64_t)field, (int64_t)o->cluster, (int64_t)o->cluster_wait_us,
                      (int64_t)o->predictor})
        key.words.push_back(v);
    // the time-series request is part of the captured kernel arguments
    key.words.push_back((int64_t)(uintptr_t)tr.out);
    key.words.push_back(tr.nrec);
    key.words.push_back(tr.npts);
    for (int k = 0; k < 2 * tr.npts; ++k) {
        int64_t b;
        std::memcpy(&b, &tr.pts[k], 8);
        key.words.push_back(b);
    }
    {
        int64_t b;
        std::memcpy(&b, &tr.fresh, 8);
        key.words.push_back(b);
    }
    hipStream_t cs = ctx->cap_stream;
    if (hipEventRecord(ctx->cap_in, s0) != hipSuccess) return HENRY_EHIP;
    if (hipStreamWaitEvent(cs, ctx->cap_in, 0) != hipSuccess) return HENRY_EHIP;
    if (!ctx->graph_exec || !(key == ctx->graph_key)) {
        if (ctx->graph_exec) { (void)hipGraphExecDestroy(ctx->graph_exec); ctx->graph_exec = nullptr; }
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) return HENRY_EHIP;
        int rc = enqueue_groups(ctx, order, gstart, solves, o, lp, dtable, rmax, cs, serial, false);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(cs, &g);
        if (rc != HENRY_OK || ec != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return rc != HENRY_OK ? rc : HENRY_EHIP;
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return HENRY_EHIP;
        ctx->graph_exec = ex;
        ctx->graph_key = key;
    }
    if (o->profile) {
        henry_group_time_t& pt = ctx->prof[0];
        pt.nx = 0; pt.ny = 0; pt.nsolves = nsolves; pt.launches = 0; pt.cell_steps = 0;
        pt.threads = 0; pt.cluster = 0;
        for (int k = 0; k < nsolves; ++k) pt.cell_steps += (int64_t)solves[k].nx * solves[k].ny * solves[k].nsteps;
        for (int gi = 0; gi < ng; ++gi) pt.launches += (rmax + spl - 1) / spl;
        if (hipEventRecord(ctx->prof_ev[0], cs) != hipSuccess) return HENRY_EHIP;
    }
    if (hipGraphLaunch(ctx->graph_exec, cs) != hipSuccess) return HENRY_EHIP;
    if (o->profile && hipEventRecord(ctx->prof_ev[1], cs) != hipSuccess) return HENRY_EHIP;
    if (hipEventRecord(ctx->cap_out, cs) != hipSuccess) return HENRY_EHIP;
    if (hipStreamWaitEvent(s0, ctx->cap_out, 0) != hipSuccess) return HENRY_EHIP;
    return HENRY_OK;
}

}  // namespace

int henry_residual_batch(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field,
                         const double* xi, const double* phi, const double* logk, const double* qin,
                         const double* p, const double* c, const double* cn, double* rp_out, double* rc_out,
                         void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx || nsolves < 0) return HENRY_EINVAL;
    if (nsolves == 0) return HENRY_OK;
    if (!solves || !p || !c || !cn || !rp_out || !rc_out || !workspace) return HENRY_EINVAL;
    if (field == HENRY_FIELD_CLOSED3 || field == HENRY_FIELD_TWOLAYER3) {
        if (!xi) return HENRY_EINVAL;
        if (field == HENRY_FIELD_TWOLAYER3 && !(1.74 * ctx->ph.phi0 < 1.0)) return HENRY_EINVAL;
    } else if (field == HENRY_FIELD_KL41) {
        if (!xi) return HENRY_EINVAL;
        for (int k = 0; k < nsolves; ++k)
            if (ctx->kl.find(solves[k].nx) == ctx->kl.end()) return HENRY_EINVAL;
    } else if (field == HENRY_FIELD_EXPLICIT) {
        if (!phi || !logk || !qin) return HENRY_EINVAL;
    } else {
        return HENRY_EINVAL;
    }
    size_t need = 0;
    if (int rc = henry_workspace_bytes(ctx, solves, nsolves, nullptr, &need)) return rc;
    if (ws_bytes < need) return HENRY_ENOMEM;
    if (((uintptr_t)workspace & 255) != 0) return HENRY_EINVAL;
    // the layout of the mixed-precision solve (the residual is FP64 either way)
    std::vector<henry::SolveDesc> desc(nsolves);
    int64_t off = desc_bytes(nsolves), foff = 0;
    std::map<long, Group> groups;
    for (int k = 0; k < nsolves; ++k) {
        const henry_grid_t& g = solves[k];
        henry::SolveDesc& d = desc[k];
        d.nx = g.nx; d.ny = g.ny; d.nsteps = g.nsteps; d.nlev = henry::num_levels(g.ny);
        d.reserved = 0; d.index = k; d.ws_off = off; d.field_off = foff; d.adj_off = 0;
        off += solve_bytes(g.nx, g.ny, HENRY_PREC_MIXED);
        foff += (int64_t)g.nx * g.ny;
        Group& G = groups[(long)g.nx];
        G.nx = g.nx; G.ny = g.ny;
        G.members.push_back(k);
    }
    std::vector<henry::SolveDesc> table;
    std::vector<std::pair<int, const Group*>> starts;
    for (auto& kv : groups) {
        starts.emplace_back((int)table.size(), &kv.second);
        for (int k : kv.second.members) table.push_back(desc[k]);
    }
    DeviceGuard dg(ctx->device);
    hipStream_t s0 = reinterpret_cast<hipStream_t>(stream);
    const size_t tbytes = sizeof(henry::SolveDesc) * (size_t)nsolves;
    if (ctx->pinned && hipEventSynchronize(ctx->staging_done) != hipSuccess) return HENRY_EHIP;
    if (ctx->pinned_bytes < tbytes) {
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        ctx->pinned = nullptr;
        ctx->pinned_bytes = 0;
        if (hipHostMalloc(&ctx->pinned, tbytes, hipHostMallocDefault) != hipSuccess) return HENRY_ENOMEM;
        ctx->pinned_bytes = tbytes;
    }
    std::memcpy(ctx->pinned, table.data(), tbytes);
    uint8_t* ws = reinterpret_cast<uint8_t*>(workspace);
    henry::SolveDesc* dtable = reinterpret_cast<henry::SolveDesc*>(ws);
    if (hipMemcpyAsync(dtable, ctx->pinned, tbytes, hipMemcpyHostToDevice, s0) != hipSuccess) return HENRY_EHIP;
    if (hipEventRecord(ctx->staging_done, s0) != hipSuccess) return HENRY_EHIP;
    henry::Launch lp{};
    lp.ws = ws;
    lp.xi = xi; lp.phi_in = phi; lp.logk_in = logk; lp.qin_in = qin;
    std::memcpy(&lp.ph, &ctx->ph, sizeof(lp.ph));
    lp.field_kind = field_kind_of(field);
    lp.xi_dim = field == HENRY_FIELD_KL41 ? 41 : 3;
    lp.cluster = 1;
    for (const auto& st : starts) {
        const Group& G = *st.second;
        henry::Launch l = lp;
        l.descs = dtable + st.first;
        l.nsolves = (int)G.members.size();
        if (l.field_kind == 2) {
            const KlGrid& kg = ctx->kl.at(G.nx);
            l.kl_modes = kg.modes;
            l.kl_sigma_phi = kg.sigma_phi;
            l.kl_sigma_logk = kg.sigma_logk;
        }
        hipLaunchKernelGGL(henry::henry_fields_kernel, dim3(l.nsolves), dim3(256), 0, s0, l);
        hipLaunchKernelGGL(henry::henry_residual_kernel, dim3(l.nsolves), dim3(256), 0, s0, l, p, c, cn, rp_out,
                           rc_out);
    }
    if (hipGetLastError() != hipSuccess) return HENRY_EHIP;
    return HENRY_OK;
}

int henry_tune_set(henry_ctx* ctx, int32_t nx, int32_t prec, int32_t threads, int32_t cluster, int32_t stream) {
    if (!ctx || nx < 2 || nx > 1024 || (nx & (nx - 1)) != 0) return HENRY_EINVAL;
    if (prec != HENRY_PREC_FP64 && prec != HENRY_PREC_MIXED) return HENRY_EINVAL;
    if (threads != 0 && (threads < 64 || threads > max_threads(prec) || !pow2(threads))) return HENRY_EINVAL;
    if (cluster != 0 && (cluster > henry::kMaxCluster || !pow2(cluster))) return HENRY_EINVAL;
    if (stream < -1 || stream >= kStreams) return HENRY_EINVAL;
    const long key = (long)nx * 4 + prec;
    if (threads == 0 && cluster == 0 && stream == -1)
        ctx->tuned.erase(key);
    else
        ctx->tuned[key] = Tuned{threads, cluster, stream};
    if (ctx->graph_exec) {  // the cached graph was built with the old choice
        (void)hipGraphExecDestroy(ctx->graph_exec);
        ctx->graph_exec = nullptr;
    }
    return HENRY_OK;
}

int henry_tune_get(henry_ctx* ctx, int32_t nx, int32_t prec, int32_t* threads, int32_t* cluster, int32_t* stream) {
    if (!ctx || !threads || nx < 2 || nx > 1024 || (nx & (nx - 1)) != 0) return HENRY_EINVAL;
    if (prec != HENRY_PREC_FP64 && prec != HENRY_PREC_MIXED) return HENRY_EINVAL;
    const auto it = ctx->tuned.find((long)nx * 4 + prec);
    const Tuned tu = it != ctx->tuned.end() ? it->second : Tuned{};
    *threads = tu.threads > 0 ? tu.threads : default_threads(nx, nx / 2, prec);
    if (cluster) *cluster = tu.cluster;
    if (stream) *stream = tu.stream;
    return HENRY_OK;
}

int henry_profile_last(henry_ctx* ctx, henry_group_time_t* out, int32_t cap, int32_t* ngroups) {
    if (!ctx || !ngroups || cap < 0 || (cap > 0 && !out)) return HENRY_EINVAL;
    DeviceGuard dg(ctx->device);
    const int ng = (int)ctx->prof.size();
    *ngroups = ng;
    for (int g = 0; g < ng && g < cap; ++g) {
        float ms = 0.0f;
        if (hipEventSynchronize(ctx->prof_ev[2 * g + 1]) != hipSuccess) return HENRY_EHIP;
        if (hipEventElapsedTime(&ms, ctx->prof_ev[2 * g], ctx->prof_ev[2 * g + 1]) != hipSuccess) return HENRY_EHIP;
        ctx->prof[g].ms = ms;
        out[g] = ctx->prof[g];
    }
    return HENRY_OK;
}

int henry_adjoint_workspace_bytes(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves,
                                  const henry_opts_t* opts, int32_t ckpt_every, size_t* bytes_out) {
    (void)ctx;
    if (!bytes_out || nsolves < 0 || (nsolves > 0 && !solves) || ckpt_every < 1) return HENRY_EINVAL;
    henry_opts_t def;
    henry_opts_default(&def);
    const henry_opts_t* o = opts ? opts : &def;
    if (int rc = check_opts(o)) return rc;
    int64_t total = desc_bytes(nsolves);
    for (int k = 0; k < nsolves; ++k) {
        if (int rc = check_grid(solves[k])) return rc;
        total += solve_bytes(solves[k].nx, solves[k].ny, o->prec);
        total += henry::adjoint_bytes(solves[k].nx, solves[k].ny, solves[k].nsteps, ckpt_every);
    }
    *bytes_out = (size_t)total;
    return HENRY_OK;
}

int henry_adjoint_batch(henry_ctx* ctx, const henry_grid_t* solves, int32_t nsolves, int32_t field, const double* xi,
                        const double* phi, const double* logk, const double* qin, const henry_opts_t* opts,
                        int32_t ckpt_every, double adj_tol, int32_t adj_max_it, double* qoi_out, double* dq_dxi,
                        double* dq_dlogk, double* dq_dphi, double* dq_dq, int32_t* status, int32_t* iters,
                        void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx || nsolves < 0) return HENRY_EINVAL;
    if (nsolves == 0) return HENRY_OK;
    if (!solves || ckpt_every < 1 || !(adj_tol > 0.0) || !std::isfinite(adj_tol) || adj_max_it < 1)
        return HENRY_EINVAL;
    henry_opts_t def;
    henry_opts_default(&def);
    const henry_opts_t* o = opts ? opts : &def;
    if (int rc = check_opts(o)) return rc;
    if (o->threads > kAdjMaxThreads) return HENRY_EINVAL;
    if (field == HENRY_FIELD_CLOSED3 || field == HENRY_FIELD_TWOLAYER3) {
        if (!xi) return HENRY_EINVAL;
        if (field == HENRY_FIELD_TWOLAYER3 && !(1.74 * ctx->ph.phi0 < 1.0)) return HENRY_EINVAL;
    } else if (field == HENRY_FIELD_KL41) {
        if (!xi) return HENRY_EINVAL;
        for (int k = 0; k < nsolves; ++k)
            if (ctx->kl.find(solves[k].nx) == ctx->kl.end()) return HENRY_EINVAL;
    } else if (field == HENRY_FIELD_EXPLICIT) {
        if (!phi || !logk || !qin || dq_dxi) return HENRY_EINVAL;
    } else {
        return HENRY_EINVAL;
    }
    if (!qoi_out || !status || !workspace) return HENRY_EINVAL;
    size_t need = 0;
    if (int rc = henry_adjoint_workspace_bytes(ctx, solves, nsolves, o, ckpt_every, &need)) return rc;
    if (ws_bytes < need) return HENRY_ENOMEM;
    if (((uintptr_t)workspace & 255) != 0) return HENRY_EINVAL;
    const int prec = o->prec;
    // plan: one descriptor per solve, grouped by grid
    std::vector<henry::SolveDesc> desc(nsolves);
    int64_t off = desc_bytes(nsolves), foff = 0;
    std::map<long, Group> groups;
    for (int k = 0; k < nsolves; ++k) {
        const henry_grid_t& g = solves[k];
        henry::SolveDesc& d = desc[k];
        d.nx = g.nx; d.ny = g.ny; d.nsteps = g.nsteps; d.nlev = henry::num_levels(g.ny);
        d.reserved = 0; d.index = k; d.field_off = foff;
        d.ws_off = off;
        off += solve_bytes(g.nx, g.ny, prec);
        d.adj_off = off;
        off += henry::adjoint_bytes(g.nx, g.ny, g.nsteps, ckpt_every);
        foff += (int64_t)g.nx * g.ny;
        Group& G = groups[(long)g.nx];
        G.nx = g.nx; G.ny = g.ny;
        G.members.push_back(k);
        G.cost += (double)g.nx * g.ny * g.nsteps;
    }
    std::vector<Group> order;
    for (auto& kv : groups) order.push_back(kv.second);
    std::sort(order.begin(), order.end(), [](const Group& a, const Group& b) { return a.cost > b.cost; });
    std::vector<henry::SolveDesc> table;
    std::vector<int> gstart;
    for (auto& G : order) {
        gstart.push_back((int)table.size());
        for (int k : G.members) table.push_back(desc[k]);
        const auto it = ctx->tuned.find((long)G.nx * 4 + prec);
        const Tuned tu = it != ctx->tuned.end() ? it->second : Tuned{};
        int t = o->threads;
        if (t == 0) t = tu.threads > 0 ? tu.threads : default_threads(G.nx, G.ny, prec);
        G.threads = std::min(t, kAdjMaxThreads);
        G.cluster = cluster_size(G.nx, G.ny, (int)G.members.size(), o->cluster > 0 ? o->cluster : tu.cluster);
        G.stream = tu.stream;
    }
    DeviceGuard dg(ctx->device);
    hipStream_t s0 = reinterpret_cast<hipStream_t>(stream);
    const size_t tbytes = sizeof(henry::SolveDesc) * (size_t)nsolves;
    if (ctx->pinned && hipEventSynchronize(ctx->staging_done) != hipSuccess) return HENRY_EHIP;
    if (ctx->pinned_bytes < tbytes) {
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        ctx->pinned = nullptr;
        ctx->pinned_bytes = 0;
        if (hipHostMalloc(&ctx->pinned, tbytes, hipHostMallocDefault) != hipSuccess) return HENRY_ENOMEM;
        ctx->pinned_bytes = tbytes;
    }
    std::memcpy(ctx->pinned, table.data(), tbytes);
    uint8_t* ws = reinterpret_cast<uint8_t*>(workspace);
    henry::SolveDesc* dtable = reinterpret_cast<henry::SolveDesc*>(ws);
    if (hipMemcpyAsync(dtable, ctx->pinned, tbytes, hipMemcpyHostToDevice, s0) != hipSuccess) return HENRY_EHIP;
    if (hipEventRecord(ctx->staging_done, s0) != hipSuccess) return HENRY_EHIP;
    henry::Launch lp{};
    lp.ws = ws;
    lp.xi = xi; lp.phi_in = phi; lp.logk_in = logk; lp.qin_in = qin; lp.c0 = nullptr;
    lp.qoi_out = qoi_out; lp.status = status; lp.iters = iters;
    std::memcpy(&lp.ph, &ctx->ph, sizeof(lp.ph));
    lp.tol = o->tol;
    lp.max_outer = o->max_outer;
    lp.predictor = o->predictor;
    lp.field_kind = field_kind_of(field);
    lp.xi_dim = field == HENRY_FIELD_KL41 ? 41 : 3;
    henry::AdjLaunch al{};
    al.ckpt = ckpt_every;
    al.max_it = adj_max_it;
    al.tol = adj_tol;
    al.dq_dxi = dq_dxi; al.dq_dlogk = dq_dlogk; al.dq_dphi = dq_dphi; al.dq_dq = dq_dq;
    const int ng = (int)order.size();
    const int nstreams = std::min(kStreams, ng);
    if (hipEventRecord(ctx->fork, s0) != hipSuccess) return HENRY_EHIP;
    for (int k = 0; k < nstreams; ++k)
        if (hipStreamWaitEvent(ctx->streams[k], ctx->fork, 0) != hipSuccess) return HENRY_EHIP;
    const std::vector<int> si = stream_plan(order, nstreams);
    for (int gi = 0; gi < ng; ++gi) {
        const Group& G = order[gi];
        hipStream_t st = ctx->streams[si[gi]];
        henry::Launch l = lp;
        l.descs = dtable + gstart[gi];
        const int nb = (int)G.members.size();
        const int K = G.cluster;
        const int nblk = K == 1 ? nb : (nb + 7) / 8 * 8 * K;  // see henry::cluster_of_block
        l.nsolves = nb;
        l.cluster = K;
        l.cluster_wait = (uint64_t)(o->cluster_wait_us > 0 ? o->cluster_wait_us : 10000000) * 100u;  // 100 MHz
        if (l.field_kind == 2) {
            const KlGrid& kg = ctx->kl.at(G.nx);
            l.kl_modes = kg.modes;
            l.kl_sigma_phi = kg.sigma_phi;
            l.kl_sigma_logk = kg.sigma_logk;
        }
        hipLaunchKernelGGL(henry::henry_fields_kernel, dim3(nb), dim3(256), 0, st, l);
        l.lds_cells = kLdsCells;
        l.lds_block_cells = lds_block_cells(prec);
        const size_t lds = lds_bytes(G.nx, G.ny, prec);  // no line staging in the adjoint kernel
        l.lds_bytes = (int32_t)lds;
        if (prec == HENRY_PREC_MIXED)
            hipLaunchKernelGGL(henry::henry_adjoint_kernel<float>, dim3(nblk), dim3(G.threads), lds, st, l, al);
        else
            hipLaunchKernelGGL(henry::henry_adjoint_kernel<double>, dim3(nblk), dim3(G.threads), lds, st, l, al);
        if (hipGetLastError() != hipSuccess) return HENRY_EHIP;
    }
    for (int k = 0; k < nstreams; ++k) {
        if (hipEventRecord(ctx->joins[k], ctx->streams[k]) != hipSuccess) return HENRY_EHIP;
        if (hipStreamWaitEvent(s0, ctx->joins[k], 0) != hipSuccess) return HENRY_EHIP;
    }
    return HENRY_OK;
}

int mlmc_level_estimate(henry_ctx* ctx, int32_t L, const henry_grid_t* fine, const int32_t* m,
                        const double* const* c_fine, const double* const* c_coarse, const double* const* q_fine,
                        const double* const* q_coarse, double* const* mean_Y, double* const* var_Y, double* qstats,
                        double* Ec_finest, double* var_est, void* stream) {
    if (!ctx || L < 0 || L > 15 || !fine || !m || !c_fine || !q_fine || !mean_Y || !var_Y || !qstats ||
        !Ec_finest || !var_est)
        return HENRY_EINVAL;
    for (int l = 0; l <= L; ++l) {
        if (check_grid(fine[l]) != HENRY_OK || m[l] < 2 || !c_fine[l] || !q_fine[l] || !mean_Y[l] || !var_Y[l])
            return HENRY_EINVAL;
        if (l > 0) {
            if (!c_coarse || !q_coarse || !c_coarse[l] || !q_coarse[l]) return HENRY_EINVAL;
            if (fine[l].nx != 2 * fine[l - 1].nx) return HENRY_EINVAL;
        }
    }
    DeviceGuard dg(ctx->device);
    hipStream_t s0 = reinterpret_cast<hipStream_t>(stream);
    henry::LevelPtrs lp{};
    for (int l = 0; l <= L; ++l) {
        const int nx = fine[l].nx, ny = fine[l].ny;
        const double* cc = l > 0 ? c_coarse[l] : nullptr;
        const double* qc = l > 0 ? q_coarse[l] : nullptr;
        const int cells = nx * ny;
        const int blocks = (cells * 64 + 255) / 256;
        hipLaunchKernelGGL(henry::mlmc_field_stats_kernel, dim3(blocks), dim3(256), 0, s0, c_fine[l], cc, m[l], nx,
                           ny, mean_Y[l], var_Y[l]);
        hipLaunchKernelGGL(henry::mlmc_qoi_stats_kernel, dim3(1), dim3(64), 0, s0, q_fine[l], qc, m[l],
                           qstats + 2 * l);
        lp.mean[l] = mean_Y[l];
        lp.var[l] = var_Y[l];
        lp.m[l] = m[l];
        lp.nx[l] = nx;
    }
    hipLaunchKernelGGL(henry::mlmc_combine_kernel, dim3(1), dim3(1024), 0, s0, lp, L, fine[L].nx, fine[L].ny,
                       qstats, Ec_finest, var_est);
    if (hipGetLastError() != hipSuccess) return HENRY_EHIP;
    return HENRY_OK;
}

int henry_mlmc_telescope(henry_ctx* ctx, int32_t nlevels, int32_t nvals, const double* const* mean,
                         const double* const* var, const int32_t* m, const int64_t* off, double* pmean_out,
                         double* pvar_out, void* stream) {
    if (!ctx || nlevels < 1 || nlevels > henry::kMaxTelescopeLevels || nvals < 0 || !mean || !m || !pmean_out ||
        (var && !pvar_out))
        return HENRY_EINVAL;
    henry::TelescopePtrs tp{};
    for (int l = 0; l < nlevels; ++l) {
        if (!mean[l] || m[l] < 1 || (var && !var[l]) || (off && off[l] < 0)) return HENRY_EINVAL;
        tp.mean[l] = mean[l];
        tp.var[l] = var ? var[l] : nullptr;
        tp.off[l] = off ? off[l] : 0;
        tp.m[l] = (double)m[l];
    }
    if (nvals == 0) return HENRY_OK;
    DeviceGuard dg(ctx->device);
    hipStream_t s0 = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(henry::mlmc_telescope_kernel, dim3((nvals + 255) / 256), dim3(256), 0, s0, tp, nlevels,
                       nvals, pmean_out, pvar_out);
    if (hipGetLastError() != hipSuccess) return HENRY_EHIP;
    return HENRY_OK;
}

int henry_level_smooth(henry_ctx* ctx, int32_t nx, int32_t ny, int32_t kind, int32_t prec, int32_t sweeps,
                       const double* coef, const double* b, double* x, void* workspace, size_t ws_bytes,
                       void* stream) {
    henry_grid_t g{nx, ny, 1, 0};
    if (!ctx || check_grid(g) != HENRY_OK || kind < 0 || kind > 2 || sweeps < 0 || !coef || !b || !x || !workspace)
        return HENRY_EINVAL;
    if (prec != HENRY_PREC_FP64 && prec != HENRY_PREC_MIXED) return HENRY_EINVAL;
    const size_t elt = prec == HENRY_PREC_MIXED ? 4 : 8;
    if (ws_bytes < elt * (10 * (size_t)nx * ny + 4 * (size_t)ny)) return HENRY_ENOMEM;
    if (((uintptr_t)workspace & 255) != 0) return HENRY_EINVAL;
    DeviceGuard dg(ctx->device);
    hipStream_t s0 = reinterpret_cast<hipStream_t>(stream);
    if (prec == HENRY_PREC_MIXED)
        hipLaunchKernelGGL(henry::level_smooth_kernel<float>, dim3(1), dim3(1024), 0, s0, nx, ny, kind, sweeps,
                           coef, b, x, reinterpret_cast<float*>(workspace));
    else
        hipLaunchKernelGGL(henry::level_smooth_kernel<double>, dim3(1), dim3(512), 0, s0, nx, ny, kind, sweeps,
                           coef, b, x, reinterpret_cast<double*>(workspace));
    if (hipGetLastError() != hipSuccess) return HENRY_EHIP;
    return HENRY_OK;
}

int henry_sample_stats(henry_ctx* ctx, int32_t nsamples, int32_t nvals, const double* x, const double* x_sub,
                       int32_t nq, const double* probs, double* mean_out, double* var_out, double* q_out,
                       void* stream) {
    if (!ctx || nsamples < 1 || (nq > 0 && nsamples > henry::kMaxStatSamples) || nvals < 0 || nq < 0 ||
        nq > henry::kMaxQuantiles || (nq > 0 && (!probs || !q_out)) || !x || !mean_out || !var_out)
        return HENRY_EINVAL;
    henry::Probs pr{};
    pr.n = nq;
    for (int k = 0; k < nq; ++k) {
        if (!(probs[k] >= 0.0 && probs[k] <= 1.0)) return HENRY_EINVAL;
        pr.p[k] = probs[k];
    }
    if (nvals == 0) return HENRY_OK;
    int P = 0;  // sort buffer, only for quantiles
    if (nq > 0)
        for (P = 1; P < nsamples;) P <<= 1;
    DeviceGuard dg(ctx->device);
    hipStream_t s0 = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(henry::sample_stats_kernel, dim3(nvals), dim3(256), (size_t)P * sizeof(double), s0, x,
                       x_sub, nsamples, nvals, P, pr, mean_out, var_out, q_out);
    if (hipGetLastError() != hipSuccess) return HENRY_EHIP;
    return HENRY_OK;
}

int henry_first_passage(henry_ctx* ctx, int32_t nsamples, int32_t nrec, int32_t stride, int32_t col,
                        const double* trace, double threshold, int32_t below, int32_t* t_out, int32_t* hist_out,
                        void* stream) {
    if (!ctx || nsamples < 0 || nrec < 1 || stride < 1 || col < 0 || col >= stride || !trace || !t_out ||
        !std::isfinite(threshold))
        return HENRY_EINVAL;
    if (nsamples == 0 && !hist_out) return HENRY_OK;
    DeviceGuard dg(ctx->device);
    hipStream_t s0 = reinterpret_cast<hipStream_t>(stream);
    if (nsamples > 0)
        hipLaunchKernelGGL(henry::first_passage_kernel, dim3((nsamples + 255) / 256), dim3(256), 0, s0, trace,
                           nsamples, nrec, stride, col, threshold, below, t_out);
    if (hist_out)
        hipLaunchKernelGGL(henry::passage_hist_kernel, dim3((nrec + 64) / 64), dim3(64), 0, s0, t_out, nsamples,
                           nrec, hist_out);
    if (hipGetLastError() != hipSuccess) return HENRY_EHIP;
    return HENRY_OK;
}

}  // extern "C"
