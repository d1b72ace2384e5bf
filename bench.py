"""Benchmark: batched MLMC ensemble of Henry solves on one MI355X.

One step = one pass of the whole hot path over the L = 4 MLMC workload:
levels 0..4 on grids 16x8/50 ... 256x128/800 steps with m = 4096, 1024, 256,
64, 16 samples (every level > 0 solves its fine and coarse grid on shared
samples): 6816 solves, 910,950,400 cell-steps, through `henry_solve_batch`
(mixed precision: FP32 multigrid/line relaxation inside FP64 defect
correction), then `mlmc_level_estimate` (level means/variances, telescoped
E[c]).  Inputs (xi) are resident in HBM before the timed region.

Printed: one JSON line with the metric (cell-steps/s of the batched path),
the plain one-solve-at-a-time FP64 GPU path on a bounded sample (its rate
is extrapolated to the workload's composition and labelled as such), the
error of both against the FP64 oracle on a bounded sample of the same
solves, the roofline of the dominant kernel and the oracle's own rate on
the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import henry_inputs as hi  # noqa: E402

M_PER_LEVEL = (4096, 1024, 256, 64, 16)
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_per_outer(elt: int) -> float:
    """Bytes per fine cell that one defect-correction iteration must move
    if every phase reads its operands once and writes its results once
    (elt = bytes of the inner type).  Hierarchy phases carry the 4/3 factor
    of the multigrid levels below the fine grid."""
    f64 = 8
    residual_p = 5 * f64 + 4 * elt                    # p,c,c^n,phi,K in; te,tn,b,x out (norms reduced)
    coarsen_p = (2 * elt + 2 * elt / 4) / 3            # te,tn -> coarse levels
    sweep_p = 4 * elt + elt                            # x,b,te,tn in; x out (both colours)
    vcycle_p = (4 * sweep_p + (4 * elt + elt) + (elt + elt / 2) + (elt / 4 + 2 * elt)) * 4 / 3
    update = 2 * f64 + elt                             # p (or c) read-modify-write, correction in
    residual_c = 5 * f64 + 7 * elt                    # same inputs; acc,mx,my,dx,dy,b,x out
    coarsen_c = (5 * elt + 5 * elt / 4) / 3
    sweep_c = 7 * elt + elt                            # one line direction: 5 coefs, b, neighbours in; x out
    vcycle_c = (2 * sweep_c + (7 * elt + elt) + (elt + elt / 2) + (elt / 4 + 2 * elt)) * 4 / 3  # x pre, y post
    return residual_p + coarsen_p + vcycle_p + update + residual_c + coarsen_c + vcycle_c + update


def algorithmic_bytes_per_step() -> float:
    """Per fine cell and time step outside the iterations: c -> c^n copy
    and the final (converged) residual evaluation."""
    return 2 * 8 + (5 * 8 + 4 * 4)


def workload():
    solves, pairs = hi.mlmc_solves(M_PER_LEVEL)
    return solves, pairs


def xi_for(hm, solves):
    """xi for every solve from the library's generator, keyed (seed, level, index)."""
    out = np.empty((len(solves), 3))
    cache = {}
    for k, s in enumerate(solves):
        if s.level not in cache:
            m = max(x.index for x in solves if x.level == s.level) + 1
            cache[s.level] = hm.henry_sample_xi(hi.SEED, s.level, 0, m, 3)
        out[k] = cache[s.level][s.index]
    return out


def cpu_baseline_sample(solves, pairs):
    """Bounded sample of the workload for the oracle: the first fine solves
    of level 0, fine+coarse pairs of level 1, and one level-2 pair."""
    pick = list(pairs[0][0][:48])
    pick += list(pairs[1][0][:8]) + list(pairs[1][1][:8])
    pick += list(pairs[2][0][:1]) + list(pairs[2][1][:1])
    return pick


CALIB_BYTES = 512 << 20
TRAFFIC_PATH = os.path.join(ROOT, "profiles", "henry_solve_kernel_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2302_07804_amd", "csrc", f)
                  for f in ("henry_device.hpp", "henry_api.hip")]


def kernel_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _read_counters(d):
    """{(kernel name, dispatch id): value} of a rocprofv3 --pmc csv run."""
    import csv
    import glob
    out = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                key = (row["Kernel_Name"], int(row["Dispatch_Id"]))
                out[key] = out.get(key, 0.0) + float(row["Counter_Value"])
    return out


def summarize_pmc(fetch_dir, write_dir):
    """HBM traffic of the solve kernel from FETCH_SIZE and WRITE_SIZE runs
    (KiB per dispatch), each scaled by what the same counter reads for the
    calibration copy of CALIB_BYTES (read once, written once)."""
    fetch, write = _read_counters(fetch_dir), _read_counters(write_dir)

    def pick(cs, pat):
        return [v for (k, _), v in sorted(cs.items(), key=lambda kv: kv[0][1]) if pat in k]

    copy_f = max(pick(fetch, "copy") + pick(fetch, "Copy") + pick(fetch, "elementwise"))
    copy_w = max(pick(write, "copy") + pick(write, "Copy") + pick(write, "elementwise"))
    sf = CALIB_BYTES / (copy_f * 1024.0)
    sw = CALIB_BYTES / (copy_w * 1024.0)
    sol_f = pick(fetch, "henry_solve_kernel")
    sol_w = pick(write, "henry_solve_kernel")
    per_launch = (sum(sol_f) * 1024.0 * sf + sum(sol_w) * 1024.0 * sw) / len(sol_f)
    rec = dict(kernel="henry_solve_kernel<float>", kernel_hash=kernel_hash(), launches=len(sol_f),
               fetch_kib=sol_f, write_kib=sol_w, calib_bytes=CALIB_BYTES, calib_fetch_kib=copy_f,
               calib_write_kib=copy_w, fetch_scale=sf, write_scale=sw, bytes_per_launch=per_launch)
    with open(TRAFFIC_PATH, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def load_traffic():
    """Measured HBM bytes per solve-kernel launch, if the committed record
    was taken on the current kernel sources."""
    try:
        with open(TRAFFIC_PATH) as f:
            rec = json.load(f)
    except OSError:
        return None
    return rec["bytes_per_launch"] if rec.get("kernel_hash") == kernel_hash() else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--steps-per-launch", type=int, default=0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adjoint and 1024x512 throughput lines (other workloads, not the metric)")
    ap.add_argument("--kl-adjoint", action="store_true",
                    help="also run the discrete adjoint of the 32-sample 1024x512 KL workload at full length "
                         "(3200 steps, checkpoints every 100; ~95 s) and check dQ/dxi of sample 0 against "
                         "central differences of the forward map in three coefficients")
    ap.add_argument("--qmc-reference", nargs=2, type=int, metavar=("POINTS", "SHIFTS"), default=None,
                    help="compare the MLMC estimates truncated after each level with a randomly shifted Halton "
                         "reference (POINTS points x SHIFTS shifts) on 512x256/1600, at (1.60, -0.95) and for E[Q] "
                         "(default 128 4 with the other workloads, ~25 s)")
    ap.add_argument("--paper-setup", action="store_true",
                    help="run the paper-set-up workloads even with --no-extras")
    ap.add_argument("--no-paper-setup", action="store_true",
                    help="skip the paper's own set-up (two-layer porosity, Table 1 constants, T = 6016 s, "
                         "32x16-based hierarchy with r0 = 188): one-sample solve times per level 0..5, the MLMC "
                         "run with Table 3's counts for eps^2 = 1e-7, 600 time series and their MLMC mean (~50 s)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one device copy of CALIB_BYTES before the batch (HBM-counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs into the committed traffic record and exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the ensemble shards by sample across "
              "GPUs by design but this build measures a single MI355X.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2302_07804_amd as hm
    hm.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)

    solves, pairs = workload()
    grids = [(s.nx, s.ny, s.nsteps) for s in solves]
    cell_steps = sum(s.cell_steps for s in solves)
    xi_h = xi_for(hm, solves)
    xi = torch.tensor(xi_h, dtype=torch.float64, device=dev)
    ctx = hm.Context(hi.PHYS, 0)
    opts = hm.make_opts(prec=hm.PREC_MIXED, tol=args.tol, max_outer=60, steps_per_launch=args.steps_per_launch)

    # persistent buffers (allocated once, outside the timed region)
    cells = sum(s.cells for s in solves)
    wsb = hm.henry_workspace_bytes(grids, opts)
    ws_raw = torch.empty(wsb // 8 + 64, dtype=torch.float64, device=dev)
    off = (-ws_raw.data_ptr()) % 256 // 8
    ws = ws_raw[off:off + (wsb + 7) // 8]
    c_out = torch.empty(cells, dtype=torch.float64, device=dev)
    qoi = torch.empty(len(solves), dtype=torch.float64, device=dev)
    status = torch.empty(len(solves), dtype=torch.int32, device=dev)
    iters = torch.empty(len(solves), dtype=torch.int32, device=dev)
    offs = np.concatenate([[0], np.cumsum([s.cells for s in solves])])
    L = len(M_PER_LEVEL) - 1
    fine_grids = [hi.level_grid(l) for l in range(L + 1)]
    c_fine, c_coarse, q_fine, q_coarse = [], [], [], []
    for l, (fi, ci) in enumerate(pairs):
        c_fine.append(c_out[offs[fi[0]]:offs[fi[-1] + 1]])
        q_fine.append(qoi[fi[0]:fi[-1] + 1])
        c_coarse.append(None if ci is None else c_out[offs[ci[0]]:offs[ci[-1] + 1]])
        q_coarse.append(None if ci is None else qoi[ci[0]:ci[-1] + 1])
    mean_Y = [torch.empty(g[0] * g[1], dtype=torch.float64, device=dev) for g in fine_grids]
    var_Y = [torch.empty(g[0] * g[1], dtype=torch.float64, device=dev) for g in fine_grids]
    qstats = torch.empty(2 * (L + 1), dtype=torch.float64, device=dev)
    Ec = torch.empty(fine_grids[-1][0] * fine_grids[-1][1], dtype=torch.float64, device=dev)
    var_est = torch.empty(2, dtype=torch.float64, device=dev)

    def step(o=opts):
        hm.henry_solve_batch(ctx, grids, hm.FIELD_CLOSED3, xi=xi, opts=o, c_out=c_out, qoi_out=qoi, status=status,
                             iters=iters, workspace=ws)
        hm.mlmc_level_estimate(ctx, fine_grids, M_PER_LEVEL, c_fine, c_coarse, q_fine, q_coarse, mean_Y, var_Y,
                               qstats, Ec, var_est)

    log(f"workload: {len(solves)} solves, {cell_steps} cell-steps, workspace {wsb / 2**20:.1f} MiB")
    tuned = {}
    if not args.no_tune:
        t = time.time()
        res = hm.autotune(ctx, grids, xi, opts)
        tuned = {f"{nx}x{nx // 2}": v[0] for (nx, _), v in res.items()}
        log(f"autotune ({time.time() - t:.1f} s): threads per solve-workgroup {tuned}")
    if args.calib_copy:
        src = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for w in range(args.warmup):
        t = time.time()
        step()
        torch.cuda.synchronize()
        log(f"warmup {w}: {time.time() - t:.3f} s")
    st = status.cpu().numpy()
    if (st != 0).any():
        log(f"WARNING: {int((st != 0).sum())} solves reported status != 0")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    ms_per_step = 1000.0 * wall / args.steps
    value = cell_steps * args.steps / wall
    log(f"timed {args.steps} steps: {wall:.3f} s wall ({ev_ms / args.steps:.1f} ms/step by events)")
    iters_h = iters.cpu().numpy().astype(np.int64)
    status_h = status.cpu().numpy()

    # ---- dominant kernel: per-group HIP-event times of the solve kernels
    prof_opts = hm.make_opts(prec=hm.PREC_MIXED, tol=args.tol, max_outer=60, profile=1)
    step(prof_opts)
    torch.cuda.synchronize()
    groups = hm.henry_profile_last(ctx)
    b_outer = algorithmic_bytes_per_outer(4)
    b_step = algorithmic_bytes_per_step()
    per_group = []
    for g in groups:
        members = [k for k, s in enumerate(solves) if s.nx == g["nx"]]
        alg = sum(solves[k].cells * (b_outer * iters_h[k] + b_step * solves[k].nsteps + 16) for k in members)
        per_group.append(dict(g, alg_bytes=alg, gbs=alg / (g["ms"] * 1e-3) / 1e9,
                              mean_outer_per_step=float(np.mean([iters_h[k] / solves[k].nsteps for k in members]))))
    for g in per_group:
        log(f"group {g['nx']}x{g['ny']}: {g['nsolves']} solves, {g['ms']:.1f} ms, outer/step "
            f"{g['mean_outer_per_step']:.2f}, algorithmic {g['gbs']:.0f} GB/s")
    dom = max(per_group, key=lambda g: g["ms"])
    achieved = sum(g["alg_bytes"] for g in per_group) / (sum(g["ms"] for g in per_group) * 1e-3) / 1e9

    # ---- plain path: one solve per call, FP64 inner, bounded sample
    plain = None
    sample_idx = cpu_baseline_sample(solves, pairs)
    plain_opts = hm.make_opts(prec=hm.PREC_FP64, tol=args.tol, max_outer=60)
    if not args.no_plain:
        per_grid_t = {}
        reps = {16: 8, 32: 4, 64: 2, 128: 1, 256: 1}
        for nx, rep in reps.items():
            ks = [k for k, s in enumerate(solves) if s.nx == nx][:rep]
            ts = []
            for k in ks:
                x1 = xi[k:k + 1].contiguous()
                torch.cuda.synchronize()
                t = time.perf_counter()
                hm.solve(ctx, [grids[k]], xi=x1, opts=plain_opts)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            per_grid_t[nx] = float(np.median(ts))
            log(f"plain {nx}x{nx // 2}: {per_grid_t[nx] * 1e3:.1f} ms per solve")
        t_plain = sum(per_grid_t[s.nx] for s in solves)
        plain = dict(value=cell_steps / t_plain, unit="cell-steps/s", extrapolated=True,
                     per_solve_ms={f"{nx}x{nx // 2}": round(v * 1e3, 3) for nx, v in per_grid_t.items()},
                     note="median time of one-solve calls per grid, summed over the workload's 6816 solves")

    # ---- oracle on a bounded sample (CPU baseline) and errors of both paths
    cpu = None
    errs = {}
    if not args.no_cpu:
        import oracle
        threads = min(16, len(os.sched_getaffinity(0)))
        jobs = [(solves[k].nx, solves[k].ny, solves[k].nsteps, xi_h[k]) for k in sample_idx]
        t = time.perf_counter()
        refs = oracle.solve_many(hi.PHYS, jobs, threads=threads)
        tcpu = time.perf_counter() - t
        cs_sample = sum(solves[k].cell_steps for k in sample_idx)
        cpu = dict(value=cs_sample / tcpu, unit="cell-steps/s", cores=threads, kind="oracle",
                   sample=f"{len(sample_idx)} solves of the workload (48 level-0, 8 level-1 pairs, 1 level-2 "
                          f"pair; {cs_sample} cell-steps), one solve per thread, {tcpu:.1f} s wall")
        c_all = c_out.cpu().numpy()
        worst = worst_l2 = 0.0
        for k, r in zip(sample_idx, refs):
            c = c_all[offs[k]:offs[k + 1]].reshape(solves[k].ny, solves[k].nx)
            worst = max(worst, np.abs(c - r["c"]).max() / np.abs(r["c"]).max())
            worst_l2 = max(worst_l2, np.linalg.norm(c - r["c"]) / np.linalg.norm(r["c"]))
        errs["batched_mixed_max_rel_c_err"] = worst
        errs["batched_mixed_l2_rel_c_err"] = worst_l2
        # E[c] of level 0 over the sampled solves
        mean_gpu = np.mean([c_all[offs[k]:offs[k + 1]] for k in sample_idx[:48]], axis=0)
        mean_ora = np.mean([r["c"].ravel() for r in refs[:48]], axis=0)
        errs["batched_mixed_Ec_rel_err_level0_sample"] = float(np.abs(mean_gpu - mean_ora).max() / np.abs(mean_ora).max())
        if not args.no_plain:
            worst_p = 0.0
            for k, r in list(zip(sample_idx, refs))[::7]:
                out = hm.solve(ctx, [grids[k]], xi=xi[k:k + 1].contiguous(), opts=plain_opts)
                c = out["c"].cpu().numpy().reshape(solves[k].ny, solves[k].nx)
                worst_p = max(worst_p, np.abs(c - r["c"]).max() / np.abs(r["c"]).max())
            errs["plain_fp64_max_rel_c_err"] = worst_p
        log(f"oracle: {cpu['value']:.3e} cell-steps/s on {threads} threads; errors {errs}")
    # the finest level is beyond the oracle's reach (banded LU, hours per
    # solve): check two of its solves against tightly converged FP64 GPU solves
    fine_idx = [k for k, s in enumerate(solves) if s.nx == 256][:2]
    if fine_idx and not args.no_cpu:
        log("checking two 256x128 solves against FP64 solves at tol 1e-10")
        tight = hm.make_opts(prec=hm.PREC_FP64, tol=1e-10, max_outer=30)
        ref = hm.solve(ctx, [grids[k] for k in fine_idx], xi=xi[fine_idx[0]:fine_idx[-1] + 1].contiguous(),
                       opts=tight)
        torch.cuda.synchronize()
        c_all = c_out.cpu().numpy()
        rc = ref["c"].cpu().numpy()
        worst = 0.0
        for j, k in enumerate(fine_idx):
            a = c_all[offs[k]:offs[k + 1]]
            b = rc[j * solves[k].cells:(j + 1) * solves[k].cells]
            worst = max(worst, np.abs(a - b).max() / np.abs(b).max())
        errs["batched_mixed_max_rel_c_err_256x128_vs_fp64_tol1e-10"] = worst
        log(f"256x128 vs tight FP64: {worst:.3e}")

    # ---- other workloads of the method, reported beside the metric
    extras = None
    if not args.no_extras:
        extras = {}
        # discrete adjoint: 512 samples of 128x64/400, checkpoints every 20
        ag = [(128, 64, 400)] * 512
        axi = torch.tensor(hm.henry_sample_xi(hi.SEED, 3, 0, 512, 3), dtype=torch.float64, device=dev)
        aopts = hm.make_opts(prec=hm.PREC_MIXED, tol=args.tol, max_outer=60)
        hm.adjoint(ctx, ag, xi=axi, opts=aopts, ckpt_every=20, adj_tol=args.tol, adj_max_it=60)
        torch.cuda.synchronize()
        t = time.perf_counter()
        a = hm.adjoint(ctx, ag, xi=axi, opts=aopts, ckpt_every=20, adj_tol=args.tol, adj_max_it=60)
        torch.cuda.synchronize()
        ta = time.perf_counter() - t
        extras["adjoint_128x64"] = dict(
            workload="512 samples, 128x64, 400 steps, checkpoints every 20, dQ/dxi and dQ/dlog K per cell",
            seconds=ta, forward_cell_steps_per_s=512 * 128 * 64 * 400 / ta,
            nonconverged=int((a["status"].cpu().numpy() != 0).sum()), tol=args.tol)
        log(f"adjoint 512 x 128x64/400: {ta:.2f} s")
        del a
        # adaptive MLMC (Sec. 3) on the L = 4 hierarchy: pilot, eq:M_ell on the
        # measured variances and GPU costs, final batch, MSE split
        t = time.perf_counter()
        am = hm.mlmc_run(ctx, [hi.level_grid(l) for l in range(5)], 0.05, m_pilot=16, seed=hi.SEED,
                         opts=hm.make_opts(prec=hm.PREC_MIXED, tol=args.tol, max_outer=60))
        ta = time.perf_counter() - t
        extras["mlmc_adaptive_L4"] = dict(
            workload="adaptive MLMC for E[Q], eps = 0.05, 16-sample pilots, levels 16x8/50 .. 256x128/800",
            seconds=ta, final_batch_seconds=am["seconds"], m=[int(x) for x in am["m"]],
            seconds_per_sample=[float(x) for x in am["s"]], V=[float(x) for x in am["V"]], EQ=am["EQ"],
            var_est=am["var_est"], alpha=am["alpha"], beta=am["beta"], bias_estimate=am["bias"],
            mse_within_eps2=am["mse_ok"], nonconverged=am["nonconverged"])
        log(f"adaptive MLMC L4 eps 0.05: {ta:.2f} s, m = {extras['mlmc_adaptive_L4']['m']}, E[Q] = {am['EQ']:.5f}")
        # KL fields on 1024x512: 32 samples, all 3200 steps (tau = T/3200)
        steps = 3200
        kctx = hm.Context(hi.PHYS, 0)
        kctx.set_kl(1024, 512)
        kxi = torch.tensor(hm.henry_sample_xi_kl(hi.SEED, 6, 0, 32), dtype=torch.float64, device=dev)
        kg = [(1024, 512, steps)] * 32
        torch.cuda.synchronize()
        t = time.perf_counter()
        ko = hm.solve(kctx, kg, xi=kxi, opts=hm.make_opts(prec=hm.PREC_MIXED, tol=args.tol, max_outer=60))
        torch.cuda.synchronize()
        tk = time.perf_counter() - t
        extras["kl_1024x512"] = dict(
            workload="32 KL samples (20+20 modes + recharge), 1024x512, 3200 steps",
            seconds=tk, cell_steps_per_s=32 * 1024 * 512 * steps / tk,
            mean_outer_iters_per_step=float(ko["iters"].cpu().numpy().mean() / steps),
            nonconverged=int((ko["status"].cpu().numpy() != 0).sum()))
        log(f"1024x512 KL, 32 x 3200 steps: {tk:.2f} s")
        del ko
        if args.kl_adjoint:
            torch.cuda.synchronize()
            t = time.perf_counter()
            ka = hm.adjoint(kctx, kg, xi=kxi, opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-8, max_outer=60),
                            ckpt_every=100, adj_tol=1e-8, adj_max_it=60)
            torch.cuda.synchronize()
            tka = time.perf_counter() - t
            g0 = ka["dq_dxi"][0].cpu().numpy()
            log(f"1024x512 KL adjoint, 32 x 3200 steps: {tka:.2f} s")
            # central differences of the forward map, sample 0, coefficients 1, 21, 41
            h, ks = 1e-3, [0, 20, 40]
            x0 = kxi[0].cpu().numpy()
            pts = []
            for k in ks:
                for sg in (1.0, -1.0):
                    x = x0.copy()
                    x[k] += sg * h
                    pts.append(x)
            fo = hm.solve(kctx, [(1024, 512, steps)] * len(pts),
                          xi=torch.tensor(np.array(pts), dtype=torch.float64, device=dev),
                          opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-9, max_outer=40))
            qf = fo["qoi"].cpu().numpy()
            fd = [(qf[2 * i] - qf[2 * i + 1]) / (2 * h) for i in range(len(ks))]
            extras["kl_1024x512_adjoint"] = dict(
                workload="32 KL samples, 1024x512, 3200 steps, checkpoints every 100, dQ/dxi (41), dQ/dlog K, "
                         "dQ/dphi per cell", seconds=tka, tol=1e-8,
                nonconverged=int((ka["status"].cpu().numpy() != 0).sum()),
                outer_iters_per_step=float(ka["iters"].cpu().numpy().mean() / steps),
                fd_check={f"xi{k + 1}": dict(adjoint=float(g0[k]), central_difference=float(d),
                                             rel_diff=float(abs(g0[k] - d) / abs(d))) for k, d in zip(ks, fd)})
            log(f"1024x512 KL adjoint vs central differences: {extras['kl_1024x512_adjoint']['fd_check']}")
            del ka, fo
        kctx.close()

    qmc_ref = args.qmc_reference or (None if args.no_extras else (128, 4))
    if qmc_ref:
        # the reference of Fig. 11: a QMC mean on a grid one level finer than the
        # hierarchy, against the MLMC estimates truncated after each level
        npts, nsh = qmc_ref
        ref_grid = hi.level_grid(L + 1)
        shifts = (hm.henry_sample_xi(hi.SEED, 99, 0, nsh, 3) + 1.0) / 2.0
        qr = hm.qmc_run(ctx, ref_grid, npts, shifts=list(shifts),
                        opts=hm.make_opts(prec=hm.PREC_MIXED, tol=args.tol, max_outer=60))
        kp = hm.point_cell(ref_grid, 1.60, -0.95)
        Ec_ref = float(qr["Ec"][kp].item())
        c_shift = np.array([float(e[kp].item()) for e in qr["Ec_shift"]])
        tel_c = hm.telescoped_at(fine_grids, mean_Y, 1.60, -0.95)
        qs = qstats.cpu().numpy().reshape(L + 1, 2)
        tel_q = np.cumsum(qs[:, 0])
        # standard errors of the truncated estimators: sqrt(sum_l V_l / m_l)
        se_q = np.sqrt(np.cumsum(qs[:, 1] / np.array(M_PER_LEVEL)))
        vpt = [float(var_Y[l][hm.point_cell(fine_grids[l], 1.60, -0.95)].item()) for l in range(L + 1)]
        se_c = np.sqrt(np.cumsum(np.array(vpt) / np.array(M_PER_LEVEL)))
        extras = extras if extras is not None else {}
        extras["mlmc_vs_qmc"] = dict(
            workload=f"QMC reference: {npts} Halton points x {nsh} random shifts on "
                     f"{ref_grid[0]}x{ref_grid[1]}/{ref_grid[2]}; MLMC: the timed batch, truncated after each level",
            seconds=qr["seconds"], nonconverged=qr["nonconverged"],
            qmc_EQ=qr["EQ"], qmc_EQ_se=qr["se"], qmc_c_point=Ec_ref,
            qmc_c_mean_range=[float(qr["Ec"].min().item()), float(qr["Ec"].max().item())],
            qmc_c_var_max=float(qr["Varc"].max().item()), qmc_c_var_mean=float(qr["Varc"].mean().item()),
            qmc_c_point_se=float(c_shift.std(ddof=1) / np.sqrt(nsh)) if nsh > 1 else None,
            mlmc_c_point_by_level=[float(v) for v in tel_c], mlmc_EQ_by_level=[float(v) for v in tel_q],
            mlmc_c_point_se_by_level=[float(v) for v in se_c], mlmc_EQ_se_by_level=[float(v) for v in se_q],
            abs_err_c_point=[float(abs(v - Ec_ref)) for v in tel_c],
            rel_err_c_point=[float(abs(v - Ec_ref) / abs(Ec_ref)) for v in tel_c],
            abs_err_EQ=[float(abs(v - qr["EQ"])) for v in tel_q],
            rel_err_EQ=[float(abs(v - qr["EQ"]) / abs(qr["EQ"])) for v in tel_q])
        log(f"QMC {npts}x{nsh} on {ref_grid}: {qr['seconds']:.1f} s, E[Q] = {qr['EQ']:.6f} +- {qr['se']:.1e}, "
            f"c(1.60,-0.95) = {Ec_ref:.6f}; MLMC by level c: {tel_c}, E[Q]: {tel_q}")

    if args.paper_setup or not (args.no_extras or args.no_paper_setup):
        extras = extras if extras is not None else {}
        pctx = hm.Context(hi.PHYS_TABLE1, 0)
        popts = hm.make_opts(prec=hm.PREC_MIXED, tol=args.tol, max_outer=60)
        pxi = torch.tensor(hm.henry_sample_xi(hi.SEED, 30, 0, 1, 3), dtype=torch.float64, device=dev)
        per_sample = {}
        for l in range(6):
            g = hi.paper_level_grid(l)
            hm.solve(pctx, [(g[0], g[1], 2)], xi=pxi, opts=popts, model="two_layer")
            torch.cuda.synchronize()
            t = time.perf_counter()
            o = hm.solve(pctx, [g], xi=pxi, opts=popts, model="two_layer")
            torch.cuda.synchronize()
            per_sample[f"{g[0]}x{g[1]}/{g[2]}"] = dict(seconds=time.perf_counter() - t,
                                                       outer_iters_per_step=int(o["iters"].item()) / g[2],
                                                       status=int(o["status"].item()))
            log(f"paper set-up, one sample on {g}: {per_sample[f'{g[0]}x{g[1]}/{g[2]}']}")
            del o
        m3 = [1714, 344, 78, 14, 4, 2]
        plevels = [hi.paper_level_grid(l) for l in range(6)]
        pr = hm.mlmc_fixed(pctx, plevels, m3, seed=hi.SEED, opts=popts, model="two_layer")
        tel = hm.telescoped_at(plevels, pr["mean_Y"], 1.60, -0.95)
        vpt = [float(pr["var_Y"][l][hm.point_cell(plevels[l], 1.60, -0.95)].item()) for l in range(6)]
        extras["paper_setup"] = dict(
            workload="two-layer porosity (eq:poro_2levels), Kozeny-Carman K, recharge +-50 %, Table 1 constants, "
                     "T = 6016 s, levels 32x16/188 .. 1024x512/6016",
            one_sample=per_sample,
            table3_run=dict(m=m3, seconds=pr["seconds"], nonconverged=pr["nonconverged"], EQ=pr["EQ"],
                            c_point_by_level=[float(v) for v in tel], V_c_point=vpt,
                            V_Q=[float(v) for v in pr["V"]], alpha=pr["alpha"], beta=pr["beta"]))
        log(f"paper set-up, Table 3 counts (eps^2 = 1e-7): {pr['seconds']:.1f} s, {pr['nonconverged']} "
            f"non-converged, c(1.60,-0.95) by level {tel}, V at the point {vpt}")
        # the paper's MLMC target, c at (1.60, -0.95) at T, by the adaptive driver on
        # levels 0..3 at eps^2 = 1e-6 (Table 3's second row)
        pa = hm.mlmc_run(pctx, plevels[:4], 1e-3, m_pilot=16, seed=hi.SEED, opts=popts, model="two_layer",
                         point=(1.60, -0.95))
        extras["paper_setup"]["mlmc_adaptive_point"] = dict(
            workload="adaptive MLMC for E[c(1.60,-0.95)] at T, eps^2 = 1e-6, 16-sample pilots, levels 0..3",
            m=[int(v) for v in pa["m"]], V=[float(v) for v in pa["V"]], seconds_per_sample=[float(v) for v in pa["s"]],
            E=pa["EQ"], var_est=pa["var_est"], alpha=pa["alpha"], beta=pa["beta"], bias_estimate=pa["bias"],
            final_batch_seconds=pa["seconds"], mse_within_eps2=pa["mse_ok"], nonconverged=pa["nonconverged"])
        log(f"paper set-up, adaptive MLMC for c(1.60,-0.95), eps^2 1e-6: m = {list(pa['m'])}, "
            f"E = {pa['EQ']:.5f}, V = {[float(v) for v in pa['V']]}, {pa['seconds']:.2f} s final batch")
        # Figs. 4-7: 600 QMC realisations of the time series on the coarsest grid
        from paper_2302_07804_amd.mlmc import POINTS12, QUANTILES
        g0 = hi.paper_level_grid(0)
        nrec = 47  # records every 4 steps of 188: t = 128 s .. T
        pas = ((0, 1.2, True), (0, 1.7, True), (4, 0.9, False))
        sr = hm.series_run(pctx, g0, hm.henry_qmc_points(1, 600, 3), nrec, passages=pas, opts=popts, model="two_layer")
        q = sr["q"].cpu().numpy()
        mean = sr["mean"].cpu().numpy()
        fp = {}
        for (col, thr, below), (t, hist) in zip(pas, sr["passage"]):
            hh = hist.cpu().numpy()
            k = np.arange(len(hh))
            fp[f"{'Q_FW' if col == 0 else 'c(1.85,-0.95)'} {'<' if below else '>'} {thr}"] = dict(
                mean_record=float((k[1:] * hh[1:]).sum() / max(hh[1:].sum(), 1)), never=int(hh[0]),
                hist=[int(v) for v in hh])
        extras["paper_setup"]["series_600"] = dict(
            workload="600 Halton samples, 32x16/188, 47 records (every 4 steps, 128 s apart), Q_FW and c at the "
                     "12 points", seconds=sr["seconds"], nonconverged=sr["nonconverged"],
            Q_FW_mean=[float(v) for v in mean[:, 0]],
            Q_FW_quantiles={str(p): [float(v) for v in q[k, :, 0]] for k, p in enumerate(QUANTILES)},
            c_1p85_m0p95_quantiles_at_T={str(p): float(q[k, -1, 4]) for k, p in enumerate(QUANTILES)},
            first_passage=fp)
        log(f"paper set-up, 600-sample series: {sr['seconds']:.2f} s, first passage (records of 128 s): "
            f"{ {k: round(v['mean_record'], 2) for k, v in fp.items()} }")
        # the MLMC estimate of the mean series with Table 3's counts (Figs. 8-10)
        ms = hm.mlmc_series(pctx, plevels, m3, nrec, seed=hi.SEED, opts=popts, model="two_layer")
        ip = 1 + POINTS12.index((1.60, -0.95))
        extras["paper_setup"]["mlmc_series_table3"] = dict(
            workload="Table 3 counts for eps^2 = 1e-7, levels 32x16/188 .. 1024x512/6016, 47 records",
            seconds=ms["seconds"], nonconverged=ms["nonconverged"],
            Q_FW_mean=[float(v) for v in ms["mean"][:, 0]],
            c_1p60_m0p95_mean=[float(v) for v in ms["mean"][:, ip]],
            c_1p60_m0p95_level_mean=[[float(v) for v in ms["level_mean"][l, :, ip]] for l in range(6)],
            c_1p60_m0p95_level_var=[[float(v) for v in ms["level_var"][l, :, ip]] for l in range(6)],
            Q_FW_level_var=[[float(v) for v in ms["level_var"][l, :, 0]] for l in range(6)],
            c_1p60_m0p95_level_amplitude=[[float(max(-a, b)) for a, b in zip(ms["level_min"][l, :, ip],
                                                                              ms["level_max"][l, :, ip])]
                                          for l in range(6)])
        # the rates of Fig. 10 at the point, record 14 and T (levels 1..4; level 5 has two samples)
        rates = {}
        for rec in (13, nrec - 1):
            try:
                a_, b_, _ = hm.henry_mlmc_rates(ms["level_mean"][:5, rec, ip], ms["level_var"][:5, rec, ip], 1)
                rates[f"record {rec + 1}"] = dict(alpha=a_, beta=b_)
            except hm.HenryError:
                rates[f"record {rec + 1}"] = None
        extras["paper_setup"]["mlmc_series_table3"]["rates_c_1p60_m0p95"] = rates
        log(f"paper set-up, rates at (1.60,-0.95): {rates}")
        log(f"paper set-up, MLMC series (Table 3 counts): {ms['seconds']:.1f} s, {ms['nonconverged']} non-converged; "
            f"V_l of c(1.60,-0.95) at record 14: {[float(ms['level_var'][l, 13, ip]) for l in range(6)]}; "
            f"max |Y_l| there over all records: "
            f"{[float(np.max(np.maximum(-ms['level_min'][l, :, ip], ms['level_max'][l, :, ip]))) for l in range(6)]}")
        pctx.close()

    res = {
        "metric": "Henry sample solves/s (cell-steps/s) batched vs plain, same 1e-5 E[c] error",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "mlmc_L4: 16x8/50, 32x16/100, 64x32/200, 128x64/400, 256x128/800 steps, "
                               "m=4096,1024,256,64,16 (fine+coarse pairs), 6816 solves, 910950400 cell-steps",
                   "precision": "FP32 V-cycles inside FP64 defect correction", "tol": args.tol,
                   "steps_per_launch": args.steps_per_launch,
                   "parallelism": "one workgroup per solve; the finest grid's solves each shared by a cluster "
                                  "of workgroups on one XCD",
                   "threads_per_solve": tuned,
                   "workgroups_per_solve": {f"{g['nx']}x{g['ny']}": g["cluster"] for g in per_group}},
        "solves_per_s": len(solves) * args.steps / wall,
        "plain": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "errors_vs_oracle": errs,
        "nonconverged_solves": int((status_h != 0).sum()),
        "mean_outer_iters_per_step": float(iters_h.sum() / sum(s.nsteps for s in solves)),
        "outer_iters_per_step_by_grid": {f"{g['nx']}x{g['ny']}": round(g["mean_outer_per_step"], 3)
                                         for g in per_group},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(),
                     "algorithmic_bytes_per_launch": sum(g["alg_bytes"] for g in per_group) / len(per_group),
                     "kernel": "henry_solve_kernel<float>",
                     "per_group": [{k: v for k, v in g.items()} for g in per_group],
                     "dominant_group": f"{dom['nx']}x{dom['ny']}"},
        "cpu_baseline": cpu,
        "other_workloads": extras,
    }
    print(json.dumps(res, default=lambda o: o.item() if hasattr(o, "item") else str(o)))
    ctx.close()


if __name__ == "__main__":
    main()
