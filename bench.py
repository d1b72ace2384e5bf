"""Benchmark: batched MLMC ensemble of Henry solves on one MI355X.

One step = one pass of the whole hot path over the L = 4 MLMC workload:
levels 0..4 on grids 16x8/50 ... 256x128/800 steps with m = 4096, 1024, 256,
64, 16 samples (every level > 0 solves its fine and coarse grid on shared
samples): 6816 solves, 910,950,400 cell-steps, through `henry_solve_batch`
(mixed precision: FP32 multigrid/line relaxation inside FP64 defect
correction), then `mlmc_level_estimate` (level means/variances, telescoped
E[c]).  Inputs (xi) are resident in HBM before the timed region.

Printed on stdout: ONE compact JSON line (under 4 KB) with the metric
(cell-steps/s of the batched path), the plain one-solve-at-a-time FP64 GPU
path (per-grid one-solve times summed over the workload, labelled as an
extrapolation), errors against the FP64 oracle (stored oracle solves of
the same samples for levels 0-3 and sample 0 of level 4, and live oracle
solves of a bounded sample), the roofline of the dominant kernel on this
workload and on the 1024x512 KL workload, and the oracle's own rate on the
host cores.  Progress goes to stderr.  `--extras` also runs the method's
other workloads (adjoint, adaptive MLMC, QMC reference, the paper's set-up)
and writes their records to stderr and to `--extras-out`, never to stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import henry_inputs as hi  # noqa: E402

M_PER_LEVEL = (4096, 1024, 256, 64, 16)
HBM_PEAK_GBS = 8000.0
METRIC = "Henry sample solves/s (cell-steps/s) batched vs plain, same 1e-5 E[c] error"
RECORD_LIMIT = 4096
GOLDEN = os.path.join(ROOT, "tests", "golden")
KL_GRID = (1024, 512, 3200)
KL_SAMPLES = 32


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


def solve_alg_bytes(cells: int, nsteps: int, outer_iters: int, elt: int = 4) -> float:
    """Algorithmic bytes of one solve: every outer iteration, the per-step
    work and the 16 B per cell of c, p written at T."""
    return cells * (algorithmic_bytes_per_outer(elt) * outer_iters + algorithmic_bytes_per_step() * nsteps + 16)


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


# ------------------------------------------------------------------ traffic counters
CALIB_BYTES = 512 << 20
TRAFFIC_PATHS = {
    "mlmc_L4": os.path.join(ROOT, "profiles", "henry_solve_kernel_traffic_mlmc_L4.json"),
    "kl_1024x512": os.path.join(ROOT, "profiles", "henry_solve_kernel_traffic_kl_1024x512.json"),
}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2302_07804_amd", "csrc", f)
                  for f in ("henry_device.hpp", "henry_api.hip", "henry_solve512.hip")]


def kernel_hash() -> str:
    """Hash of the solve kernel's sources with their comments and blank
    lines removed: counters taken on a kernel stay valid while only its
    comments change, and become stale with any change to its code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        lines = [ln.rstrip() for ln in text.splitlines()]
        h.update("\n".join(ln for ln in lines if ln).encode())
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


def summarize_pmc(fetch_dir, write_dir, workload_name="mlmc_L4", path=None):
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
    sol_f = pick(fetch, "henry_solve_kernel<float>")
    sol_w = pick(write, "henry_solve_kernel<float>")
    per_launch = (sum(sol_f) * 1024.0 * sf + sum(sol_w) * 1024.0 * sw) / len(sol_f)
    rec = dict(kernel="henry_solve_kernel<float>", workload=workload_name, kernel_hash=kernel_hash(),
               launches=len(sol_f), fetch_kib=sol_f, write_kib=sol_w, calib_bytes=CALIB_BYTES,
               calib_fetch_kib=copy_f, calib_write_kib=copy_w, fetch_scale=sf, write_scale=sw,
               bytes_per_launch=per_launch)
    with open(path or TRAFFIC_PATHS[workload_name], "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def load_traffic(workload_name="mlmc_L4"):
    """Measured HBM bytes per solve-kernel launch, if the committed record
    was taken on the current kernel sources."""
    try:
        with open(TRAFFIC_PATHS[workload_name]) as f:
            rec = json.load(f)
    except OSError:
        return None
    return rec["bytes_per_launch"] if rec.get("kernel_hash") == kernel_hash() else None


# ------------------------------------------------------------------ the compact record
def sig(v, digits=4):
    """Round floats (also inside lists and dicts) to `digits` significant digits."""
    if isinstance(v, dict):
        return {k: sig(x, digits) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [sig(x, digits) for x in v]
    if isinstance(v, (float, np.floating)):
        v = float(v)
        if v == 0.0 or not math.isfinite(v):
            return v if math.isfinite(v) else None
        return float(f"{v:.{digits}g}")
    if isinstance(v, np.integer):
        return int(v)
    return v


def roofline_entry(groups, traffic):
    """Roofline of the solve kernel from per-group launches: groups is a list
    of dicts (nx, ny, ms, launches, alg_bytes).  achieved = algorithmic bytes
    per launch / mean launch duration (the sum over launches of each)."""
    launches = sum(g["launches"] for g in groups)
    ms = sum(g["ms"] for g in groups)
    alg = sum(g["alg_bytes"] for g in groups)
    achieved = alg / (ms * 1e-3) / 1e9
    dom = max(groups, key=lambda g: g["ms"])
    dom_gbs = dom["alg_bytes"] / (dom["ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "henry_solve_kernel<float>",
            "launches": launches, "alg_bytes_per_launch": alg / launches, "mean_launch_ms": ms / launches,
            "dominant_group": f"{dom['nx']}x{dom['ny']}", "dominant_group_frac": dom_gbs / HBM_PEAK_GBS,
            "groups_ms_frac": {f"{g['nx']}x{g['ny']}": [g["ms"], g["alg_bytes"] / (g["ms"] * 1e-3) / 1e9 /
                                                       HBM_PEAK_GBS] for g in groups}}


def make_record(*, value, steps, warmup, ms_per_step, tol, threads, clusters, solves_per_s, plain, errors,
                nonconverged, outer_per_step, roofline, roofline_kl, kl, cpu):
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "mlmc_L4: 16x8/50 .. 256x128/800 steps, m=4096,1024,256,64,16 fine+coarse pairs, "
                               "6816 solves, 910950400 cell-steps",
                   "precision": "FP32 V-cycles inside FP64 defect correction", "tol": tol,
                   "threads": threads, "cluster": clusters},
        "solves_per_s": solves_per_s,
        "plain": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "errors_vs_oracle": errors,
        "nonconverged_solves": nonconverged,
        "outer_iters_per_step": outer_per_step,
        "roofline": roofline,
        "roofline_kl_1024x512": roofline_kl,
        "kl_1024x512": kl,
        "cpu_baseline": cpu,
    }
    return sig(rec)


def record_line(rec) -> str:
    line = json.dumps(rec, separators=(",", ":"))
    if len(line) > RECORD_LIMIT:
        raise ValueError(f"benchmark record is {len(line)} bytes, over {RECORD_LIMIT}")
    return line


# ------------------------------------------------------------------ the oracle on the host cores
def host_cores() -> int:
    """Threads the oracle pool uses: every core this process may run on,
    capped by the job's OMP_NUM_THREADS share when one is set."""
    n = len(os.sched_getaffinity(0))
    share = os.environ.get("OMP_NUM_THREADS")
    if share and share.isdigit() and int(share) > 0:
        n = min(n, int(share))
    return n


# Bounded sample: per grid, whole solves of the workload (or the first steps
# of one, at the workload's own tau, for the grids the oracle takes minutes
# to hours on).
CPU_SAMPLE = ((16, 64, None), (32, 16, None), (64, 2, None), (128, 1, 8), (256, 1, 1))


def cpu_baseline(solves, xi_h, cores):
    """Oracle (FP64 Newton + banded LU, one solve per thread) on a bounded
    sample of the workload: per-grid rates, and the whole workload's time on
    `cores` threads extrapolated from them.  Returns (record, jobs, results)
    where jobs lists the workload solves run in full (for error checks)."""
    import oracle
    jobs, meta = [], []
    for nx, n, first_steps in CPU_SAMPLE:
        ks = [k for k, s in enumerate(solves) if s.nx == nx][:n]
        for k in ks:
            s = solves[k]
            ph = dict(hi.PHYS)
            steps = s.nsteps
            if first_steps is not None:
                ph["T"] = hi.PHYS["T"] * first_steps / s.nsteps  # same tau, first steps only
                steps = first_steps
            jobs.append((ph, s.nx, s.ny, steps, xi_h[k]))
            meta.append((k, steps, first_steps is None))

    def run(job):
        ph, nx, ny, steps, x = job
        t = time.perf_counter()
        r = oracle.solve_xi(ph, nx, ny, steps, x)
        return r, time.perf_counter() - t

    import concurrent.futures as cf
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        out = list(ex.map(run, jobs))
    wall = time.perf_counter() - t0
    rate = {}
    for (k, steps, _), (_, dt) in zip(meta, out):
        s = solves[k]
        cs, tt = rate.get(s.nx, (0.0, 0.0))
        rate[s.nx] = (cs + s.cells * steps, tt + dt)
    per_grid = {nx: cs / tt for nx, (cs, tt) in rate.items()}   # cell-steps/s of one thread
    core_s = sum(s.cell_steps / per_grid[s.nx] for s in solves)
    total_s = core_s / cores
    cell_steps = sum(s.cell_steps for s in solves)
    per_level = {}
    for l in range(len(M_PER_LEVEL)):
        ls = [s for s in solves if s.level == l]
        per_level[f"L{l}"] = sum(s.cell_steps for s in ls) / sum(s.cell_steps / per_grid[s.nx] for s in ls)
    rec = {"value": cell_steps / total_s, "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
           "sample": (f"{len(jobs)} solves of the workload on {cores} threads in {wall:.1f} s: 64 of 16x8/50, "
                      "16 of 32x16/100, 2 of 64x32/200 whole, the first 8 of 400 steps of one 128x64 and the "
                      "first step of one 256x128 solve; value = workload cell-steps / extrapolated time"),
           "per_grid_thread_rate": {f"{nx}x{nx // 2}": v for nx, v in per_grid.items()},
           "per_level_thread_rate": per_level,
           "extrapolated_total_s": total_s, "extrapolated": True}
    full = [(k, r) for (k, _, whole), (r, _) in zip(meta, out) if whole]
    return rec, full


# ------------------------------------------------------------------ stored oracle references
def load_oracle_level(level):
    path = os.path.join(GOLDEN, f"oracle_mlmc_L4_level{level}.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def load_oracle_finest():
    path = os.path.join(GOLDEN, "oracle_mlmc_L4_level4_sample0.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def inject(c, factor):
    return np.repeat(np.repeat(c, factor, axis=-2), factor, axis=-1)


def errors_vs_stored_oracle(solves, pairs, c_all, q_all, mean_Y):
    """Errors of the batch against the stored oracle solves of the same
    samples: level means of Y_l (l = 0..3), the telescoped E[c] through
    level 3, every QoI of levels 0..3, and the c fields of level 4's
    sample 0 (fine and coarse); max-norm, relative to the oracle's max."""
    errs = {}
    levels = [load_oracle_level(l) for l in range(4)]
    have = [z is not None for z in levels]
    offs = np.concatenate([[0], np.cumsum([s.cells for s in solves])])
    if all(have):
        E_gpu = E_ora = None
        worst_mean = worst_q = 0.0
        for l, z in enumerate(levels):
            fx, fy, _ = hi.level_grid(l)
            mg = mean_Y[l].reshape(fy, fx)
            worst_mean = max(worst_mean, np.abs(mg - z["mean_Y"]).max() / max(np.abs(z["mean_Y"]).max(), 1e-300))
            E_gpu = mg if E_gpu is None else inject(E_gpu, 2) + mg
            E_ora = z["mean_Y"] if E_ora is None else inject(E_ora, 2) + z["mean_Y"]
            fi, ci = pairs[l]
            q = q_all[fi]
            worst_q = max(worst_q, np.abs(q - z["Q_fine"]).max() / np.abs(z["Q_fine"]).max())
            if ci is not None:
                worst_q = max(worst_q, np.abs(q_all[ci] - z["Q_coarse"]).max() / np.abs(z["Q_coarse"]).max())
        errs["Ec_through_L3"] = np.abs(E_gpu - E_ora).max() / np.abs(E_ora).max()
        errs["mean_Y_L0_3"] = worst_mean
        errs["Q_all_L0_3"] = worst_q
    fz = load_oracle_finest()
    if fz is not None:
        fi, ci = pairs[4]
        for name, k, ref in (("c_L4_fine0", fi[0], fz["c_fine0"]), ("c_L4_coarse0", ci[0], fz["c_coarse0"])):
            c = c_all[offs[k]:offs[k + 1]].reshape(ref.shape)
            errs[name] = np.abs(c - ref).max() / np.abs(ref).max()
    return errs


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--steps-per-launch", type=int, default=0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-kl", action="store_true", help="skip the 1024x512 KL workload's roofline")
    ap.add_argument("--kl-steps", type=int, default=KL_GRID[2],
                    help="run only the first K steps (tau = T/3200 kept) of the 1024x512 KL workload")
    ap.add_argument("--only-kl", action="store_true",
                    help="run only the 1024x512 KL workload (for counter runs) and print its record")
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-cache", default=None, metavar="JSON",
                    help="autotuner choices: used as they are when the file holds every grid, else tuned and "
                         "written there (counter runs reuse the bench's launch configuration this way)")
    ap.add_argument("--extras", action="store_true",
                    help="also run the method's other workloads (adjoint, adaptive MLMC, QMC reference, the "
                         "paper's set-up); their records go to stderr and --extras-out, not to stdout")
    ap.add_argument("--extras-out", default=None)
    ap.add_argument("--kl-adjoint", action="store_true",
                    help="with --extras: the full-length 1024x512 KL adjoint of the 32 samples, with a "
                         "central-difference check of sample 0")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one device copy of CALIB_BYTES before the batch (HBM-counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs into the committed traffic record and exit")
    ap.add_argument("--pmc-workload", default="mlmc_L4", choices=tuple(TRAFFIC_PATHS))
    ap.add_argument("--phase-timers", nargs="*", type=int, metavar="K", default=None,
                    help="time the phases of the outer iteration of the 16 finest solves (256x128/800) alone with "
                         "the instrumented build (compiled first if missing), for each cluster size K (default 4)")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, workload_name=args.pmc_workload)
        return
    if args.phase_timers is not None:
        phase_timers(args.phase_timers or [4], args.tol)
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

    if args.calib_copy:
        src = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.only_kl:
        kl, rl = run_kl(hm, torch, dev, args, log)
        print(record_line(sig({"kl_1024x512": kl, "roofline_kl_1024x512": rl})))
        return

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
    ws = hm.aligned_workspace(wsb, dev)
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
        res = hm.autotune(ctx, grids, xi, opts, cache_path=args.tune_cache)
        tuned = {f"{nx}x{nx // 2}": v[0] for (nx, _), v in res.items()}
        log(f"autotune ({time.time() - t:.1f} s): {tuned}")
    for w in range(args.warmup):
        t = time.time()
        step()
        torch.cuda.synchronize()
        log(f"warmup {w}: {time.time() - t:.3f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / args.steps
    value = cell_steps * args.steps / wall
    log(f"timed {args.steps} steps: {wall:.3f} s wall, {ms_per_step:.1f} ms/step, {value:.4e} cell-steps/s")
    iters_h = iters.cpu().numpy().astype(np.int64)
    status_h = status.cpu().numpy()
    c_all = c_out.cpu().numpy()
    q_all = qoi.cpu().numpy()
    mean_h = [t.cpu().numpy() for t in mean_Y]

    # ---- dominant kernel: per-group HIP-event times of the solve kernels
    prof_opts = hm.make_opts(prec=hm.PREC_MIXED, tol=args.tol, max_outer=60, profile=1)
    step(prof_opts)
    torch.cuda.synchronize()
    groups = []
    for g in hm.henry_profile_last(ctx):
        members = [k for k, s in enumerate(solves) if s.nx == g["nx"]]
        alg = sum(solve_alg_bytes(solves[k].cells, solves[k].nsteps, iters_h[k]) for k in members)
        groups.append(dict(g, alg_bytes=alg,
                           outer=float(np.mean([iters_h[k] / solves[k].nsteps for k in members]))))
        log(f"group {g['nx']}x{g['ny']}: {g['nsolves']} solves x {g['cluster']} workgroups of {g['threads']}, "
            f"{g['ms']:.1f} ms, outer/step {groups[-1]['outer']:.2f}")
    roofline = roofline_entry(groups, load_traffic("mlmc_L4"))
    log(f"roofline: {roofline['achieved']:.0f} GB/s algorithmic, frac {roofline['frac']:.3f}")

    # ---- plain path: one solve per call, FP64 inner, per-grid median
    plain = None
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
                     per_solve_ms={f"{nx}x{nx // 2}": v * 1e3 for nx, v in per_grid_t.items()})

    # ---- errors against the oracle
    errs = errors_vs_stored_oracle(solves, pairs, c_all, q_all, mean_h)
    cpu = None
    if not args.no_cpu:
        cores = host_cores()
        cpu, full = cpu_baseline(solves, xi_h, cores)
        worst = 0.0
        for k, r in full:
            c = c_all[offs[k]:offs[k + 1]].reshape(solves[k].ny, solves[k].nx)
            worst = max(worst, np.abs(c - r["c"]).max() / np.abs(r["c"]).max())
        errs["c_sampled_live"] = worst
        if not args.no_plain:
            worst_p = 0.0
            for k, r in full[::9]:
                out = hm.solve(ctx, [grids[k]], xi=xi[k:k + 1].contiguous(), opts=plain_opts)
                c = out["c"].cpu().numpy().reshape(solves[k].ny, solves[k].nx)
                worst_p = max(worst_p, np.abs(c - r["c"]).max() / np.abs(r["c"]).max())
            errs["plain_fp64_c_sampled_live"] = worst_p
        log(f"oracle: {cpu['value']:.3e} cell-steps/s extrapolated on {cores} threads")
    log(f"errors vs oracle: {errs}")

    # ---- the 1024x512 KL workload (HBM-bound shape)
    kl = rl = None
    if not args.no_kl:
        kl, rl = run_kl(hm, torch, dev, args, log)

    rec = make_record(
        value=value, steps=args.steps, warmup=args.warmup, ms_per_step=ms_per_step, tol=args.tol,
        threads={f"{g['nx']}x{g['ny']}": g["threads"] for g in groups},
        clusters={f"{g['nx']}x{g['ny']}": g["cluster"] for g in groups},
        solves_per_s=len(solves) * args.steps / wall, plain=plain, errors=errs,
        nonconverged=int((status_h != 0).sum()),
        outer_per_step={f"{g['nx']}x{g['ny']}": g["outer"] for g in groups},
        roofline=roofline, roofline_kl=rl, kl=kl, cpu=cpu)

    if args.extras:
        extras = run_extras(hm, torch, dev, ctx, args, log, fine_grids, mean_Y, var_Y, qstats)
        text = json.dumps(sig(extras, 6), default=lambda o: o.item() if hasattr(o, "item") else str(o))
        print("[bench] extras " + text, file=sys.stderr, flush=True)
        if args.extras_out:
            with open(args.extras_out, "w") as f:
                f.write(text + "\n")
    ctx.close()
    print(record_line(rec), flush=True)


PHASES = {7: "step start", 13: "c update tail", 23: "residual p pass", 0: "residual p norms (reduction)",
          1: "coarsen p", 9: "p level 0 down", 10: "p cluster levels down", 11: "p leader levels",
          12: "p cluster levels up", 14: "p level 0 up", 2: "after p cycle", 15: "p update",
          21: "residual c pass", 3: "residual c barrier", 4: "coarsen c", 17: "c level 0 down",
          18: "c cluster levels down", 19: "c leader levels", 20: "c cluster levels up", 22: "c level 0 up",
          5: "after c cycle", 6: "c update"}


def phase_timers(clusters, tol):
    """Microseconds per outer iteration of each phase of the 256x128/800
    solves of the L = 4 workload (16 solves alone), on the leader's thread 0,
    from the HENRY_PHASE_TIMERS build: slots 8..31 of each solve's scratch
    region (100 MHz wall-clock ticks)."""
    import paper_2302_07804_amd as hm
    if not os.path.exists(hm.PHASE_TIMER_LIB_PATH):
        hm.build(hm.PHASE_TIMER_LIB_PATH, defines=("HENRY_PHASE_TIMERS",))
    hm.LIB_PATH = hm.PHASE_TIMER_LIB_PATH
    hm.lib()
    import torch
    dev = torch.device("cuda", 0)
    ctx = hm.Context(hi.PHYS, 0)
    n, grid = M_PER_LEVEL[-1], hi.level_grid(len(M_PER_LEVEL) - 1)
    xi = torch.tensor(hm.henry_sample_xi(hi.SEED, 4, 0, n, 3), dtype=torch.float64, device=dev)
    cells = grid[0] * grid[1]
    for K in clusters:
        opts = hm.make_opts(prec=hm.PREC_MIXED, tol=tol, max_outer=60, cluster=K)
        hm.solve(ctx, [grid] * n, xi=xi, opts=opts)
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = hm.solve(ctx, [grid] * n, xi=xi, opts=opts)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        ws = out["workspace"].cpu().numpy()
        desc = (n * 48 + 255) // 256 * 256
        sb = hm.henry_workspace_bytes([grid] * 2, opts) - hm.henry_workspace_bytes([grid], opts)
        acc = np.zeros(24)
        for k in range(n):
            off = (desc + k * sb) // 8 + 17 * cells  # the scratch doubles follow the 17 FP64 arrays
            acc += ws[off + 8:off + 32]
        acc /= n
        iters = float(out["iters"].cpu().numpy().mean())
        per = {PHASES.get(k, str(k)): round(acc[k] * 0.01 / iters, 1) for k in range(24) if acc[k] > 0}
        print(json.dumps(dict(cluster=K, wall_ms=round(1e3 * wall, 1), outer_per_step=round(iters / grid[2], 3),
                              us_per_outer=round(acc.sum() * 0.01 / iters, 1), phases=per)), flush=True)
    ctx.close()


def run_kl(hm, torch, dev, args, log):
    """32 KL samples (20 + 20 modes, recharge) on 1024x512 at tau = T/3200,
    the first `kl_steps` steps, one launch with clusters of workgroups:
    throughput, roofline of the solve kernel, and the mixed path's error
    against the FP64-inner path at a tight tolerance on sample 0."""
    nx, ny, r = KL_GRID
    steps = args.kl_steps
    ph = dict(hi.PHYS)
    ph["T"] = hi.PHYS["T"] * steps / r  # same tau, first steps
    kctx = hm.Context(ph, 0)
    kctx.set_kl(nx, ny)
    kxi = torch.tensor(hm.henry_sample_xi_kl(hi.SEED, 6, 0, KL_SAMPLES), dtype=torch.float64, device=dev)
    kg = [(nx, ny, steps)] * KL_SAMPLES
    o = hm.make_opts(prec=hm.PREC_MIXED, tol=args.tol, max_outer=60, profile=1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ko = hm.solve(kctx, kg, xi=kxi, opts=o)
    torch.cuda.synchronize()
    tk = time.perf_counter() - t
    g = hm.henry_profile_last(kctx)[0]
    it = ko["iters"].cpu().numpy().astype(np.int64)
    alg = sum(solve_alg_bytes(nx * ny, steps, int(v)) for v in it)
    rl = roofline_entry([dict(g, alg_bytes=alg)], load_traffic("kl_1024x512"))
    # mixed vs FP64-inner on sample 0
    ref = hm.solve(kctx, [kg[0]], xi=kxi[:1].contiguous(),
                   opts=hm.make_opts(prec=hm.PREC_FP64, tol=1e-9, max_outer=60))
    torch.cuda.synchronize()
    c0 = ko["c"][:nx * ny].cpu().numpy()
    rc = ref["c"].cpu().numpy()
    kl = dict(samples=KL_SAMPLES, steps=steps, seconds=tk, cell_steps_per_s=KL_SAMPLES * nx * ny * steps / tk,
              outer_per_step=float(it.mean() / steps), nonconverged=int((ko["status"].cpu().numpy() != 0).sum()),
              c_err_vs_fp64_tol1e9=float(np.abs(c0 - rc).max() / np.abs(rc).max()), cluster=g["cluster"])
    log(f"1024x512 KL: {KL_SAMPLES} x {steps} steps in {tk:.2f} s, frac {rl['frac']:.3f}, "
        f"error vs FP64 {kl['c_err_vs_fp64_tol1e9']:.2e}")
    kctx.close()
    del ko, ref
    return kl, rl


def run_extras(hm, torch, dev, ctx, args, log, fine_grids, mean_Y, var_Y, qstats):
    """The method's other workloads beside the metric (records for stderr)."""
    from paper_2302_07804_amd.mlmc import POINTS12, QUANTILES
    L = len(fine_grids) - 1
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
    extras["adjoint_128x64"] = dict(seconds=ta, forward_cell_steps_per_s=512 * 128 * 64 * 400 / ta,
                                    nonconverged=int((a["status"].cpu().numpy() != 0).sum()))
    log(f"adjoint 512 x 128x64/400: {ta:.2f} s")
    del a
    # adaptive MLMC (Sec. 3) on the L = 4 hierarchy
    t = time.perf_counter()
    am = hm.mlmc_run(ctx, [hi.level_grid(l) for l in range(5)], 0.05, m_pilot=16, seed=hi.SEED,
                     opts=hm.make_opts(prec=hm.PREC_MIXED, tol=args.tol, max_outer=60))
    extras["mlmc_adaptive_L4"] = dict(seconds=time.perf_counter() - t, m=[int(x) for x in am["m"]], EQ=am["EQ"],
                                      V=[float(x) for x in am["V"]], alpha=am["alpha"], beta=am["beta"],
                                      bias=am["bias"], mse_ok=am["mse_ok"])
    if args.kl_adjoint:
        nx, ny, r = KL_GRID
        kctx = hm.Context(hi.PHYS, 0)
        kctx.set_kl(nx, ny)
        kxi = torch.tensor(hm.henry_sample_xi_kl(hi.SEED, 6, 0, KL_SAMPLES), dtype=torch.float64, device=dev)
        t = time.perf_counter()
        ka = hm.adjoint(kctx, [KL_GRID] * KL_SAMPLES, xi=kxi,
                        opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-8, max_outer=60), ckpt_every=100,
                        adj_tol=1e-8, adj_max_it=60)
        torch.cuda.synchronize()
        seconds = time.perf_counter() - t
        g0 = ka["dq_dxi"][0].cpu().numpy()
        # central differences of the forward map: sample 0, coefficients 1, 21 and 41
        fd_h, ks = 1e-3, (0, 20, 40)
        x0 = kxi[0].cpu().numpy()
        pts = []
        for k in ks:
            for sgn in (1.0, -1.0):
                x = x0.copy()
                x[k] += sgn * fd_h
                pts.append(x)
        fo = hm.solve(kctx, [KL_GRID] * len(pts), xi=torch.tensor(np.array(pts), dtype=torch.float64, device=dev),
                      opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-9, max_outer=60))
        qf = fo["qoi"].cpu().numpy()
        fd = [(qf[2 * i] - qf[2 * i + 1]) / (2 * fd_h) for i in range(len(ks))]
        extras["kl_1024x512_adjoint"] = dict(
            seconds=seconds, nonconverged=int((ka["status"].cpu().numpy() != 0).sum()),
            fd_check={f"xi{k + 1}": dict(adjoint=float(g0[k]), central_difference=float(d),
                                         rel_diff=float(abs(g0[k] - d) / abs(d))) for k, d in zip(ks, fd)})
        log(f"1024x512 KL adjoint: {extras['kl_1024x512_adjoint']}")
        del ka, fo
        kctx.close()
    # the QMC reference of Fig. 11 on one level above the hierarchy
    npts, nsh = 128, 4
    ref_grid = hi.level_grid(L + 1)
    shifts = (hm.henry_sample_xi(hi.SEED, 99, 0, nsh, 3) + 1.0) / 2.0
    qr = hm.qmc_run(ctx, ref_grid, npts, shifts=list(shifts),
                    opts=hm.make_opts(prec=hm.PREC_MIXED, tol=args.tol, max_outer=60))
    kp = hm.point_cell(ref_grid, 1.60, -0.95)
    tel_c = hm.telescoped_at(ctx, fine_grids, mean_Y, 1.60, -0.95)
    extras["mlmc_vs_qmc"] = dict(seconds=qr["seconds"], qmc_EQ=qr["EQ"], qmc_EQ_se=qr["se"],
                                 qmc_c_point=float(qr["Ec"][kp].item()), mlmc_c_point_by_level=list(tel_c),
                                 mlmc_EQ_by_level=list(hm.telescoped_q(ctx, qstats)[0]))
    # the paper's own set-up: one sample per level of its hierarchy, Table 3's MLMC run, 600 time series
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
        per_sample[f"{g[0]}x{g[1]}/{g[2]}"] = time.perf_counter() - t
        del o
    m3 = [1714, 344, 78, 14, 4, 2]
    plevels = [hi.paper_level_grid(l) for l in range(6)]
    pr = hm.mlmc_fixed(pctx, plevels, m3, seed=hi.SEED, opts=popts, model="two_layer")
    g0 = hi.paper_level_grid(0)
    sr = hm.series_run(pctx, g0, hm.henry_qmc_points(1, 600, 3), 47, passages=((0, 1.2, True), (0, 1.7, True)),
                       opts=popts, model="two_layer")
    extras["paper_setup"] = dict(one_sample_seconds=per_sample, table3_seconds=pr["seconds"], table3_EQ=pr["EQ"],
                                 table3_nonconverged=pr["nonconverged"], series_600_seconds=sr["seconds"],
                                 Q_FW_median_at_T=float(sr["q"][QUANTILES.index(0.5), -1, 0].item()),
                                 points=len(POINTS12))
    pctx.close()
    return extras


if __name__ == "__main__":
    main()
