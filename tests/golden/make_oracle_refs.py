"""Write the stored oracle references of the L = 4 MLMC workload.

Every value this script stores comes from `oracle/` alone (plain FP64
Newton with a banded LU) on samples drawn by the oracle's own Philox
generator; nothing is read from the HIP library.  The GPU parity tests
compare the batched mixed-precision solves of the same samples with these
files, because the finer levels take the oracle minutes to hours per solve
and cannot be recomputed inside a test.

Workload: level l is a (16 2^l) x (8 2^l) grid with 50 2^l implicit Euler
steps to T = 3.6e4 s; level l > 0 pairs the fine solve with a coarse solve
on level l - 1 that shares its sample key (seed 0, l, i) (eq:A, Sec. 3 of
the paper); m = 4096, 1024, 256, 64, 16 samples.

Files (numpy .npz, no pickled objects):
  oracle_mlmc_L4_level{l}.npz, l = 0..3 -- every sample of the level:
      Q_fine[m], Q_coarse[m] (absent at l = 0), the level-difference mean
      and unbiased variance fields mean_Y, var_Y [ny][nx] (coarse fields
      injected, oracle.level_stats), the QoI difference's mean and variance
      q_stats[2], and the c fields of sample 0 (c_fine0, c_coarse0).
  oracle_mlmc_L4_level4_sample0.npz -- sample 0 of level 4 only (a
      256x128/800 oracle solve takes hours): c_fine0, Q_fine0, c_coarse0,
      Q_coarse0.

Usage:
  python tests/golden/make_oracle_refs.py levels 0 1 2 --threads 6
  python tests/golden/make_oracle_refs.py levels 3 --threads 6
  python tests/golden/make_oracle_refs.py finest
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import henry_inputs as hi  # noqa: E402
import oracle  # noqa: E402

M_PER_LEVEL = hi.CONFIGS["mlmc_L4"]["m"]


def level_file(level: int) -> str:
    return os.path.join(HERE, f"oracle_mlmc_L4_level{level}.npz")


FINEST_FILE = os.path.join(HERE, "oracle_mlmc_L4_level4_sample0.npz")


def run_level(level: int, threads: int) -> None:
    m = M_PER_LEVEL[level]
    xi = oracle.sample_xi(hi.SEED, level, 0, m, 3)
    fx, fy, fr = hi.level_grid(level)
    jobs = [(fx, fy, fr, xi[i]) for i in range(m)]
    if level > 0:
        cx, cy, cr = hi.level_grid(level - 1)
        jobs += [(cx, cy, cr, xi[i]) for i in range(m)]
    t = time.time()
    res = oracle.solve_many(hi.PHYS, jobs, threads=threads)
    c_f = np.array([r["c"] for r in res[:m]])
    q_f = np.array([r["qoi"] for r in res[:m]])
    out = dict(m=np.int64(m), grid=np.array([fx, fy, fr]), Q_fine=q_f, c_fine0=c_f[0])
    if level > 0:
        c_c = np.array([r["c"] for r in res[m:]])
        q_c = np.array([r["qoi"] for r in res[m:]])
        mean, var = oracle.level_stats(c_f, c_c)
        qm, qv = oracle.level_stats(q_f, q_c)
        out.update(Q_coarse=q_c, c_coarse0=c_c[0])
    else:
        mean, var = oracle.level_stats(c_f)
        qm, qv = oracle.level_stats(q_f)
    out.update(mean_Y=mean, var_Y=var, q_stats=np.array([qm, qv]))
    np.savez_compressed(level_file(level), **out)
    print(f"level {level}: {len(jobs)} oracle solves on {threads} threads in {time.time() - t:.0f} s "
          f"-> {level_file(level)}", flush=True)


def run_finest(threads: int) -> None:
    xi = oracle.sample_xi(hi.SEED, 4, 0, 1, 3)[0]
    fx, fy, fr = hi.level_grid(4)
    cx, cy, cr = hi.level_grid(3)
    t = time.time()
    res = oracle.solve_many(hi.PHYS, [(fx, fy, fr, xi), (cx, cy, cr, xi)], threads=threads)
    np.savez_compressed(FINEST_FILE, grid=np.array([fx, fy, fr]), c_fine0=res[0]["c"], Q_fine0=res[0]["qoi"],
                        c_coarse0=res[1]["c"], Q_coarse0=res[1]["qoi"])
    print(f"level 4 sample 0: fine and coarse oracle solves in {time.time() - t:.0f} s -> {FINEST_FILE}",
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=("levels", "finest"))
    ap.add_argument("levels", nargs="*", type=int)
    ap.add_argument("--threads", type=int, default=len(os.sched_getaffinity(0)))
    a = ap.parse_args()
    if a.what == "finest":
        run_finest(min(a.threads, 2))
    else:
        for lev in a.levels:
            if not 0 <= lev <= 3:
                raise SystemExit("levels 0..3 (level 4 only through 'finest')")
            run_level(lev, a.threads)


if __name__ == "__main__":
    main()
