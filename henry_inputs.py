"""Seeded synthetic workloads for the Henry ensemble solves.

This module is the one piece shared by the oracle side and the GPU side of
the tests and the benchmark.  It holds inputs only -- physical constants,
grid/step hierarchies, sample-key lists and seeded random states for unit
checks -- and none of the method's arithmetic (no fluxes, no fields, no
random-number generator: both sides implement the sample generator
themselves from its published definition).

Workloads (all synthetic; the Henry problem is a benchmark problem, not a
dataset).  The uncertain inputs are porosity, permeability and recharge
(Sec. 2.2 of the paper); a level-l grid is (16 2^l) x (8 2^l) cells with
50 2^l implicit Euler steps to T = 3.6e4 s (space and time refined together,
Sec. 2.3).
"""
from __future__ import annotations

import dataclasses

import numpy as np

# Physical constants (SI).  Table 1 of the paper lists rho0, mu, D and E[phi];
# the workload fixes rho1 = 1025, g = 9.81, k0 = 1.0194e-9, q_in = 6.6e-5 m/s
# and T = 3.6e4 s.
PHYS = dict(rho0=1000.0, rho1=1025.0, mu=1e-3, g=9.81, D=18.8571e-6,
            phi0=0.35, k0=1.0194e-9, q_in=6.6e-5, T=3.6e4)
PHYS_ORDER = ("rho0", "rho1", "mu", "g", "D", "phi0", "k0", "q_in", "T")

SEED = 0

# The paper's own set-up (Table 1 and Sec. 4): Table 1's constants, the
# recharge 6.6e-2 kg/s read as 6.6e-5 m/s of fresh water, T = 6016 s, and a
# hierarchy that starts from 32 x 16 cells with r0 = 188 steps (Table 2).
# Its random fields are the two-layer porosity model (field model
# "two_layer").
PHYS_TABLE1 = dict(rho0=1000.0, rho1=1024.99, mu=1e-3, g=9.8, D=18.8571e-6,
                   phi0=0.35, k0=1.020408e-9, q_in=6.6e-5, T=6016.0)


def paper_level_grid(level: int) -> tuple[int, int, int]:
    """(nx, ny, nsteps) of level `level` of the paper's hierarchy."""
    return 32 << level, 16 << level, 188 << level


def level_grid(level: int) -> tuple[int, int, int]:
    """(nx, ny, nsteps) of hierarchy level `level`."""
    nx = 16 << level
    return nx, nx // 2, 50 << level


@dataclasses.dataclass(frozen=True)
class Solve:
    """One deterministic solve: a grid, a step count and a sample key."""
    nx: int
    ny: int
    nsteps: int
    level: int      # key level (RNG stream), not necessarily the grid level
    index: int      # key sample index

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    @property
    def cell_steps(self) -> int:
        return self.nx * self.ny * self.nsteps


def mlmc_solves(m_per_level, seed_level_offset: int = 0):
    """Solve list of an MLMC run: level 0 solves g_0 on grid 0; level l > 0
    solves the pair (g_l, g_{l-1}) on grids l and l-1 with the same key
    (l, i), as in the telescoping estimator eq:A (Sec. 3).  Returns
    (solves, pairs) where pairs[l] = (fine indices, coarse indices or None)."""
    solves: list[Solve] = []
    pairs = []
    for lev, m in enumerate(m_per_level):
        fine = []
        coarse = []
        nx, ny, r = level_grid(lev)
        for i in range(m):
            fine.append(len(solves))
            solves.append(Solve(nx, ny, r, lev + seed_level_offset, i))
        if lev > 0:
            cx, cy, cr = level_grid(lev - 1)
            for i in range(m):
                coarse.append(len(solves))
                solves.append(Solve(cx, cy, cr, lev + seed_level_offset, i))
        pairs.append((fine, coarse if lev > 0 else None))
    return solves, pairs


# The five workloads.  Sizes are what the benchmark and the parity tests use.
CONFIGS = {
    "single_16x8": dict(solves=[Solve(16, 8, 50, 0, 0)]),
    "pair_64x32_32x16": dict(m=256),
    "mlmc_L4": dict(m=(4096, 1024, 256, 64, 16)),
    "adjoint_128x64": dict(grid=(128, 64, 400), samples=512, ckpt=20),
    "kl_1024x512": dict(grid=(1024, 512, 3200), samples=32, ckpt=100),
}


def pair_solves(m: int = 256):
    """Fine 64x32/200 and coarse 32x16/100 sharing keys (2, i)."""
    fine = [Solve(64, 32, 200, 2, i) for i in range(m)]
    coarse = [Solve(32, 16, 100, 2, i) for i in range(m)]
    return fine, coarse


def random_state(nx: int, ny: int, seed: int, phys=PHYS):
    """Seeded random (p, c, c_prev, phi, K, q) for residual-level checks:
    p near the fresh hydrostatic profile, c and c_prev in [0, 1], phi and K
    in the ranges the closed-form fields produce."""
    rng = np.random.default_rng(seed)
    h = 1.0 / ny
    y = -1.0 + (np.arange(ny) + 0.5) * h
    p = (-phys["rho0"] * phys["g"] * y)[:, None] + rng.uniform(-50.0, 50.0, (ny, nx))
    c = rng.uniform(0.0, 1.0, (ny, nx))
    cn = np.clip(c + rng.uniform(-0.1, 0.1, (ny, nx)), 0.0, 1.0)
    phi = phys["phi0"] * (1.0 + 0.2 * rng.uniform(-1.0, 1.0, (ny, nx)))
    K = phys["k0"] * np.exp(0.5 * rng.uniform(-1.0, 1.0, (ny, nx)))
    q = phys["q_in"] * (1.0 + 0.2 * rng.uniform(-1.0, 1.0))
    return p, c, cn, phi, K, q
