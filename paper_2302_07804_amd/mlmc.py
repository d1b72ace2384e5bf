"""Adaptive multilevel Monte Carlo for the expected QoI (Sec. 3 of arXiv
2302.07804): pilot runs give the per-level variances V_l of
Y_l = Q_l - Q_{l-1} and the GPU cost s_l of one sample pair; eq:M_ell gives
the sample counts for the estimator variance eps^2 / 2; the final batch
solves every level's samples at once; the MSE split eq:MSE checks the bias
of the finest level, estimated from the fitted weak rate.

The quasi-Monte Carlo reference of Sec. 4 (Fig. 11): a randomly shifted
Halton rule on one fine grid gives E[Q] and E[c] with an error estimate from
the spread of the shifts; MLMC estimates truncated after each level are
compared with it at a point.

Orchestration only: the solves (henry_solve_batch), the level statistics
(mlmc_level_estimate, henry_sample_stats), the estimator sums over levels
(henry_mlmc_telescope, FP64 on the device), the points (henry_qmc_points)
and the planning arithmetic (henry_mlmc_allocate, henry_mlmc_rates) are
calls into libhenry; this module copies results to the host, it does not
add them up."""
from __future__ import annotations

import time

import numpy as np

from . import (FIELD_CLOSED3, Context, Opts, henry_first_passage, henry_mlmc_allocate, henry_mlmc_rates,
               henry_mlmc_telescope, henry_qmc_points, henry_sample_stats, henry_sample_xi, mlmc_level_estimate,
               solve, telescoped_q)


def _pairs(levels, m, seed):
    """Solve list, xi and per-level (fine, coarse) index ranges: level l
    solves grid l and grid l-1 for samples 0 .. m[l]-1, both with the key
    (seed, l, i) (eq:A)."""
    solves, xis, ranges = [], [], []
    for l, ml in enumerate(m):
        xi = henry_sample_xi(seed, l, 0, int(ml), 3)
        f0 = len(solves)
        solves += [tuple(levels[l])] * int(ml)
        xis.append(xi)
        c0 = len(solves)
        if l > 0:
            solves += [tuple(levels[l - 1])] * int(ml)
            xis.append(xi)
        ranges.append((f0, c0, len(solves)))
    return solves, np.concatenate(xis), ranges


def _level_statistics(ctx, levels, m, outs, with_var=False):
    """mlmc_level_estimate over per-level outputs: outs[l] = (solves, out,
    (f0, c0, c1)) with the fine solves f0..c0-1 and the coarse ones c0..c1-1."""
    import torch
    dev = torch.device("cuda", ctx.device)
    L = len(levels) - 1
    c_fine, c_coarse, q_fine, q_coarse = [], [], [], []
    for l, (sol, out, (f0, c0, c1)) in enumerate(outs):
        offs = np.concatenate([[0], np.cumsum([s[0] * s[1] for s in sol])])
        c_fine.append(out["c"][offs[f0]:offs[c0]])
        q_fine.append(out["qoi"][f0:c0])
        c_coarse.append(out["c"][offs[c0]:offs[c1]] if l > 0 else None)
        q_coarse.append(out["qoi"][c0:c1] if l > 0 else None)
    mean_Y = [torch.empty(g[0] * g[1], dtype=torch.float64, device=dev) for g in levels]
    var_Y = [torch.empty(g[0] * g[1], dtype=torch.float64, device=dev) for g in levels]
    qstats = torch.empty(2 * (L + 1), dtype=torch.float64, device=dev)
    Ec = torch.empty(levels[-1][0] * levels[-1][1], dtype=torch.float64, device=dev)
    var_est = torch.empty(2, dtype=torch.float64, device=dev)
    mlmc_level_estimate(ctx, levels, m, c_fine, c_coarse, q_fine, q_coarse, mean_Y, var_Y, qstats, Ec, var_est)
    EQ, _ = telescoped_q(ctx, qstats)
    torch.cuda.synchronize(dev)
    qs = qstats.cpu().numpy().reshape(L + 1, 2)
    if with_var:
        return qs[:, 0].copy(), qs[:, 1].copy(), float(var_est[0].item()), Ec, mean_Y, var_Y, float(EQ[-1])
    return qs[:, 0].copy(), qs[:, 1].copy(), float(var_est[0].item()), Ec, mean_Y, float(EQ[-1])


def _point_statistics(ctx, levels, m, outs):
    """Level means and variances of c at the trace's one point at T: outs[l]
    = (out, (f0, c0, c1)) with the fine solves f0..c0-1 and the coarse ones
    c0..c1-1 of level l (henry_sample_stats on their difference).  Returns
    the host copies of the level means and variances, and the telescoped
    estimate and sum V_l / m_l (henry_mlmc_telescope)."""
    import torch
    mean, var = [], []
    for l, (out, (f0, c0, c1)) in enumerate(outs):
        fine = out["trace"][f0:c0, 0, 1:2].contiguous()
        coarse = out["trace"][c0:c1, 0, 1:2].contiguous() if l > 0 else None
        mu, v, _ = henry_sample_stats(ctx, fine, (), x_sub=coarse)
        mean.append(mu)
        var.append(v)
    pm, pv = henry_mlmc_telescope(ctx, mean, var, m, nvals=1)
    torch.cuda.synchronize(mean[0].device)
    est, var_est = float(pm[-1, 0].item()), float(pv[-1, 0].item())
    mean = np.array([float(t.item()) for t in mean])
    var = np.array([float(t.item()) for t in var])
    return mean, var, est, var_est


def mlmc_run(ctx: Context, levels, eps: float, m_pilot: int = 32, seed: int = 0, opts: Opts | None = None,
             max_samples: int | None = None, model: str | None = None, point=None):
    """Adaptive MLMC estimate of E[Q] (or, with point = (x, y), of c at that
    point at T, the paper's own QoI of Table 3) to root-mean-square error eps.

    levels: fine grids (nx, ny, nsteps) of levels 0..L (nx = 2 ny, each
    twice the one before it); level l > 0 pairs grid l with grid l-1.
    model: the random fields of the three coefficients (None or "closed":
    the closed forms; "two_layer": the two-layer porosity model).
    Returns a dict: EQ (sum of the level means), var_est (sum V_l / m_l),
    m, V, s (seconds per sample at each level, fine and coarse solve), the
    level means, alpha, beta, the bias estimate, mse_ok (var_est <= eps^2/2
    and bias^2 <= eps^2/2), the final batch's seconds, and for E[Q] also
    E[c] on the finest grid and the level mean fields of Y_l = c_l - c_{l-1}
    (device tensors)."""
    if point is not None:
        return _mlmc_run_point(ctx, levels, eps, m_pilot, seed, opts, max_samples, model, point)
    import torch
    levels = [tuple(int(v) for v in g) for g in levels]
    L = len(levels) - 1
    if L < 0 or m_pilot < 2:
        raise ValueError("need at least one level and a pilot of at least two samples")
    dev = torch.device("cuda", ctx.device)
    # ---- pilot: one batch per level, timed on the GPU stream
    pilot, s = [], []
    for l in range(L + 1):
        sol, xi, rng = _pairs(levels[:l + 1], [0] * l + [m_pilot], seed)
        xi_d = torch.tensor(xi, dtype=torch.float64, device=dev)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        out = solve(ctx, sol, xi=xi_d, opts=opts, model=model)
        torch.cuda.synchronize(dev)
        s.append((time.perf_counter() - t0) / m_pilot)
        pilot.append((sol, out, rng[l]))
    mean_p, V, _, _, _, _ = _level_statistics(ctx, levels, [m_pilot] * (L + 1), pilot)
    # ---- allocation (eq:M_ell) for the variance half of the MSE (eq:MSE)
    m, cost = henry_mlmc_allocate(V, np.array(s), eps * eps / 2)
    m = np.maximum(m, m_pilot)
    if max_samples is not None:
        m = np.minimum(m, max_samples)
    # ---- final batch: every level's samples at once
    res = mlmc_fixed(ctx, levels, m, seed=seed, opts=opts, model=model)
    half = eps * eps / 2
    res.update(V_pilot=V, s=np.array(s), planned_cost=cost,
               mse_ok=bool(res["var_est"] <= half * (1 + 1e-12) and (L < 2 or res["bias"] ** 2 <= half)))
    return res


def _mlmc_run_point(ctx, levels, eps, m_pilot, seed, opts, max_samples, model, point):
    """mlmc_run for c at a point at T: every solve records one time-series
    record (the final state) at the point."""
    import torch
    levels = [tuple(int(v) for v in g) for g in levels]
    L = len(levels) - 1
    if L < 0 or m_pilot < 2:
        raise ValueError("need at least one level and a pilot of at least two samples")
    dev = torch.device("cuda", ctx.device)
    trace = (1, [tuple(point)])
    pilot, s = [], []
    for l in range(L + 1):
        sol, xi, rng = _pairs(levels[:l + 1], [0] * l + [m_pilot], seed)
        xi_d = torch.tensor(xi, dtype=torch.float64, device=dev)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        out = solve(ctx, sol, xi=xi_d, opts=opts, model=model, trace=trace)
        torch.cuda.synchronize(dev)
        s.append((time.perf_counter() - t0) / m_pilot)
        pilot.append((out, rng[l]))
    _, V, _, _ = _point_statistics(ctx, levels, [m_pilot] * (L + 1), pilot)
    m, cost = henry_mlmc_allocate(V, np.array(s), eps * eps / 2)
    m = np.maximum(m, m_pilot)
    if max_samples is not None:
        m = np.minimum(m, max_samples)
    sol, xi, rng = _pairs(levels, m, seed)
    xi_d = torch.tensor(xi, dtype=torch.float64, device=dev)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    out = solve(ctx, sol, xi=xi_d, opts=opts, model=model, trace=trace)
    torch.cuda.synchronize(dev)
    seconds = time.perf_counter() - t0
    status = out["status"].cpu().numpy()
    mean, var, est, var_est = _point_statistics(ctx, levels, m, [(out, r) for r in rng])
    alpha = beta = bias = float("nan")
    if L >= 2:
        alpha, beta, bias = henry_mlmc_rates(mean, var, 1)
    half = eps * eps / 2
    return dict(EQ=est, var_est=var_est, m=m, V=var, V_pilot=V, s=np.array(s), mean=mean,
                alpha=alpha, beta=beta, bias=bias, planned_cost=cost, seconds=seconds,
                nonconverged=int((status != 0).sum()),
                mse_ok=bool(var_est <= half * (1 + 1e-12) and (L < 2 or bias * bias <= half)))


def mlmc_fixed(ctx: Context, levels, m, seed: int = 0, opts: Opts | None = None, model: str | None = None):
    """MLMC estimate with given sample counts m[l] (eq:A): every level's
    pairs solved in one batch, then the level statistics.  Returns a dict:
    EQ, var_est (sum V_l / m_l), m, V, the level means, alpha, beta and the
    bias estimate (nan below three levels), the batch's seconds,
    nonconverged, E[c] on the finest grid and the level mean and variance
    fields of Y_l = c_l - c_{l-1} (device tensors)."""
    import torch
    levels = [tuple(int(v) for v in g) for g in levels]
    L = len(levels) - 1
    m = np.asarray(m, dtype=np.int64)
    if len(m) != L + 1 or (m < 2).any():
        raise ValueError("one sample count of at least two per level")
    dev = torch.device("cuda", ctx.device)
    sol, xi, rng = _pairs(levels, m, seed)
    xi_d = torch.tensor(xi, dtype=torch.float64, device=dev)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    out = solve(ctx, sol, xi=xi_d, opts=opts, model=model)
    torch.cuda.synchronize(dev)
    seconds = time.perf_counter() - t0
    status = out["status"].cpu().numpy()
    mean, var, var_est, Ec, mean_Y, var_Y, EQ = _level_statistics(ctx, levels, m, [(sol, out, r) for r in rng],
                                                                  with_var=True)
    alpha = beta = bias = float("nan")
    if L >= 2:
        alpha, beta, bias = henry_mlmc_rates(mean, var, 1)
    return dict(EQ=EQ, var_est=var_est, m=m, V=var, mean=mean, alpha=alpha, beta=beta, bias=bias,
                seconds=seconds, nonconverged=int((status != 0).sum()), Ec=Ec, mean_Y=mean_Y, var_Y=var_Y)


def point_cell(grid, x: float, y: float) -> int:
    """Index in the [ny][nx] layout of the cell of `grid` that contains the
    point (x, y) of D = [0,2] x [-1,0].  The finite-volume solution is
    constant per cell, so this cell's value is the solution at the point,
    and on nested grids the injected coarse value at the point is the
    coarse cell's.  A point on a cell face is ambiguous and rejected."""
    nx, ny = int(grid[0]), int(grid[1])
    if not (0.0 < x < 2.0 and -1.0 < y < 0.0):
        raise ValueError(f"({x}, {y}) is not inside the domain")
    u, v = x * ny, (y + 1.0) * ny  # h = 1 / ny
    if u == int(u) or v == int(v):
        raise ValueError(f"({x}, {y}) lies on a cell face of {nx}x{ny}")
    return int(v) * nx + int(u)


def qmc_run(ctx: Context, grid, n: int, shifts=None, first: int = 1, opts: Opts | None = None,
            model: str | None = None):
    """Quasi-Monte Carlo estimate of E[Q] and E[c] on one grid (nx, ny,
    nsteps): R = len(shifts) Halton rules of n points each, rule r rotated
    by shifts[r] (values in [0, 1); None: one unshifted rule), all R*n
    solves in one batch.  Returns a dict: EQ (mean over all points),
    EQ_shift (the R rule means), se (their standard deviation over sqrt(R),
    the usual error estimate of a randomly shifted rule; nan for R = 1), Ec
    (mean field), Ec_shift (each rule's mean field) and Varc (the sample
    variance of c per cell over all points; device tensors), seconds (the
    batch), nonconverged."""
    import torch
    grid = tuple(int(v) for v in grid)
    if n < 2:
        raise ValueError("a QMC rule needs at least two points")
    shifts = [None] if shifts is None else [np.asarray(sh, dtype=np.float64) for sh in shifts]
    R = len(shifts)
    dev = torch.device("cuda", ctx.device)
    xi = np.concatenate([henry_qmc_points(first, n, 3, sh) for sh in shifts])
    xi_d = torch.tensor(xi, dtype=torch.float64, device=dev)
    sol = [grid] * (R * n)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    out = solve(ctx, sol, xi=xi_d, opts=opts, model=model)
    torch.cuda.synchronize(dev)
    seconds = time.perf_counter() - t0
    status = out["status"].cpu().numpy()
    cells = grid[0] * grid[1]
    mean, _, _, Ec, _, var_Y, _ = _level_statistics(ctx, [grid], [R * n], [(sol, out, (0, R * n, R * n))],
                                                    with_var=True)
    Ec_shift = []
    for r in range(R):
        sl = dict(c=out["c"][r * n * cells:(r + 1) * n * cells], qoi=out["qoi"][r * n:(r + 1) * n])
        _, _, _, Er, _, _ = _level_statistics(ctx, [grid], [n], [(sol[:n], sl, (0, n, n))])
        Ec_shift.append(Er)
    # each rule's mean (column r of the [n][R] view), then the spread of the R means
    rule_mean, _, _ = henry_sample_stats(ctx, out["qoi"].view(R, n).t().contiguous(), ())
    se = float("nan")
    if R > 1:
        _, rv, _ = henry_sample_stats(ctx, rule_mean.view(R, 1), ())
        se = float(np.sqrt(rv.item() / R))
    per = rule_mean.cpu().numpy()
    return dict(EQ=float(mean[0]), EQ_shift=per, se=se, Ec=Ec, Ec_shift=Ec_shift, Varc=var_Y[0], seconds=seconds,
                nonconverged=int((status != 0).sum()))


def telescoped_at(ctx: Context, levels, mean_Y, x: float, y: float) -> np.ndarray:
    """MLMC estimates of E[c] at the point (x, y) truncated after each level:
    entry L is the sum over l <= L of level l's mean difference field at the
    cell containing the point (the partial sums of the telescoping estimator
    eq:A that Fig. 11 compares with the reference), summed on the device.
    mean_Y[l] is level l's field on grid l, as mlmc_run returns it."""
    offs = [point_cell(levels[l], x, y) for l in range(len(levels))]
    pm, _ = henry_mlmc_telescope(ctx, list(mean_Y), None, None, offsets=offs, nvals=1)
    return pm[:, 0].cpu().numpy()


# the paper's output points (eq:12points) and quantiles (Figs. 4 and 6)
POINTS12 = ((1.10, -0.95), (1.35, -0.95), (1.60, -0.95), (1.85, -0.95), (1.10, -0.75), (1.35, -0.75),
            (1.60, -0.75), (1.85, -0.75), (1.10, -0.50), (1.35, -0.50), (1.60, -0.50), (1.85, -0.50))
QUANTILES = (0.025, 0.25, 0.5, 0.75, 0.975)


def series_run(ctx: Context, grid, xi, nrec: int, points=POINTS12, probs=QUANTILES, passages=(),
               c_fresh: float = 0.012178, opts: Opts | None = None, model: str | None = None):
    """Time-series statistics of an ensemble on one grid (Sec. 4, Figs. 4-7):
    every sample xi[k] solved with nrec records of the fresh-water area and
    c at the points, then per record and quantity the mean, variance and
    quantiles over the samples, and for each (col, threshold, below) in
    passages the first-passage record of every sample and their histogram
    (col 0 is the fresh-water area, col 1 + i point i).  Returns a dict of
    device tensors (trace [n][nrec][1 + npts], mean and var [nrec][1 + npts],
    q [len(probs)][nrec][1 + npts], passage list of (t, hist)), the batch's
    seconds and the number of solves that did not converge."""
    import torch
    grid = tuple(int(v) for v in grid)
    dev = torch.device("cuda", ctx.device)
    xi_d = torch.as_tensor(np.ascontiguousarray(xi, dtype=np.float64), device=dev)
    n = int(xi_d.shape[0])
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    out = solve(ctx, [grid] * n, xi=xi_d, opts=opts, model=model, trace=(nrec, list(points), c_fresh))
    torch.cuda.synchronize(dev)
    seconds = time.perf_counter() - t0
    tr = out["trace"]
    nv = nrec * (1 + len(points))
    mean, var, q = henry_sample_stats(ctx, tr.view(n, nv), probs)
    pas = [henry_first_passage(ctx, tr, col, thr, below) for col, thr, below in passages]
    torch.cuda.synchronize(dev)
    shape = (nrec, 1 + len(points))
    return dict(trace=tr, mean=mean.view(shape), var=var.view(shape), q=q.view((len(probs),) + shape),
                passage=pas, seconds=seconds, nonconverged=int((out["status"].cpu().numpy() != 0).sum()))


def mlmc_series(ctx: Context, levels, m, nrec: int, points=POINTS12, seed: int = 0, c_fresh: float = 0.012178,
                opts: Opts | None = None, model: str | None = None):
    """MLMC estimate of mean time series (Sec. 4: the paper estimates the
    mean of Q_FW(t) and of c at points by MLMC): the telescoping sum eq:A
    per record and quantity, level l's differences Y_l = g_l - g_{l-1}
    taken between the fine and coarse solves of its pairs (keys (seed, l,
    i)).  Each level's nsteps should be a multiple of nrec so that the
    records of all levels fall at the same times k T / nrec.  Returns a
    dict: mean [nrec][1 + npts] (the estimate), var_est (sum_l V_l / m_l,
    same shape), level_mean, level_var, level_min and level_max (the
    smallest and largest Y_l over the level's samples) [L+1][nrec][1 + npts],
    the batch's seconds and the number of non-converged solves."""
    import torch
    levels = [tuple(int(v) for v in g) for g in levels]
    L = len(levels) - 1
    m = np.asarray(m, dtype=np.int64)
    if len(m) != L + 1 or (m < 2).any():
        raise ValueError("one sample count of at least two per level")
    dev = torch.device("cuda", ctx.device)
    sol, xi, rng = _pairs(levels, m, seed)
    xi_d = torch.tensor(xi, dtype=torch.float64, device=dev)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    out = solve(ctx, sol, xi=xi_d, opts=opts, model=model, trace=(nrec, list(points), c_fresh))
    torch.cuda.synchronize(dev)
    seconds = time.perf_counter() - t0
    tr = out["trace"]
    nv = nrec * (1 + len(points))
    lm, lv, lq = [], [], []
    for l, (f0, c0, c1) in enumerate(rng):
        fine = tr[f0:c0].reshape(c0 - f0, nv)
        coarse = tr[c0:c1].reshape(c1 - c0, nv) if l > 0 else None
        mean, var, q = henry_sample_stats(ctx, fine, (0.0, 1.0), x_sub=coarse)
        lm.append(mean)
        lv.append(var)
        lq.append(q)
    pm, pv = henry_mlmc_telescope(ctx, lm, lv, m, nvals=nv)
    torch.cuda.synchronize(dev)
    shape = (nrec, 1 + len(points))
    est = pm[-1].cpu().numpy().reshape(shape)
    var_est = pv[-1].cpu().numpy().reshape(shape)
    lm = np.stack([v.cpu().numpy().reshape(shape) for v in lm])
    lv = np.stack([v.cpu().numpy().reshape(shape) for v in lv])
    lq = np.stack([v.cpu().numpy().reshape((2,) + shape) for v in lq])
    return dict(mean=est, var_est=var_est, level_mean=lm, level_var=lv,
                level_min=lq[:, 0], level_max=lq[:, 1], m=m, seconds=seconds,
                nonconverged=int((out["status"].cpu().numpy() != 0).sum()))
