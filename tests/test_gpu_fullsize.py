"""Parity at the workloads' full sizes, on sampled outputs the oracle can
compute one by one and on properties that hold at any size.

  * mlmc_L4 (6816 solves, 16x8/50 ... 256x128/800), in the launch
    configuration of the benchmark (mixed precision, tol 1e-7): every solve
    converges; sampled solves of levels 0-2 against the oracle (1e-5); one
    256x128/800 solve against the FP64 path at tol 1e-10; the level
    statistics of the batch against numpy on the same outputs.
  * pair_64x32_32x16 (256 pairs, FP64, tol 1e-11): sampled pairs against
    the oracle (1e-8); level-difference statistics against numpy.
  * adjoint_128x64 (512 samples, 400 steps, checkpoints every 20, mixed,
    forward and adjoint tolerances 1e-10):
    every solve converges; dQ/dxi of samples 0..7 against central
    differences of the FP64 forward map (h = 1e-6, 1e-4 relative).
  * kl_1024x512 (KL fields, tau = T/3200): the first three steps of two
    samples, mixed and FP64 inner precision; the final state satisfies the
    oracle's FP64 discrete equations (the oracle evaluates its residual at
    the GPU's state; its banded direct solve is out of reach at 2^20
    unknowns); the 41-coefficient gradient equals the projection of the
    per-cell gradients on the oracle's KL basis.  At full length (3200
    steps, checkpoints every 100) the adjoint's dQ/dxi of two samples in
    xi1, xi21 and xi41 (a porosity mode, a log-permeability mode, the
    recharge) agrees with central differences of the forward map to 1e-4.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import henry_inputs as hi
import oracle
import paper_2302_07804_amd as hm
from oracle import kl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible for a gpu-marked test")
    hm.lib()
    oracle.build(force=False)
    return torch


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    c = hm.Context(hi.PHYS, 0)
    yield c
    c.close()


def dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def xi_of(solves, dim=3):
    """xi per solve from the library sampler, keyed (seed, level, index)."""
    out = np.empty((len(solves), dim))
    for k, s in enumerate(solves):
        out[k] = hm.henry_sample_xi(hi.SEED, s.level, s.index, 1, dim)[0]
    return out


def oracle_many(jobs):
    """jobs: (nx, ny, r, level, index) -> oracle results, xi from the oracle's own sampler."""
    def one(jb):
        nx, ny, r, lev, idx = jb
        xi = oracle.sample_xi(hi.SEED, lev, idx, 1, 3)[0]
        return oracle.solve_xi(hi.PHYS, nx, ny, r, xi)
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        return list(ex.map(one, jobs))


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_mlmc_L4_full_batch_sampled_against_oracle(torch_cuda, ctx):
    torch = torch_cuda
    solves, pairs = hi.mlmc_solves(hi.CONFIGS["mlmc_L4"]["m"])
    grids = [(s.nx, s.ny, s.nsteps) for s in solves]
    print(f"mlmc_L4 full batch: {len(solves)} solves", flush=True)
    opts = hm.make_opts(prec=hm.PREC_MIXED, tol=1e-7)
    out = hm.solve(ctx, grids, xi=dev(torch, xi_of(solves)), opts=opts)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert (st == hm.STATUS_OK).all(), np.unique(st, return_counts=True)
    cs = hm.unpack(out["c"], grids)
    q = out["qoi"].cpu().numpy()
    rng = np.random.default_rng(11)
    picks = list(rng.choice(pairs[0][0], 3, replace=False))
    i1 = int(rng.integers(len(pairs[1][0])))
    picks += [pairs[1][0][i1], pairs[1][1][i1]]
    i2 = int(rng.integers(len(pairs[2][0])))
    picks += [pairs[2][0][i2], pairs[2][1][i2]]
    print(f"oracle on solves {picks}", flush=True)
    refs = oracle_many([(solves[k].nx, solves[k].ny, solves[k].nsteps, solves[k].level, solves[k].index)
                        for k in picks])
    for k, r in zip(picks, refs):
        assert rel(cs[k].cpu().numpy(), r["c"]) <= 1e-5, (k, solves[k])
        assert abs(q[k] - r["qoi"]) <= 1e-5 * abs(r["qoi"]), (k, solves[k])
    # one finest-level solve against the FP64 path at a tight tolerance
    k4 = pairs[4][0][int(rng.integers(len(pairs[4][0])))]
    s4 = solves[k4]
    print(f"FP64 check of solve {k4} {s4}", flush=True)
    tight = hm.solve(ctx, [(s4.nx, s4.ny, s4.nsteps)], xi=dev(torch, xi_of([s4])),
                     opts=hm.make_opts(prec=hm.PREC_FP64, tol=1e-10, max_outer=60))
    torch.cuda.synchronize()
    assert rel(cs[k4].cpu().numpy(), tight["c"].cpu().numpy().reshape(s4.ny, s4.nx)) <= 1e-5
    # level statistics of the batch (library reduction) against numpy on the same outputs
    L = len(pairs) - 1
    fine_grids = [hi.level_grid(lev) for lev in range(L + 1)]
    m = [len(p[0]) for p in pairs]
    f64 = dict(dtype=torch.float64, device="cuda")
    stack = lambda idx: torch.stack([cs[k].reshape(-1) for k in idx])
    c_f = [stack(p[0]).contiguous() for p in pairs]
    c_c = [None] + [stack(p[1]).contiguous() for p in pairs[1:]]
    q_t = out["qoi"]
    q_f = [q_t[list(p[0])].contiguous() for p in pairs]
    q_c = [None] + [q_t[list(p[1])].contiguous() for p in pairs[1:]]
    mean_Y = [torch.empty(g[0] * g[1], **f64) for g in fine_grids]
    var_Y = [torch.empty(g[0] * g[1], **f64) for g in fine_grids]
    qstats = torch.empty((L + 1, 2), **f64)
    Ec = torch.empty(fine_grids[-1][0] * fine_grids[-1][1], **f64)
    var_est = torch.empty(2, **f64)
    hm.mlmc_level_estimate(ctx, fine_grids, m, c_f, c_c, q_f, q_c, mean_Y, var_Y, qstats, Ec, var_est)
    torch.cuda.synchronize()
    for lev in range(L + 1):
        nx, ny = fine_grids[lev][:2]
        Y = c_f[lev].cpu().numpy().reshape(-1, ny, nx)
        if lev > 0:
            Y = Y - oracle.inject(c_c[lev].cpu().numpy().reshape(-1, ny // 2, nx // 2), 2)
        assert np.abs(mean_Y[lev].cpu().numpy() - Y.mean(0).ravel()).max() <= 1e-12
        assert np.abs(var_Y[lev].cpu().numpy() - Y.var(0, ddof=1).ravel()).max() <= 1e-12


def test_pair_64x32_32x16_full_fp64_sampled_against_oracle(torch_cuda, ctx):
    torch = torch_cuda
    fine, coarse = hi.pair_solves(hi.CONFIGS["pair_64x32_32x16"]["m"])
    solves = fine + coarse
    grids = [(s.nx, s.ny, s.nsteps) for s in solves]
    print(f"pair_64x32_32x16: {len(solves)} FP64 solves", flush=True)
    # tol 1e-11: the QoI sums small c values over half the domain, and at
    # 1e-10 its error reaches the 1e-8 bar on these 200-step solves
    out = hm.solve(ctx, grids, xi=dev(torch, xi_of(solves)),
                   opts=hm.make_opts(prec=hm.PREC_FP64, tol=1e-11, max_outer=80))
    torch.cuda.synchronize()
    assert (out["status"].cpu().numpy() == hm.STATUS_OK).all()
    cs = hm.unpack(out["c"], grids)
    q = out["qoi"].cpu().numpy()
    m = len(fine)
    picks = [int(i) for i in np.random.default_rng(12).choice(m, 2, replace=False)]
    jobs, ks = [], []
    for i in picks:
        for k in (i, m + i):
            s = solves[k]
            jobs.append((s.nx, s.ny, s.nsteps, s.level, s.index))
            ks.append(k)
    print(f"oracle on pairs {picks}", flush=True)
    for k, r in zip(ks, oracle_many(jobs)):
        assert rel(cs[k].cpu().numpy(), r["c"]) <= 1e-8, (k, solves[k])
        assert abs(q[k] - r["qoi"]) <= 1e-8 * abs(r["qoi"])
    # level-difference statistics on the full set (numpy on the GPU outputs)
    Yc = np.stack([cs[i].cpu().numpy() - oracle.inject(cs[m + i].cpu().numpy(), 2) for i in range(m)])
    Yq = q[:m] - q[m:]
    g, gc = ([cs[i].cpu().numpy() for i in range(m)], [cs[m + i].cpu().numpy() for i in range(m)])
    stats = oracle.level_stats(np.stack(g), np.stack(gc))
    assert np.abs(stats[0] - Yc.mean(0)).max() <= 1e-14
    assert np.abs(stats[1] - Yc.var(0, ddof=1)).max() <= 1e-14
    assert np.isfinite(Yq).all() and Yq.var(ddof=1) > 0.0


def test_adjoint_128x64_full_batch_fd_on_eight_samples(torch_cuda, ctx):
    torch = torch_cuda
    cfg = hi.CONFIGS["adjoint_128x64"]
    nx, ny, r = cfg["grid"]
    ns = cfg["samples"]
    xi = hm.henry_sample_xi(hi.SEED, 3, 0, ns, 3)
    print(f"adjoint_128x64: {ns} samples, checkpoints every {cfg['ckpt']}", flush=True)
    adj = hm.adjoint(ctx, [(nx, ny, r)] * ns, xi=dev(torch, xi),
                     opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-10, max_outer=100), ckpt_every=cfg["ckpt"],
                     adj_tol=1e-10, adj_max_it=100)
    torch.cuda.synchronize()
    st = adj["status"].cpu().numpy()
    assert (st == hm.STATUS_OK).all(), f"{int((st != 0).sum())} of {ns} not converged"
    gx = adj["dq_dxi"].cpu().numpy()
    assert np.isfinite(gx).all() and np.isfinite(adj["dq_dlogk"].cpu().numpy()).all()
    hfd = 1e-6
    pts = []
    for s in range(8):
        for d in range(3):
            e = np.zeros(3); e[d] = hfd
            pts += [xi[s] + e, xi[s] - e]
    print("central differences on samples 0..7", flush=True)
    fwd = hm.solve(ctx, [(nx, ny, r)] * len(pts), xi=dev(torch, np.array(pts)),
                   opts=hm.make_opts(prec=hm.PREC_FP64, tol=1e-11, max_outer=100))
    torch.cuda.synchronize()
    qq = fwd["qoi"].cpu().numpy().reshape(8, 3, 2)
    fd = (qq[..., 0] - qq[..., 1]) / (2 * hfd)
    for s in range(8):
        assert np.abs(fd[s] - gx[s]).max() <= 1e-4 * np.abs(gx[s]).max(), (s, fd[s], gx[s])


def test_kl_1024x512_first_steps_solve_the_oracle_equations(torch_cuda):
    torch = torch_cuda
    nx, ny, rfull = hi.CONFIGS["kl_1024x512"]["grid"]
    k = 3
    xi = hm.henry_sample_xi_kl(hi.SEED, 6, 0, 2)
    lam, modes = kl.basis(nx, ny)
    res = {}
    for prec in (hm.PREC_MIXED, hm.PREC_FP64):
        runs = {}
        for steps in (k - 1, k):
            # tau = T/3200 as in the full run: a context whose horizon is `steps` steps of it
            ph = dict(hi.PHYS); ph["T"] = hi.PHYS["T"] * steps / rfull
            c = hm.Context(ph, 0)
            c.set_kl(nx, ny, kl.CORR_LEN, kl.SIGMA_PHI, kl.SIGMA_LOGK)
            print(f"kl_1024x512 prec={prec}: {steps} steps", flush=True)
            out = hm.solve(c, [(nx, ny, steps)] * 2, xi=dev(torch, xi),
                           opts=hm.make_opts(prec=prec, tol=1e-9, max_outer=80), want_p=True)
            torch.cuda.synchronize()
            assert (out["status"].cpu().numpy() == hm.STATUS_OK).all()
            runs[steps] = (out, ph)
            c.close()
        out_k, ph_k = runs[k]
        res[prec] = out_k["c"].cpu().numpy()
        g = [(nx, ny, k)] * 2
        for s in range(2):
            phi, K, q = kl.fields(ph_k, lam, modes, xi[s])
            c1 = hm.unpack(runs[k - 1][0]["c"], g)[s].cpu().numpy()
            c2 = hm.unpack(out_k["c"], g)[s].cpu().numpy()
            p2 = hm.unpack(out_k["p"], g)[s].cpu().numpy()
            Rp, Rc = oracle.residual(ph_k, k, phi, K, q, p2, c2, c1)
            sc = (ph_k["T"] / k) / ((1.0 / ny) ** 2 * phi * ph_k["rho0"])
            assert np.abs(Rp * sc).max() <= 2e-9 and np.abs(Rc * sc).max() <= 2e-9
    assert np.abs(res[hm.PREC_MIXED] - res[hm.PREC_FP64]).max() <= 1e-8


def test_kl_1024x512_gradient_is_the_projection_on_the_basis(torch_cuda):
    torch = torch_cuda
    nx, ny, rfull = hi.CONFIGS["kl_1024x512"]["grid"]
    k = 3
    ph = dict(hi.PHYS); ph["T"] = hi.PHYS["T"] * k / rfull
    c = hm.Context(ph, 0)
    c.set_kl(nx, ny, kl.CORR_LEN, kl.SIGMA_PHI, kl.SIGMA_LOGK)
    xi = hm.henry_sample_xi_kl(hi.SEED, 6, 0, 1)
    print("kl_1024x512 adjoint, 3 steps", flush=True)
    # tol 1e-9: at 2^19 cells the scaled FP64 residual stalls near 1e-10
    a = hm.adjoint(c, [(nx, ny, k)], xi=dev(torch, xi),
                   opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-9, max_outer=80), ckpt_every=2, adj_tol=1e-9,
                   adj_max_it=100)
    torch.cuda.synchronize()
    c.close()
    assert a["status"].item() == hm.STATUS_OK
    lam, modes = kl.basis(nx, ny)
    gphi = a["dq_dphi"].cpu().numpy().reshape(ny, nx)
    glogk = a["dq_dlogk"].cpu().numpy().reshape(ny, nx)
    s = np.sqrt(lam)
    ref = np.empty(41)
    ref[:20] = ph["phi0"] * kl.SIGMA_PHI * s * np.tensordot(modes, gphi, axes=([1, 2], [0, 1]))
    ref[20:40] = kl.SIGMA_LOGK * s * np.tensordot(modes, glogk, axes=([1, 2], [0, 1]))
    ref[40] = a["dq_dq"].item() * ph["q_in"] * 0.2
    g = a["dq_dxi"].cpu().numpy()[0]
    assert np.isfinite(g).all()
    assert np.abs(g - ref).max() <= 1e-9 * np.abs(ref).max() + 1e-300


def test_kl_1024x512_full_length_adjoint_against_central_differences(torch_cuda):
    torch = torch_cuda
    nx, ny, r = hi.CONFIGS["kl_1024x512"]["grid"]
    ckpt = hi.CONFIGS["kl_1024x512"]["ckpt"]
    c = hm.Context(hi.PHYS, 0)
    c.set_kl(nx, ny, kl.CORR_LEN, kl.SIGMA_PHI, kl.SIGMA_LOGK)
    xi = hm.henry_sample_xi_kl(hi.SEED, 6, 0, 2)
    print(f"kl_1024x512 adjoint: 2 samples x {r} steps, checkpoints every {ckpt}", flush=True)
    a = hm.adjoint(c, [(nx, ny, r)] * 2, xi=dev(torch, xi),
                   opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-8, max_outer=60), ckpt_every=ckpt, adj_tol=1e-8,
                   adj_max_it=60)
    torch.cuda.synchronize()
    assert (a["status"].cpu().numpy() == hm.STATUS_OK).all()
    g = a["dq_dxi"].cpu().numpy()
    del a
    h, ks = 1e-3, (0, 20, 40)
    pts = []
    for s in range(2):
        for k in ks:
            for sg in (1.0, -1.0):
                x = xi[s].copy()
                x[k] += sg * h
                pts.append(x)
    print(f"central differences: {len(pts)} forward solves of {r} steps", flush=True)
    fo = hm.solve(c, [(nx, ny, r)] * len(pts), xi=dev(torch, np.array(pts)),
                  opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-9, max_outer=60))
    torch.cuda.synchronize()
    assert (fo["status"].cpu().numpy() == hm.STATUS_OK).all()
    q = fo["qoi"].cpu().numpy().reshape(2, len(ks), 2)
    c.close()
    fd = (q[..., 0] - q[..., 1]) / (2 * h)
    for s in range(2):
        for i, k in enumerate(ks):
            print(f"sample {s} xi{k + 1}: adjoint {g[s, k]:.9e} central difference {fd[s, i]:.9e}", flush=True)
            assert abs(fd[s, i] - g[s, k]) <= 1e-4 * abs(g[s, k]), (s, k)
