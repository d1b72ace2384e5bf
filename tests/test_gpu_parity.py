"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (element by element on the same seeded inputs):
  * FP64 inner path: max |c_gpu - c_oracle| <= 1e-8 * max |c_oracle|, and
    the QoI within 1e-8 relative;
  * mixed path (FP32 V-cycles inside FP64 defect correction): 1e-5.
Both paths stop a step when the scaled FP64 residual max norms fall below
tol = 1e-10; the prototype study of this iteration gave c errors of about
1e-11 at that tolerance, so the bars leave three orders of headroom.
"""
import numpy as np
import pytest

import henry_inputs as hi
import oracle
import paper_2302_07804_amd as hm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible for a gpu-marked test")
    hm.lib()  # raises if the native library is missing
    return torch


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    c = hm.Context(hi.PHYS, 0)
    yield c
    c.close()


def run(torch, ctx, solves, xi=None, prec=hm.PREC_FP64, **kw):
    opts = hm.make_opts(prec=prec, tol=kw.pop("tol", 1e-10), max_outer=kw.pop("max_outer", 60), **kw)
    xi_d = None if xi is None else torch.tensor(np.asarray(xi), dtype=torch.float64, device="cuda")
    out = hm.solve(ctx, solves, xi=xi_d, opts=opts, want_p=True)
    torch.cuda.synchronize()
    return out


def oracle_jobs(solves, xis):
    return oracle.solve_many(hi.PHYS, [(s[0], s[1], s[2], x) for s, x in zip(solves, xis)])


def check_against(out, solves, refs, bar):
    cs = hm.unpack(out["c"], solves)
    q = out["qoi"].cpu().numpy()
    st = out["status"].cpu().numpy()
    worst = 0.0
    for k, (s, r) in enumerate(zip(solves, refs)):
        assert st[k] == hm.STATUS_OK, f"solve {k} {s}: status {st[k]}"
        c = cs[k].cpu().numpy()
        err = np.abs(c - r["c"]).max() / np.abs(r["c"]).max()
        qerr = abs(q[k] - r["qoi"]) / abs(r["qoi"])
        worst = max(worst, err, qerr)
        assert err <= bar, f"solve {k} {s}: c rel err {err:.3e}"
        assert qerr <= bar, f"solve {k} {s}: Q rel err {qerr:.3e}"
    return worst


@pytest.mark.parametrize("prec,bar", [(hm.PREC_FP64, 1e-8), (hm.PREC_MIXED, 1e-5)])
def test_single_level0_solve(torch_cuda, ctx, prec, bar):
    solves = [(16, 8, 50)]
    xi = hm.henry_sample_xi(0, 0, 0, 1, 3)
    out = run(torch_cuda, ctx, solves, xi, prec)
    refs = oracle_jobs(solves, xi)
    worst = check_against(out, solves, refs, bar)
    print(f"16x8/50 prec={prec}: worst rel err {worst:.3e}, iterations {out['iters'].cpu().numpy()}")


@pytest.mark.parametrize("prec,bar", [(hm.PREC_FP64, 1e-8), (hm.PREC_MIXED, 1e-5)])
def test_degenerate_grids_and_single_steps(torch_cuda, ctx, prec, bar):
    """The smallest hierarchies (2x1: one level; 4x2, 8x4), single-step and
    two-step solves (no extrapolation, linear only) with time steps up to
    the whole horizon T, against the oracle.  (A single step of T on 32x16
    or finer is beyond the block iteration: it reports NOCONV.)"""
    solves = [(2, 1, 3), (4, 2, 5), (8, 4, 1), (16, 8, 1), (16, 8, 2), (32, 16, 2), (2, 1, 1)]
    xi = hm.henry_sample_xi(0, 5, 0, len(solves), 3)
    out = run(torch_cuda, ctx, solves, xi, prec, max_outer=400)
    refs = oracle_jobs(solves, xi)
    worst = check_against(out, solves, refs, bar)
    print(f"degenerate grids prec={prec}: worst rel err {worst:.3e}")


@pytest.mark.parametrize("prec,bar", [(hm.PREC_FP64, 1e-8), (hm.PREC_MIXED, 1e-5)])
def test_ragged_batch_several_grids(torch_cuda, ctx, prec, bar):
    """Solves of three grids and step counts share one call (several tiles
    per line at 64x32, odd sample counts per grid)."""
    solves = [(16, 8, 50)] * 3 + [(32, 16, 100)] * 2 + [(64, 32, 200)]
    xi = hm.henry_sample_xi(0, 1, 0, len(solves), 3)
    out = run(torch_cuda, ctx, solves, xi, prec)
    refs = oracle_jobs(solves, xi)
    worst = check_against(out, solves, refs, bar)
    print(f"ragged prec={prec}: worst rel err {worst:.3e}, iterations {out['iters'].cpu().numpy()}")


def test_mixed_and_fp64_agree_closely(torch_cuda, ctx):
    solves = [(32, 16, 100)] * 4
    xi = hm.henry_sample_xi(0, 2, 0, 4, 3)
    a = run(torch_cuda, ctx, solves, xi, hm.PREC_FP64)
    b = run(torch_cuda, ctx, solves, xi, hm.PREC_MIXED)
    assert (a["c"] - b["c"]).abs().max().item() < 1e-8


def test_explicit_fields_match_oracle(torch_cuda, ctx):
    """Caller-provided per-cell porosity and log-permeability."""
    torch = torch_cuda
    nx, ny, r = 32, 16, 60
    rng = np.random.default_rng(3)
    x = (np.arange(nx) + 0.5) / ny
    y = -1 + (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    phi = 0.35 * (1 + 0.15 * np.sin(2 * X + rng.uniform()) * np.cos(3 * Y))
    logk = np.log(hi.PHYS["k0"]) + 0.4 * np.cos(X + 2 * Y + rng.uniform())
    q = hi.PHYS["q_in"] * 1.1
    dev = lambda a: torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64, device="cuda")
    opts = hm.make_opts(prec=hm.PREC_FP64, tol=1e-10, max_outer=60)
    out = hm.solve(ctx, [(nx, ny, r)], phi=dev(phi), logk=dev(logk), qin=dev([q]), opts=opts)
    torch.cuda.synchronize()
    ref = oracle.solve(hi.PHYS, r, phi, np.exp(logk), q)
    c = out["c"].cpu().numpy().reshape(ny, nx)
    assert np.abs(c - ref["c"]).max() <= 1e-8 * np.abs(ref["c"]).max()
    assert abs(out["qoi"].item() - ref["qoi"]) <= 1e-8 * ref["qoi"]


def test_chunked_launches_match_single_launch(torch_cuda, ctx):
    solves = [(16, 8, 50)] * 2 + [(32, 16, 100)]
    xi = hm.henry_sample_xi(0, 1, 0, 3, 3)
    a = run(torch_cuda, ctx, solves, xi, hm.PREC_MIXED)
    b = run(torch_cuda, ctx, solves, xi, hm.PREC_MIXED, steps_per_launch=7)
    assert torch_cuda.equal(a["c"], b["c"]) and torch_cuda.equal(a["qoi"], b["qoi"])


@pytest.mark.parametrize("prec", [hm.PREC_FP64, hm.PREC_MIXED])
def test_batched_equals_one_solve_per_call(torch_cuda, ctx, prec):
    """The plain path (one solve per call) and the batched path run the same
    per-solve computation: bitwise equal fields and QoI, whatever the batch
    mixes in (other grids, other step counts, other workgroup sizes)."""
    solves = [(16, 8, 50), (64, 32, 200), (32, 16, 100), (16, 8, 50), (128, 64, 40)]
    xi = hm.henry_sample_xi(0, 6, 0, len(solves), 3)
    batch = run(torch_cuda, ctx, solves, xi, prec)
    cs = hm.unpack(batch["c"], solves)
    for k, s in enumerate(solves):
        one = run(torch_cuda, ctx, [s], xi[k:k + 1], prec)
        assert torch_cuda.equal(one["c"].view(s[1], s[0]), cs[k]), (k, s)
        assert one["qoi"][0].item() == batch["qoi"][k].item(), (k, s)


@pytest.mark.parametrize("prec,predictor", [(hm.PREC_MIXED, 0), (hm.PREC_FP64, 0), (hm.PREC_MIXED, 2)])
def test_cluster_sizes_are_bitwise_equal(torch_cuda, ctx, prec, predictor):
    """A solve shared by 2, 4 or 8 workgroups (fine levels split over the
    cluster, coarse levels on its leader) computes every cell and line with
    the same arithmetic as one workgroup: c, p, Q, status and iteration
    counts are bitwise equal, in one launch and in chunked graph launches
    (whose launches carry the five-state history of the least-squares
    start across chunks)."""
    torch = torch_cuda
    solves = [(128, 64, 40), (256, 128, 160), (128, 64, 40), (16, 8, 50)]
    xi = hm.henry_sample_xi(0, 7, 0, len(solves), 3)
    ref = run(torch, ctx, solves, xi, prec, tol=1e-9, cluster=1, predictor=predictor)
    assert list(ref["status"].cpu().numpy()) == [hm.STATUS_OK] * len(solves)
    for K, spl in ((2, 0), (4, 0), (8, 0), (4, 5)):
        out = run(torch, ctx, solves, xi, prec, tol=1e-9, cluster=K, steps_per_launch=spl, predictor=predictor)
        for key in ("c", "p", "qoi", "status", "iters"):
            assert torch.equal(out[key], ref[key]), (K, spl, key)


@pytest.mark.parametrize("prec", [hm.PREC_MIXED, hm.PREC_FP64])
def test_staged_line_solves_equal_the_register_path(torch_cuda, prec):
    """x-lines of 512 and 1024 cells on the cluster levels are formed from
    coalesced loads and staged through LDS; with one workgroup per solve the
    same lines are solved from the lanes' own loads.  The clusters also run
    the 512-thread build, whose residual passes form the face coefficients
    of these grids from K and phi and whose level transfers gather four
    cells per thread, where the one-workgroup solves (1024-thread build)
    load the stored coefficients and move one cell at a time.  Both do the
    same arithmetic: c, p, Q, status and iteration counts are bitwise equal
    (512x256 and 1024x512, the first steps at the 1024x512 workload's time
    step, clusters of 2 and 8)."""
    torch = torch_cuda
    ph = dict(hi.PHYS)
    ph["T"] = hi.PHYS["T"] * 4 / 3200
    c = hm.Context(ph, 0)
    solves = [(512, 256, 2), (1024, 512, 4)]
    xi = hm.henry_sample_xi(0, 8, 0, len(solves), 3)
    print(f"staged line solves, prec {prec}", flush=True)
    ref = run(torch, c, solves, xi, prec, tol=1e-9, cluster=1)
    assert list(ref["status"].cpu().numpy()) == [hm.STATUS_OK] * len(solves)
    for K in (2, 8):
        out = run(torch, c, solves, xi, prec, tol=1e-9, cluster=K)
        for key in ("c", "p", "qoi", "status", "iters"):
            assert torch.equal(out[key], ref[key]), (K, key)
    c.close()


def test_two_cluster_groups_in_one_batch(torch_cuda, ctx):
    """Two grid groups shared by clusters (512x256 on 8 workgroups, 256x128
    on 4) and a group of one workgroup per solve in one call: the cluster
    groups run one after the other, and every solve equals its
    one-workgroup result bitwise."""
    torch = torch_cuda
    solves = [(512, 256, 100), (256, 128, 160), (256, 128, 160), (16, 8, 50)]
    xi = hm.henry_sample_xi(0, 11, 0, len(solves), 3)
    ref = run(torch, ctx, solves, xi, hm.PREC_MIXED, tol=1e-7, cluster=1)
    out = run(torch, ctx, solves, xi, hm.PREC_MIXED, tol=1e-7, profile=1)
    groups = {(g["nx"], g["cluster"]) for g in hm.henry_profile_last(ctx)}
    assert {(512, 8), (256, 4), (16, 1)} <= groups, groups
    assert list(out["status"].cpu().numpy()) == [hm.STATUS_OK] * len(solves)
    for key in ("c", "p", "qoi", "status", "iters"):
        assert torch.equal(out[key], ref[key]), key


def test_cluster_wait_bound_reports_sync_status(torch_cuda, ctx):
    """A cluster whose members wait longer than opts.cluster_wait_us at a
    barrier stops (every later barrier returns at once) and reports
    HENRY_STATUS_SYNC; here the bound (1 us) is below the time the members
    spend waiting for the leader's coarse levels.  The next call starts from
    a fresh cluster state and converges."""
    torch = torch_cuda
    solves = [(256, 128, 160), (16, 8, 50)]
    xi = hm.henry_sample_xi(0, 10, 0, len(solves), 3)
    bad = run(torch, ctx, solves, xi, hm.PREC_MIXED, tol=1e-9, cluster=4, cluster_wait_us=1)
    assert list(bad["status"].cpu().numpy()) == [hm.STATUS_SYNC, hm.STATUS_OK]
    good = run(torch, ctx, solves, xi, hm.PREC_MIXED, tol=1e-9, cluster=4)
    assert list(good["status"].cpu().numpy()) == [hm.STATUS_OK] * 2


def test_cluster_solve_matches_oracle(torch_cuda, ctx):
    solves = [(128, 64, 40)]
    xi = hm.henry_sample_xi(0, 8, 0, 1, 3)
    out = run(torch_cuda, ctx, solves, xi, hm.PREC_MIXED, cluster=4)
    refs = oracle_jobs(solves, xi)
    worst = check_against(out, solves, refs, 1e-5)
    print(f"128x64/40 on a 4-workgroup cluster: worst rel err {worst:.3e}")


def test_repeat_is_bitwise_deterministic(torch_cuda, ctx):
    solves = [(32, 16, 100)] * 3
    xi = hm.henry_sample_xi(0, 5, 0, 3, 3)
    a = run(torch_cuda, ctx, solves, xi, hm.PREC_MIXED)
    b = run(torch_cuda, ctx, solves, xi, hm.PREC_MIXED)
    assert torch_cuda.equal(a["c"], b["c"]) and torch_cuda.equal(a["qoi"], b["qoi"])


def test_no_convergence_is_reported_per_solve(torch_cuda, ctx):
    solves = [(16, 8, 50)] * 2
    xi = hm.henry_sample_xi(0, 0, 0, 2, 3)
    out = run(torch_cuda, ctx, solves, xi, hm.PREC_MIXED, max_outer=1)
    assert list(out["status"].cpu().numpy()) == [hm.STATUS_NOCONV] * 2


def test_nonfinite_input_is_reported_for_its_solve_only(torch_cuda, ctx):
    """A NaN coefficient in one solve's xi makes its fields and residual
    non-finite: that solve reports HENRY_STATUS_NONFINITE and stops, while
    the other solves of the batch are bitwise those of a batch without it."""
    torch = torch_cuda
    solves = [(16, 8, 50)] * 3 + [(128, 64, 40)]
    xi = hm.henry_sample_xi(0, 15, 0, len(solves), 3)
    bad = xi.copy()
    bad[1, 0] = np.nan
    out = run(torch, ctx, solves, bad, hm.PREC_MIXED, tol=1e-9)
    ref = run(torch, ctx, [solves[k] for k in (0, 2, 3)], xi[[0, 2, 3]], hm.PREC_MIXED, tol=1e-9)
    assert list(out["status"].cpu().numpy()) == [hm.STATUS_OK, hm.STATUS_NONFINITE, hm.STATUS_OK, hm.STATUS_OK]
    cs, rs = hm.unpack(out["c"], solves), hm.unpack(ref["c"], [solves[k] for k in (0, 2, 3)])
    for a, b in zip((cs[0], cs[2], cs[3]), rs):
        assert torch.equal(a, b)
    q = out["qoi"].cpu().numpy()
    assert np.array_equal(q[[0, 2, 3]], ref["qoi"].cpu().numpy())


def test_huge_recharge_reports_nonfinite(torch_cuda, ctx):
    """Explicit fields with a recharge of 1e300 m/s overflow the fluxes."""
    torch = torch_cuda
    nx, ny, r = 16, 8, 20
    dev = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.float64).ravel(), device="cuda")
    phi = np.full((ny, nx), hi.PHYS["phi0"])
    logk = np.full((ny, nx), np.log(hi.PHYS["k0"]))
    out = hm.solve(ctx, [(nx, ny, r)] * 2, phi=dev(np.stack([phi, phi])), logk=dev(np.stack([logk, logk])),
                   qin=dev([1e300, hi.PHYS["q_in"]]), opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-9))
    torch.cuda.synchronize()
    assert list(out["status"].cpu().numpy()) == [hm.STATUS_NONFINITE, hm.STATUS_OK]


def test_small_workspace_is_rejected(torch_cuda, ctx):
    torch = torch_cuda
    solves = [(16, 8, 50)] * 2
    opts = hm.make_opts(prec=hm.PREC_MIXED)
    need = hm.henry_workspace_bytes(solves, opts)
    raw = torch.empty(need // 8 + 64, dtype=torch.float64, device="cuda")
    off = (-raw.data_ptr()) % 256 // 8
    ws = raw[off:off + need // 8 - 32]  # 256 bytes short
    xi = torch.tensor(hm.henry_sample_xi(0, 0, 0, 2, 3), dtype=torch.float64, device="cuda")
    c = torch.empty(2 * 128, dtype=torch.float64, device="cuda")
    q = torch.empty(2, dtype=torch.float64, device="cuda")
    st = torch.empty(2, dtype=torch.int32, device="cuda")
    with pytest.raises(hm.HenryError) as e:
        hm.henry_solve_batch(ctx, solves, hm.FIELD_CLOSED3, xi=xi, opts=opts, c_out=c, qoi_out=q, status=st,
                             workspace=ws)
    assert e.value.code == hm.HENRY_ENOMEM


def test_hydrostatic_seawater_on_gpu(torch_cuda):
    """c0 = 1, no recharge, no diffusion: p = -rho1 g y, zero Darcy flux."""
    torch = torch_cuda
    ph = dict(hi.PHYS, D=0.0, q_in=0.0)
    c = hm.Context(ph, 0)
    nx, ny, r = 32, 16, 10
    rng = np.random.default_rng(1)
    phi = 0.35 * (1 + 0.2 * rng.uniform(-1, 1, (ny, nx)))
    logk = np.log(ph["k0"]) + 0.5 * rng.uniform(-1, 1, (ny, nx))
    dev = lambda a: torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64, device="cuda")
    out = hm.solve(c, [(nx, ny, r)], phi=dev(phi), logk=dev(logk), qin=dev([0.0]), c0=dev(np.ones((ny, nx))),
                   opts=hm.make_opts(prec=hm.PREC_FP64, tol=1e-12, max_outer=60), want_p=True)
    torch.cuda.synchronize()
    y = -1 + (np.arange(ny) + 0.5) / ny
    p_exact = np.repeat((-ph["rho1"] * ph["g"] * y)[:, None], nx, 1)
    assert np.abs(out["c"].cpu().numpy() - 1.0).max() <= 1e-14
    np.testing.assert_allclose(out["p"].cpu().numpy().reshape(ny, nx), p_exact, rtol=1e-12)
    c.close()


def test_empty_batch_is_a_no_op(torch_cuda, ctx):
    L = hm.lib()
    assert L.henry_solve_batch(ctx.handle, None, 0, 0, None, None, None, None, None, None, None, None, None, None,
                               None, None, 0, None) == hm.HENRY_OK


def test_workspace_too_small_is_enomem(torch_cuda, ctx):
    torch = torch_cuda
    solves = [(16, 8, 50)]
    ws = torch.empty(1024, dtype=torch.float64, device="cuda")
    xi = torch.zeros(3, dtype=torch.float64, device="cuda")
    o = torch.empty(128, dtype=torch.float64, device="cuda")
    q = torch.empty(1, dtype=torch.float64, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    with pytest.raises(hm.HenryError) as e:
        hm.henry_solve_batch(ctx, solves, hm.FIELD_CLOSED3, xi=xi, c_out=o, qoi_out=q, status=st, workspace=ws)
    assert e.value.code == hm.HENRY_ENOMEM


def test_mlmc_level_estimate_matches_oracle_stats(torch_cuda, ctx):
    torch = torch_cuda
    rng = np.random.default_rng(11)
    m = [37, 9, 5]
    grids = [(16, 8, 50), (32, 16, 100), (64, 32, 200)]
    cf = [rng.uniform(size=(m[l], grids[l][1], grids[l][0])) for l in range(3)]
    cc = [None] + [rng.uniform(size=(m[l], grids[l - 1][1], grids[l - 1][0])) for l in range(1, 3)]
    qf = [rng.uniform(size=m[l]) for l in range(3)]
    qc = [None] + [rng.uniform(size=m[l]) for l in range(1, 3)]
    dev = lambda a: None if a is None else torch.tensor(a.reshape(a.shape[0], -1), dtype=torch.float64,
                                                        device="cuda")
    mean = [torch.empty(g[0] * g[1], dtype=torch.float64, device="cuda") for g in grids]
    var = [torch.empty(g[0] * g[1], dtype=torch.float64, device="cuda") for g in grids]
    qs = torch.empty(6, dtype=torch.float64, device="cuda")
    E = torch.empty(64 * 32, dtype=torch.float64, device="cuda")
    ve = torch.empty(2, dtype=torch.float64, device="cuda")
    qdev = lambda a: None if a is None else torch.tensor(a, dtype=torch.float64, device="cuda")
    hm.mlmc_level_estimate(ctx, grids, m, [dev(x) for x in cf], [dev(x) for x in cc], [qdev(x) for x in qf],
                           [qdev(x) for x in qc], mean, var, qs, E, ve)
    torch.cuda.synchronize()
    means, vars_, qm, qv = [], [], [], []
    for l in range(3):
        mu, v = oracle.level_stats(cf[l], cc[l])
        np.testing.assert_allclose(mean[l].cpu().numpy().reshape(mu.shape), mu, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(var[l].cpu().numpy().reshape(v.shape), v, rtol=1e-12, atol=1e-15)
        a, b = oracle.level_stats(qf[l], qc[l])
        assert qs[2 * l].item() == pytest.approx(float(a), rel=1e-13)
        assert qs[2 * l + 1].item() == pytest.approx(float(b), rel=1e-12)
        means.append(mu); vars_.append(v); qm.append(a); qv.append(b)
    Eo, vo = oracle.mlmc_estimate(means, vars_, m)
    np.testing.assert_allclose(E.cpu().numpy().reshape(Eo.shape), Eo, rtol=1e-13, atol=1e-15)
    _, vq = oracle.mlmc_estimate(qm, qv, m)
    assert ve[0].item() == pytest.approx(float(vq), rel=1e-13)
    assert ve[1].item() == pytest.approx(float(vo.max()), rel=1e-13)


@pytest.mark.parametrize("solves,cluster", [([(16, 8, 50)] * 3 + [(32, 16, 100)] * 2, 0),
                                            ([(128, 64, 40)] * 2 + [(16, 8, 50)], 2)])
def test_graph_replays_match_eager(torch_cuda, ctx, solves, cluster):
    """steps_per_launch > 0 captures the lockstep time loop once into a
    hipGraph; replays on the same buffers, with eager work in between, must
    all give the eager result (with clusters too: each replay starts from a
    fresh cluster state, reset by the captured fields kernel)."""
    torch = torch_cuda
    xi = torch.tensor(hm.henry_sample_xi(0, 2, 0, len(solves), 3), dtype=torch.float64, device="cuda")
    eager = hm.solve(ctx, solves, xi=xi, opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-10, max_outer=60,
                                                           cluster=cluster))
    torch.cuda.synchronize()
    assert (eager["status"].cpu().numpy() == hm.STATUS_OK).all()
    gopts = hm.make_opts(prec=hm.PREC_MIXED, tol=1e-10, max_outer=60, steps_per_launch=5, cluster=cluster)
    cells = sum(s[0] * s[1] for s in solves)
    ws_b = hm.henry_workspace_bytes(solves, gopts)
    raw = torch.empty(ws_b // 8 + 64, dtype=torch.float64, device="cuda")
    off = (-raw.data_ptr()) % 256 // 8
    ws = raw[off:off + (ws_b + 7) // 8]
    c = torch.empty(cells, dtype=torch.float64, device="cuda")
    q = torch.empty(len(solves), dtype=torch.float64, device="cuda")
    st = torch.empty(len(solves), dtype=torch.int32, device="cuda")
    for rep in range(3):
        c.fill_(-1.0)
        q.fill_(-1.0)
        hm.henry_solve_batch(ctx, solves, hm.FIELD_CLOSED3, xi=xi, opts=gopts, c_out=c, qoi_out=q, status=st,
                             workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(c, eager["c"]), f"replay {rep}"
        assert torch.equal(q, eager["qoi"]), f"replay {rep}"
        _ = (torch.randn(1000, device="cuda") ** 2).sum().item()  # eager work between replays


def test_autotune_picks_a_candidate_and_threads_do_not_change_the_solution(torch_cuda, ctx):
    """The workgroup size changes no result: c is bitwise the same for every
    size (max-norm decisions are order independent), and so is Q, whose sum
    runs in an order fixed by the grid alone."""
    torch = torch_cuda
    solves = [(16, 8, 50)] * 6 + [(32, 16, 100)] * 3
    xi = torch.tensor(hm.henry_sample_xi(0, 1, 0, len(solves), 3), dtype=torch.float64, device="cuda")
    res = hm.autotune(ctx, solves, xi, hm.make_opts(prec=hm.PREC_MIXED, tol=1e-10, max_outer=60), tune_steps=4)
    for (nx, prec), (t, kc, st, times) in res.items():
        assert t in (64, 128, 256, 512, 1024) and hm.henry_tune_get(ctx, nx, prec) == (t, kc, st)
    outs = [hm.solve(ctx, solves, xi=xi, opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-10, max_outer=60,
                                                           threads=t)) for t in (64, 256, 1024)]
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert torch.equal(outs[0]["c"], o["c"])
        assert torch.equal(outs[0]["qoi"], o["qoi"])
    for nx in (16, 32):
        hm.henry_tune_set(ctx, nx, hm.PREC_MIXED, 0)


def test_autotuned_clusters_and_streams_come_from_the_candidates_and_change_no_result(torch_cuda, ctx):
    """The tuner's second stage picks the workgroups per solve of the grids
    above 2048 cells (1, 2, 4 or 8, at most 256 workgroups per group) and
    the stream plan of the one-workgroup groups by timing the shortened
    batch; the batch solved with the tuned plan equals, bitwise in c and
    Q, the same batch with one workgroup per solve and the built-in
    streams at the same workgroup sizes."""
    torch = torch_cuda
    solves = [(128, 64, 40)] * 4 + [(64, 32, 40)] * 6 + [(16, 8, 50)] * 24 + [(32, 16, 100)] * 3
    xi = torch.tensor(hm.henry_sample_xi(0, 2, 0, len(solves), 3), dtype=torch.float64, device="cuda")
    opts = hm.make_opts(prec=hm.PREC_MIXED, tol=1e-9, max_outer=60)
    res = hm.autotune(ctx, solves, xi, opts, tune_steps=4)
    print({k: v[:3] for k, v in res.items()}, flush=True)
    for (nx, prec), (t, kc, st, times) in res.items():
        assert t in (64, 128, 256, 512, 1024)
        assert hm.henry_tune_get(ctx, nx, prec) == (t, kc, st)
        if nx == 128:
            assert kc in (1, 2, 4, 8) and {f"cluster {k}" for k in (1, 2, 4, 8)} <= set(times)
        else:
            assert kc == 0
        assert st in (-1, 0, 1, 2, 3)
    tuned = hm.solve(ctx, solves, xi=xi, opts=opts)
    for (nx, prec), (t, kc, st, _) in res.items():
        hm.henry_tune_set(ctx, nx, prec, t, 1, -1)
    plain = hm.solve(ctx, solves, xi=xi, opts=opts)
    torch.cuda.synchronize()
    assert (tuned["status"].cpu().numpy() == 0).all()
    assert torch.equal(tuned["c"], plain["c"])
    assert torch.equal(tuned["qoi"], plain["qoi"])
    for nx in (16, 32, 64, 128):
        hm.henry_tune_set(ctx, nx, hm.PREC_MIXED, 0, 0, -1)


def test_predictors_converge_to_the_same_states(torch_cuda, ctx):
    """The start of each step's iteration (interpolating cubic, or the
    least-squares cubic through five states) changes the iteration count,
    not the converged states: at tol 1e-10 both agree with each other and
    with the oracle.  At the benchmark's tol 1e-7 on a fine grid with many
    steps, where the states' own errors dominate the extrapolation error,
    the least-squares start takes fewer iterations (at tol 1e-10 it does
    not, which is why the built-in choice depends on the step count)."""
    torch = torch_cuda
    solves = [(64, 32, 400)] * 2
    xi = hm.henry_sample_xi(0, 16, 0, 2, 3)
    a = run(torch, ctx, solves, xi, hm.PREC_FP64, tol=1e-10, predictor=1)
    b = run(torch, ctx, solves, xi, hm.PREC_FP64, tol=1e-10, predictor=2)
    assert list(a["status"].cpu().numpy()) == list(b["status"].cpu().numpy()) == [0, 0]
    assert (a["c"] - b["c"]).abs().max().item() <= 1e-9
    ref = oracle.solve_xi(hi.PHYS, 64, 32, 400, xi[0])
    for out in (a, b):
        c0 = out["c"][:64 * 32].cpu().numpy().reshape(32, 64)
        assert np.abs(c0 - ref["c"]).max() <= 1e-8
    solves = [(128, 64, 400)] * 4
    xi = hm.henry_sample_xi(0, 17, 0, 4, 3)
    a = run(torch, ctx, solves, xi, hm.PREC_MIXED, tol=1e-7, predictor=1)
    b = run(torch, ctx, solves, xi, hm.PREC_MIXED, tol=1e-7, predictor=2)
    assert (a["c"] - b["c"]).abs().max().item() <= 1e-6
    assert b["iters"].sum().item() < a["iters"].sum().item()


def test_resume_from_a_stored_state(torch_cuda):
    """Checkpoint / resume: a solve of N steps equals one of s steps (to
    s T / N) followed by N - s steps (over the rest of the horizon) started
    from the stored c field, to the tolerance's reach.  p needs no storing:
    given c and c^n, the fluid balance fixes it."""
    torch = torch_cuda
    nx, ny, N, s = 64, 32, 200, 70
    xi = hm.henry_sample_xi(0, 18, 0, 1, 3)
    xi_d = torch.tensor(xi, dtype=torch.float64, device="cuda")
    opts = hm.make_opts(prec=hm.PREC_FP64, tol=1e-11, max_outer=80)
    full_ctx = hm.Context(hi.PHYS, 0)
    full = hm.solve(full_ctx, [(nx, ny, N)], xi=xi_d, opts=opts)
    tau = hi.PHYS["T"] / N
    first_ctx = hm.Context(dict(hi.PHYS, T=s * tau), 0)
    first = hm.solve(first_ctx, [(nx, ny, s)], xi=xi_d, opts=opts)
    rest_ctx = hm.Context(dict(hi.PHYS, T=(N - s) * tau), 0)
    rest = hm.solve(rest_ctx, [(nx, ny, N - s)], xi=xi_d, c0=first["c"], opts=opts)
    torch.cuda.synchronize()
    for c in (full_ctx, first_ctx, rest_ctx):
        c.close()
    assert full["status"].item() == first["status"].item() == rest["status"].item() == hm.STATUS_OK
    assert (full["c"] - rest["c"]).abs().max().item() <= 1e-9
    assert abs(full["qoi"].item() - rest["qoi"].item()) <= 1e-9 * abs(full["qoi"].item())
