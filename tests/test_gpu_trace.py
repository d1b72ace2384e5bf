"""Time series of the solves and their statistics on the GPU (Sec. 4:
eq:integral_fw, the points of eq:12points, the quantiles of Figs. 4 and 6,
the first-passage times of Figs. 5 and 7), against the oracle:
  * henry_solve_batch_trace against oracle.trace, record by record: c at the
    points to 1e-8 (FP64 path) / 1e-5 (mixed), the fresh-water area exactly
    up to the cells whose c lies within the solve's error of the threshold
    (a floating-point decision of an integer count);
  * recording leaves the solve unchanged, and the records are bitwise the
    same in one launch, in graph-replayed chunks and for clusters of 1, 2
    and 4 workgroups;
  * a solve stopped by a NaN has NaN records, the others are unchanged;
  * henry_sample_stats against numpy's mean and variance and the oracle's
    type-7 quantiles, ragged sample counts up to the 8192 limit, ties and
    NaN; henry_first_passage against oracle.first_passage and a count."""
import numpy as np
import pytest

import henry_inputs as hi
import oracle
import paper_2302_07804_amd as hm

pytestmark = pytest.mark.gpu

PTS12 = [(1.10, -0.95), (1.35, -0.95), (1.60, -0.95), (1.85, -0.95), (1.10, -0.75), (1.35, -0.75),
         (1.60, -0.75), (1.85, -0.75), (1.10, -0.50), (1.35, -0.50), (1.60, -0.50), (1.85, -0.50)]
PTS = PTS12 + [(0.0, -1.0), (2.0, 0.0), (1.0, -0.5)]
PROBS = [0.0, 0.025, 0.25, 0.5, 0.75, 0.975, 1.0]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible for a gpu-marked test")
    hm.lib()
    return torch


def dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def check_trace(tr, ref, c_final, nx, ny, bar, slack_eps):
    """tr, ref: [nrec][1 + npts]; the count of fresh cells may differ only by
    cells within slack_eps of the threshold in the oracle's state."""
    np.testing.assert_allclose(tr[:, 1:], ref[:, 1:], rtol=0, atol=bar)
    dq = np.abs(tr[:, 0] - ref[:, 0]) * ny * ny
    assert (dq == np.round(dq)).all()
    assert dq.max() <= slack_eps, dq


@pytest.mark.parametrize("model,phys,grid,nrec,prec,bar", [
    (None, hi.PHYS, (16, 8, 50), 10, hm.PREC_FP64, 1e-8),
    (None, hi.PHYS, (16, 8, 50), 7, hm.PREC_MIXED, 1e-5),
    ("two_layer", hi.PHYS_TABLE1, (32, 16, 188), 48, hm.PREC_FP64, 1e-8),
    ("two_layer", hi.PHYS_TABLE1, (32, 16, 188), 47, hm.PREC_MIXED, 1e-5),
])
def test_trace_matches_oracle(torch_cuda, model, phys, grid, nrec, prec, bar):
    torch = torch_cuda
    nx, ny, r = grid
    xi = hm.henry_sample_xi(0, 40, 0, 3, 3)
    ctx = hm.Context(phys, 0)
    out = hm.solve(ctx, [grid] * 3, xi=dev(torch, xi), opts=hm.make_opts(prec=prec, tol=1e-10, max_outer=60),
                   model=model, trace=(nrec, PTS))
    torch.cuda.synchronize()
    ctx.close()
    assert (out["status"].cpu().numpy() == 0).all()
    tr = out["trace"].cpu().numpy()
    assert tr.shape == (3, nrec, 1 + len(PTS))
    fields = oracle.fields_two_layer if model == "two_layer" else oracle.fields_closed
    for s in range(3):
        phi, K, q = fields(phys, nx, ny, xi[s])
        ref, o = oracle.trace(phys, r, phi, K, q, nrec, PTS)
        steps = oracle.record_steps(r, nrec)
        near = max(int(np.count_nonzero(np.abs(o["c_traj"][st] - oracle.FRESH) < 1e-6)) for st in steps)
        check_trace(tr[s], ref, o["c"], nx, ny, bar, near)


def test_trace_is_bitwise_the_same_across_launch_shapes(torch_cuda):
    torch = torch_cuda
    solves = [(256, 128, 40), (64, 32, 40), (16, 8, 40)]
    xi = dev(torch, hm.henry_sample_xi(0, 41, 0, len(solves), 3))
    ctx = hm.Context(hi.PHYS, 0)
    base = dict(prec=hm.PREC_MIXED, tol=1e-9, max_outer=60)
    plain = hm.solve(ctx, solves, xi=xi, opts=hm.make_opts(**base, cluster=1))
    ref = hm.solve(ctx, solves, xi=xi, opts=hm.make_opts(**base, cluster=1), trace=(8, PTS))
    torch.cuda.synchronize()
    assert torch.equal(plain["c"], ref["c"]) and torch.equal(plain["qoi"], ref["qoi"])
    variants = [dict(cluster=2), dict(cluster=4), dict(cluster=1, steps_per_launch=7), dict(cluster=4, steps_per_launch=5)]
    for v in variants:
        for rep in range(2):  # a replayed graph too
            out = hm.solve(ctx, solves, xi=xi, opts=hm.make_opts(**base, **v), trace=(8, PTS))
            torch.cuda.synchronize()
            assert torch.equal(out["trace"], ref["trace"]), v
            assert torch.equal(out["c"], ref["c"]), v
    ctx.close()


def test_nonfinite_solve_has_nan_records(torch_cuda):
    torch = torch_cuda
    solves = [(16, 8, 50)] * 3
    xi = hm.henry_sample_xi(0, 42, 0, 3, 3)
    bad = xi.copy()
    bad[1, 0] = np.nan
    ctx = hm.Context(hi.PHYS, 0)
    opts = hm.make_opts(prec=hm.PREC_MIXED, tol=1e-9, max_outer=60)
    out = hm.solve(ctx, solves, xi=dev(torch, bad), opts=opts, trace=(10, PTS))
    ref = hm.solve(ctx, [solves[0], solves[2]], xi=dev(torch, xi[[0, 2]]), opts=opts, trace=(10, PTS))
    torch.cuda.synchronize()
    ctx.close()
    assert list(out["status"].cpu().numpy()) == [hm.STATUS_OK, hm.STATUS_NONFINITE, hm.STATUS_OK]
    tr = out["trace"].cpu().numpy()
    assert np.isnan(tr[1]).all()
    assert np.array_equal(tr[[0, 2]], ref["trace"].cpu().numpy())


def test_sample_stats_match_oracle(torch_cuda):
    torch = torch_cuda
    ctx = hm.Context(hi.PHYS, 0)
    rng = np.random.default_rng(9)
    for ns, nv in ((1, 3), (2, 5), (7, 1), (600, 13), (1000, 77), (8192, 3)):
        x = rng.normal(size=(ns, nv))
        x[:, 0] = np.round(x[:, 0])  # ties
        mean, var, q = hm.henry_sample_stats(ctx, dev(torch, x), PROBS)
        torch.cuda.synchronize()
        mean, var, q = mean.cpu().numpy(), var.cpu().numpy(), q.cpu().numpy()
        np.testing.assert_allclose(mean, x.mean(axis=0), rtol=1e-13, atol=1e-15)
        if ns > 1:
            np.testing.assert_allclose(var, x.var(axis=0, ddof=1), rtol=1e-12)
        else:
            assert (var == 0).all()
        for k, p in enumerate(PROBS):
            want = [oracle.quantile7(x[:, v], p) for v in range(nv)]
            np.testing.assert_allclose(q[k], want, rtol=0, atol=4e-16 * np.abs(x).max())
    # NaN sorts last: the lower quantiles of a column with a few NaN stay defined
    x = rng.normal(size=(100, 2))
    x[:3, 1] = np.nan
    mean, var, q = hm.henry_sample_stats(ctx, dev(torch, x), [0.0, 0.5])
    torch.cuda.synchronize()
    mean, q = mean.cpu().numpy(), q.cpu().numpy()
    assert np.isnan(mean[1]) and not np.isnan(mean[0])
    assert q[0, 1] == np.nanmin(x[:, 1])
    with pytest.raises(hm.HenryError):
        hm.henry_sample_stats(ctx, dev(torch, np.zeros((8193, 1))), [0.5])
    # without quantiles there is no sort and no limit on the sample count
    x = rng.normal(size=(50000, 3))
    y = rng.normal(size=(50000, 3))
    mean, var, _ = hm.henry_sample_stats(ctx, dev(torch, x).view(50000, 3), (), x_sub=dev(torch, y).view(50000, 3))
    torch.cuda.synchronize()
    np.testing.assert_allclose(mean.cpu().numpy(), (x - y).mean(axis=0), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(var.cpu().numpy(), (x - y).var(axis=0, ddof=1), rtol=1e-12)
    with pytest.raises(hm.HenryError):
        hm.henry_sample_stats(ctx, dev(torch, np.zeros((4, 1))), [1.5])
    ctx.close()


def test_first_passage_matches_oracle(torch_cuda):
    torch = torch_cuda
    ctx = hm.Context(hi.PHYS_TABLE1, 0)
    xi = hm.henry_qmc_points(1, 64, 3)
    out = hm.solve(ctx, [(32, 16, 188)] * 64, xi=dev(torch, xi),
                   opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-9, max_outer=60), model="two_layer",
                   trace=(48, PTS12))
    torch.cuda.synchronize()
    tr = out["trace"]
    th = tr.cpu().numpy()
    for col, thr, below in ((0, 1.2, True), (0, 1.7, True), (4, 0.9, False), (1, 0.5, False), (0, -1.0, True)):
        t, hist = hm.henry_first_passage(ctx, tr, col, thr, below)
        torch.cuda.synchronize()
        want = [oracle.first_passage(th[s, :, col], thr, below) for s in range(64)]
        assert list(t.cpu().numpy()) == want
        assert list(hist.cpu().numpy()) == list(np.bincount(want, minlength=49))
    ctx.close()


def test_series_run_statistics(torch_cuda):
    """The ensemble driver's layout: its mean, variance, quantiles and
    first-passage histograms are those of its own trace, per record and
    quantity."""
    torch = torch_cuda
    ctx = hm.Context(hi.PHYS_TABLE1, 0)
    xi = hm.henry_qmc_points(1, 40, 3)
    pas = ((0, 1.7, True), (4, 0.5, False))
    res = hm.series_run(ctx, (32, 16, 188), xi, 47, passages=pas, model="two_layer",
                        opts=hm.make_opts(prec=hm.PREC_MIXED, tol=1e-9, max_outer=60))
    torch.cuda.synchronize()
    ctx.close()
    assert res["nonconverged"] == 0
    tr = res["trace"].cpu().numpy()
    assert tr.shape == (40, 47, 13)
    np.testing.assert_allclose(res["mean"].cpu().numpy(), tr.mean(axis=0), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(res["var"].cpu().numpy(), tr.var(axis=0, ddof=1), rtol=1e-11, atol=1e-18)
    q = res["q"].cpu().numpy()
    for k, p in enumerate((0.025, 0.25, 0.5, 0.75, 0.975)):
        want = np.array([[oracle.quantile7(tr[:, r, c], p) for c in range(13)] for r in range(47)])
        np.testing.assert_allclose(q[k], want, rtol=0, atol=1e-15)
    for (col, thr, below), (t, hist) in zip(pas, res["passage"]):
        want = [oracle.first_passage(tr[s, :, col], thr, below) for s in range(40)]
        assert list(t.cpu().numpy()) == want
        assert list(hist.cpu().numpy()) == list(np.bincount(want, minlength=48))


def test_mlmc_series_matches_oracle(torch_cuda):
    """MLMC of the time series on two levels (16x8/50 and 32x16/100, 10
    records at the same times on both): every level's mean and variance of
    Y_l per record and quantity, the telescoped mean and the estimator
    variance equal the oracle's statistics of oracle traces of the same
    samples (FP64 path at tol 1e-10: 1e-8)."""
    torch = torch_cuda
    levels = [(16, 8, 50), (32, 16, 100)]
    m, seed, nrec = [6, 4], 3, 10
    ctx = hm.Context(hi.PHYS, 0)
    res = hm.mlmc_series(ctx, levels, m, nrec, points=PTS12, seed=seed,
                         opts=hm.make_opts(prec=hm.PREC_FP64, tol=1e-10, max_outer=60))
    ctx.close()
    assert res["nonconverged"] == 0
    lm, lv = [], []
    for l, ml in enumerate(m):
        xi = oracle.sample_xi(seed, l, 0, ml, 3)
        fine = [oracle.trace(hi.PHYS, levels[l][2], *oracle.fields_closed(hi.PHYS, *levels[l][:2], x), nrec,
                             PTS12)[0].ravel() for x in xi]
        coarse = None
        if l > 0:
            coarse = [oracle.trace(hi.PHYS, levels[l - 1][2], *oracle.fields_closed(hi.PHYS, *levels[l - 1][:2], x),
                                   nrec, PTS12)[0].ravel() for x in xi]
        a, b = oracle.level_stats(np.array(fine), None if coarse is None else np.array(coarse))
        lm.append(a)
        lv.append(b)
    E, var = oracle.mlmc_estimate(lm, lv, m)
    shape = (nrec, 13)
    lm, lv = np.array(lm).reshape((2,) + shape), np.array(lv).reshape((2,) + shape)
    E, var = E.reshape(shape), var.reshape(shape)
    # c at the points: to the FP64 path's accuracy
    np.testing.assert_allclose(res["level_mean"][..., 1:], lm[..., 1:], rtol=0, atol=1e-8)
    np.testing.assert_allclose(res["level_var"][..., 1:], lv[..., 1:], rtol=1e-6, atol=1e-14)
    np.testing.assert_allclose(res["mean"][:, 1:], E[:, 1:], rtol=0, atol=1e-8)
    np.testing.assert_allclose(res["var_est"][:, 1:], var[:, 1:], rtol=1e-6, atol=1e-14)
    # Q_FW counts cells: equal, unless a cell within the solves' error of the
    # threshold falls on the other side (at most a cell or two per solve)
    assert np.abs(res["level_mean"][..., 0] - lm[..., 0]).max() <= 2 / 64 / min(m)
    # the extremes of the level differences at the points
    for l, ml in enumerate(m):
        xi = oracle.sample_xi(seed, l, 0, ml, 3)
        Y = np.array([oracle.trace(hi.PHYS, levels[l][2], *oracle.fields_closed(hi.PHYS, *levels[l][:2], x), nrec,
                                   PTS12)[0] for x in xi])
        if l > 0:
            Y -= np.array([oracle.trace(hi.PHYS, levels[l - 1][2],
                                        *oracle.fields_closed(hi.PHYS, *levels[l - 1][:2], x), nrec, PTS12)[0]
                           for x in xi])
        np.testing.assert_allclose(res["level_min"][l][:, 1:], Y.min(axis=0)[:, 1:], rtol=0, atol=1e-8)
        np.testing.assert_allclose(res["level_max"][l][:, 1:], Y.max(axis=0)[:, 1:], rtol=0, atol=1e-8)
    assert np.abs(res["mean"][:, 0] - E[:, 0]).max() <= 4 / 64 / min(m)


@pytest.mark.parametrize("grid,nrec", [((2, 1, 6), 6), ((4, 2, 5), 5), ((1024, 512, 3), 3)])
def test_trace_edge_grids(torch_cuda, grid, nrec):
    """Edge cases of the time series: the smallest grids (one and two rows,
    where most points fall on faces or corners), a record after every step,
    16 points (the most a call takes), thresholds that make every cell fresh
    or none, and the largest grid (three steps of 1024x512 at tau = T/3200,
    on a cluster of workgroups) against the oracle's point values and
    counts."""
    torch = torch_cuda
    nx, ny, r = grid
    pts = PTS[:13] + [(0.5, -0.5), (1.5, -0.25), (0.0, 0.0)]
    assert len(pts) == 16
    phys = hi.PHYS if nx < 1024 else dict(hi.PHYS, T=hi.PHYS["T"] * 3 / 3200)
    xi = hm.henry_sample_xi(0, 43, 0, 1, 3)
    ctx = hm.Context(phys, 0)
    opts = hm.make_opts(prec=hm.PREC_MIXED if nx >= 1024 else hm.PREC_FP64, tol=1e-9, max_outer=60)
    outs = {f: hm.solve(ctx, [grid], xi=dev(torch, xi), opts=opts, trace=(nrec, pts, f)) for f in (-1.0, 2.0, 0.012178)}
    torch.cuda.synchronize()
    ctx.close()
    assert (outs[-1.0]["trace"][..., 0] == 0.0).all()
    assert (outs[2.0]["trace"][..., 0] == 2.0).all()
    phi, K, q = oracle.fields_closed(phys, nx, ny, xi[0])
    if nx < 1024:
        ref, o = oracle.trace(phys, r, phi, K, q, nrec, pts)
        tr = outs[0.012178]["trace"][0].cpu().numpy()
        near = max(int(np.count_nonzero(np.abs(o["c_traj"][st] - oracle.FRESH) < 1e-6))
                   for st in oracle.record_steps(r, nrec))
        check_trace(tr, ref, None, nx, ny, 1e-8, near)
    else:
        # the last record against the oracle's point rule on the solve's own final state
        out = outs[0.012178]
        c = out["c"].cpu().numpy().reshape(ny, nx)
        tr = out["trace"][0, -1].cpu().numpy()
        assert tr[0] == oracle.fresh_area(c)
        np.testing.assert_allclose(tr[1:], [oracle.point_value(c, x, y) for x, y in pts], rtol=0, atol=1e-15)
