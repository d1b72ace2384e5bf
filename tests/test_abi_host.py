"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol `include/henry.h` declares, its sample generators and KL basis agree
with the oracle and with a Python integer reference of Philox4x32-10, and
argument validation rejects bad grids and options before any launch."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import henry_inputs as hi
import paper_2302_07804_amd as hm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(hm.LIB_PATH):
        pytest.fail("libhenry.so is not built (run __graft_entry__.build())")
    return hm.lib()


def test_exports_every_declared_symbol(L):
    hdr = open(os.path.join(ROOT, "include", "henry.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", hdr, re.M))
    assert declared == set(hm.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def philox_ref(ctr, key):
    """Philox4x32-10 from its published definition, Python integers."""
    M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
    x = list(ctr)
    k0, k1 = key
    for _ in range(10):
        p0, p1 = M0 * x[0], M1 * x[2]
        x = [((p1 >> 32) ^ x[1] ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF, ((p0 >> 32) ^ x[3] ^ k1) & 0xFFFFFFFF,
             p0 & 0xFFFFFFFF]
        k0, k1 = (k0 + W0) & 0xFFFFFFFF, (k1 + W1) & 0xFFFFFFFF
    return x


def test_python_philox_matches_known_answers():
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt"))
            if not l.startswith("#")]
    for r in rows:
        v = [int(x, 16) for x in r]
        assert philox_ref(v[0:4], v[4:6]) == v[6:10]


@pytest.mark.parametrize("seed,level,first,count,dim", [(0, 0, 0, 64, 3), (0, 4, 1000, 17, 3), (123456789012, 6, 5,
                                                                                                   9, 41)])
def test_sample_xi_bit_exact(L, seed, level, first, count, dim):
    import oracle
    a = hm.henry_sample_xi(seed, level, first, count, dim)
    b = oracle.sample_xi(seed, level, first, count, dim)
    assert np.array_equal(a, b)
    # Python integer reference
    for s in range(count):
        idx = first + s
        for d in range(dim):
            w = philox_ref([d // 2, level, idx & 0xFFFFFFFF, idx >> 32], [seed & 0xFFFFFFFF, seed >> 32])
            e = d % 2
            x = ((w[2 * e + 1] << 32) | w[2 * e]) >> 11
            assert a[s, d] == x * 2.0 ** -52 - 1.0


def test_workspace_validation(L):
    ok = [(16, 8, 50), (256, 128, 800), (1024, 512, 3200)]
    assert hm.henry_workspace_bytes(ok) > 0
    mixed = hm.make_opts(prec=hm.PREC_MIXED)
    fp64 = hm.make_opts(prec=hm.PREC_FP64)
    assert hm.henry_workspace_bytes(ok, fp64) > hm.henry_workspace_bytes(ok, mixed)
    for bad in [[(16, 16, 50)], [(24, 12, 50)], [(16, 8, 0)], [(2048, 1024, 10)], [(0, 0, 5)]]:
        with pytest.raises(hm.HenryError) as e:
            hm.henry_workspace_bytes(bad)
        assert e.value.code == hm.HENRY_EINVAL
    for kw in [dict(prec=7), dict(max_outer=0), dict(tol=0.0), dict(tol=float("nan")), dict(threads=96),
               dict(steps_per_launch=-1), dict(prec=hm.PREC_FP64, threads=1024), dict(threads=2048),
               dict(cluster=3), dict(cluster=16), dict(cluster=-1), dict(cluster_wait_us=-1), dict(predictor=3),
               dict(predictor=-1)]:
        with pytest.raises(hm.HenryError):
            hm.henry_workspace_bytes(ok, hm.make_opts(**kw))
    assert hm.henry_workspace_bytes(ok, hm.make_opts(prec=hm.PREC_MIXED, threads=1024)) > 0
    assert hm.henry_workspace_bytes([]) >= 0


def test_sample_xi_rejects_bad_arguments(L):
    out = (ct.c_double * 3)()
    assert L.henry_sample_xi(0, -1, 0, 1, 3, out) == hm.HENRY_EINVAL
    assert L.henry_sample_xi(0, 0, 0, 1, 0, out) == hm.HENRY_EINVAL
    assert L.henry_sample_xi(0, 0, 0, 1, 3, None) == hm.HENRY_EINVAL


def test_solve_batch_rejects_null_context(L):
    g = hm.grids([(16, 8, 50)])
    rc = L.henry_solve_batch(None, g, 1, 0, None, None, None, None, None, None, None, None, None, None, None, None,
                             0, None)
    assert rc == hm.HENRY_EINVAL
    assert hm.strerror(hm.HENRY_EINVAL) == "invalid argument"


def test_residual_batch_rejects_bad_arguments(L):
    g = hm.grids([(16, 8, 50)])
    null = [None] * 9
    assert L.henry_residual_batch(None, g, 1, 0, *null, None, 0, None) == hm.HENRY_EINVAL
    assert L.henry_residual_batch(None, g, 0, 0, *null, None, 0, None) == hm.HENRY_EINVAL


@pytest.mark.parametrize("nx,ny", [(16, 8), (64, 32), (256, 128)])
def test_kl_basis_matches_oracle(L, nx, ny):
    from oracle import kl
    lam, modes = hm.henry_kl_basis(nx, ny)
    lam_o, modes_o = kl.basis(nx, ny)
    np.testing.assert_allclose(lam, lam_o, rtol=1e-12)
    assert np.abs(modes - modes_o).max() <= 1e-11 * np.abs(modes_o).max()


@pytest.mark.parametrize("seed,level,first,count", [(0, 0, 0, 40), (hi.SEED, 3, (1 << 32) + 5, 9)])
def test_sample_xi_kl_matches_oracle(L, seed, level, first, count):
    from oracle import kl
    a = hm.henry_sample_xi_kl(seed, level, first, count)
    b = kl.sample_xi41(seed, level, first, count)
    # the uniform component is exact; the normals go through libm log/cos/sin
    assert np.array_equal(a[:, 40], b[:, 40])
    np.testing.assert_allclose(a, b, rtol=4e-16, atol=4e-16)


def test_kl_entry_points_reject_bad_arguments(L):
    lam = np.empty(20); modes = np.empty((20, 8, 16))
    dp = lambda a: a.ctypes.data_as(ct.POINTER(ct.c_double))
    assert L.henry_kl_basis(16, 8, 0, 0.3, 200, dp(lam), dp(modes)) == hm.HENRY_EINVAL
    assert L.henry_kl_basis(16, 8, 20, -0.3, 200, dp(lam), dp(modes)) == hm.HENRY_EINVAL
    assert L.henry_kl_basis(16, 9, 20, 0.3, 200, dp(lam), dp(modes)) == hm.HENRY_EINVAL
    assert L.henry_ctx_set_kl(None, 16, 8, 0.3, 0.1, 0.5) == hm.HENRY_EINVAL
    assert L.henry_sample_xi_kl(0, 0, 0, -1, dp(lam)) == hm.HENRY_EINVAL


def test_time_series_entry_points_reject_bad_arguments(L):
    """Argument checks of the time-series and statistics calls run before
    any device work (no GPU needed).  An empty batch returns at once once
    its arguments pass, so a placeholder context handle (never dereferenced
    on these paths) tells the checks apart from the missing-context one."""
    g = hm.grids([(16, 8, 50)])
    D = ct.POINTER(ct.c_double)
    pts = (ct.c_double * 4)(1.6, -0.95, 1.85, -0.95)
    far = (ct.c_double * 2)(2.5, -0.5)
    tr = ct.c_void_p(8)  # never dereferenced
    handle = ct.c_void_p(16)

    def trace(ctx=handle, nsolves=0, nrec=10, npts=2, points=pts, fresh=0.012178, out=tr):
        return L.henry_solve_batch_trace(ctx, g, nsolves, 0, None, None, None, None, None, None, nrec, npts,
                                         ct.cast(points, D) if points is not None else None, fresh, out, None, None,
                                         None, None, None, None, 0, None)

    assert trace() == hm.HENRY_OK  # valid request, empty batch
    assert trace(ctx=None) == hm.HENRY_EINVAL
    assert trace(nrec=0) == hm.HENRY_EINVAL
    assert trace(npts=17) == hm.HENRY_EINVAL
    assert trace(npts=-1) == hm.HENRY_EINVAL
    assert trace(points=None) == hm.HENRY_EINVAL
    assert trace(points=far, npts=1) == hm.HENRY_EINVAL
    assert trace(fresh=float("nan")) == hm.HENRY_EINVAL
    assert trace(out=None) == hm.HENRY_EINVAL
    assert trace(ctx=None, nsolves=1, nrec=51) == hm.HENRY_EINVAL  # more records than steps
    probs = (ct.c_double * 2)(0.25, 0.75)
    bad = (ct.c_double * 2)(0.25, 1.5)
    x = ct.c_void_p(8)
    for args in ((0, 3, x, 2, probs), (8193, 3, x, 2, probs), (10, -1, x, 2, probs), (10, 3, x, 17, probs),
                 (10, 3, x, 2, bad), (10, 3, None, 2, probs)):
        assert L.henry_sample_stats(handle, *args[:3], None, *args[3:], x, x, x, None) == hm.HENRY_EINVAL, args
    assert L.henry_sample_stats(None, 10, 3, x, None, 2, probs, x, x, x, None) == hm.HENRY_EINVAL
    for args in ((-1, 5, 3, 1), (10, 0, 3, 1), (10, 5, 0, 0), (10, 5, 3, 3), (10, 5, 3, -1)):
        assert L.henry_first_passage(handle, *args, x, 0.5, 1, x, x, None) == hm.HENRY_EINVAL, args
    assert L.henry_first_passage(handle, 10, 5, 3, 1, x, float("inf"), 1, x, x, None) == hm.HENRY_EINVAL
    assert L.henry_first_passage(handle, 0, 5, 3, 1, x, 0.5, 1, x, None, None) == hm.HENRY_OK  # nothing to do


def test_tuner_trial_batch_keeps_every_time_step():
    """The tuner's shortened trial batch (trial_frac > 1) divides every
    solve's step count by one common factor f (so each keeps its time step
    tau = T / r with horizon T / f), nearest the requested factor among the
    divisors of the steps' gcd that leave at least min_steps steps; factor 1
    (the default) is the caller's batch itself."""
    solves = [(16, 8, 50), (32, 16, 100), (64, 32, 200), (128, 64, 400), (256, 128, 800)]
    f, short = hm._short_batch(solves, target=5)
    assert f == 5 and short == [(s[0], s[1], s[2] // 5) for s in solves]
    f, short = hm._short_batch(solves, target=1)
    assert f == 1 and short == [tuple(s) for s in solves]
    # 50 / 25 = 2 steps is below min_steps = 8: the largest factor allowed is 5 (50 / 5 = 10 steps)
    f, _ = hm._short_batch(solves, target=25)
    assert f == 5
    f, short = hm._short_batch([(16, 8, 7), (32, 16, 21)], target=5)
    assert f == 1 and short == [(16, 8, 7), (32, 16, 21)]


def test_tuner_stream_plans():
    """Stream of each one-workgroup grid under the tuner's plans: the
    built-in plan (-1), one lane beside the cluster groups (stream 1), the
    costlier half on stream 1 and the cheaper on stream 2, spread over
    streams 1..3 in cost order, or everything on stream 0."""
    costs = {128: 4.0, 64: 2.0, 32: 3.0, 16: 1.0}
    assert hm._plan_streams("built-in", costs) == {nx: -1 for nx in costs}
    assert hm._plan_streams("one lane", costs) == {nx: 1 for nx in costs}
    assert hm._plan_streams("halves", costs) == {128: 1, 32: 1, 64: 2, 16: 2}
    assert hm._plan_streams("halves", {128: 3.0, 64: 2.0, 16: 1.0}) == {128: 1, 64: 1, 16: 2}
    assert hm._plan_streams("spread", costs) == {128: 1, 32: 2, 64: 3, 16: 1}
    assert hm._plan_streams("serial", costs) == {nx: 0 for nx in costs}
    assert set(hm.STREAM_PLANS) == {"built-in", "one lane", "spread", "serial"}
