"""Adaptive MLMC driver (Sec. 3) on the GPU, against the oracle: the sample
counts are eq:M_ell of the driver's own pilot variances and measured costs
(the oracle's allocation), and the estimate E[Q], the estimator variance
and the fitted rates equal those of oracle solves of the same samples (keys
(seed, l, i), FP64 path at tol 1e-10: Q agrees to ~1e-11)."""
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
    hm.lib()
    return torch


def test_adaptive_mlmc_matches_oracle(torch_cuda):
    levels = [(16, 8, 50), (32, 16, 100), (64, 32, 200)]
    eps, m_pilot, seed = 0.2, 16, 5
    ctx = hm.Context(hi.PHYS, 0)
    res = hm.mlmc_run(ctx, levels, eps, m_pilot=m_pilot, seed=seed,
                      opts=hm.make_opts(prec=hm.PREC_FP64, tol=1e-10, max_outer=60))
    ctx.close()
    assert res["nonconverged"] == 0
    m = res["m"]
    mo, _ = oracle.optimal_samples(res["V_pilot"], res["s"], eps * eps / 2)
    assert np.array_equal(m, np.maximum(mo, m_pilot)), (m, mo)
    print(f"m = {list(m)}, E[Q] = {res['EQ']:.6f}, var = {res['var_est']:.3e}, "
          f"alpha = {res['alpha']:.3f}, beta = {res['beta']:.3f}, bias = {res['bias']:.3e}")
    # the same samples through the oracle
    jobs, where = [], []
    for l, ml in enumerate(m):
        xi = oracle.sample_xi(seed, l, 0, int(ml), 3)
        for i in range(ml):
            where.append((l, 0))
            jobs.append((*levels[l], xi[i]))
            if l > 0:
                where.append((l, 1))
                jobs.append((*levels[l - 1], xi[i]))
    refs = oracle.solve_many(hi.PHYS, jobs)
    q = {}
    for (l, side), r in zip(where, refs):
        q.setdefault((l, side), []).append(r["qoi"])
    means, vars_ = [], []
    for l in range(len(levels)):
        mean, var = oracle.level_stats(np.array(q[(l, 0)]), np.array(q[(l, 1)]) if l > 0 else None)
        means.append(float(mean)); vars_.append(float(var))
    EQ, var_est = oracle.mlmc_estimate(means, vars_, list(m))
    assert res["EQ"] == pytest.approx(EQ, rel=1e-8)
    assert res["var_est"] == pytest.approx(var_est, rel=1e-6)
    np.testing.assert_allclose(res["mean"], means, rtol=1e-7, atol=1e-9 * abs(EQ))
    lev = np.arange(1, len(levels))
    assert res["alpha"] == pytest.approx(-np.polyfit(lev, np.log2(np.abs(means[1:])), 1)[0], rel=1e-6)
    assert res["beta"] == pytest.approx(-np.polyfit(lev, np.log2(vars_[1:]), 1)[0], rel=1e-6)
