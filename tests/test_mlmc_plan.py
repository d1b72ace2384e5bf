"""MLMC planning entry points of the library (host code, no GPU):
henry_mlmc_allocate against Table 3 of the paper (tests/golden) and against
the oracle's eq:M_ell on random levels; henry_mlmc_rates against numpy's
least-squares line fit and the closed form of its bias estimate."""
import math
import os

import numpy as np
import pytest

import paper_2302_07804_amd as hm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(hm.LIB_PATH):
        pytest.fail("libhenry.so is not built (run __graft_entry__.build())")
    return hm.lib()


def test_allocation_reproduces_table3(L):
    lines = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "table3_mlmc_samples.txt"))
             if not l.startswith("#")]
    s = [float(x) for x in lines[0][1:]]
    V = [float(x) for x in lines[1][1:]]
    for row in lines[2:]:
        m, cost = hm.henry_mlmc_allocate(V, s, float(row[1]))
        assert list(m) == [int(x) for x in row[2:]]
        assert cost == pytest.approx(sum(math.sqrt(v * w) for v, w in zip(V, s)) ** 2 / float(row[1]), rel=1e-15)


def test_allocation_matches_oracle_on_random_levels(L):
    import oracle
    rng = np.random.default_rng(11)
    for _ in range(50):
        n = int(rng.integers(1, 9))
        V = 10.0 ** rng.uniform(-9, -3, n)
        s = 10.0 ** rng.uniform(-1, 4, n)
        eps2 = 10.0 ** rng.uniform(-9, -5)
        m, cost = hm.henry_mlmc_allocate(V, s, eps2)
        mo, co = oracle.optimal_samples(V, s, eps2)
        assert np.array_equal(m, mo)
        # numpy adds eight levels pairwise, the library in level order
        assert cost == pytest.approx(co, rel=1e-14)
        # the allocation meets the variance target
        assert (V / np.maximum(m, 1)).sum() <= eps2 * (1 + 1e-12)


def test_rates_match_least_squares_fit(L):
    rng = np.random.default_rng(12)
    for _ in range(20):
        n = int(rng.integers(3, 8))
        lev = np.arange(n)
        mean = 0.3 * 2.0 ** (-rng.uniform(0.5, 2) * lev) * np.exp(0.1 * rng.standard_normal(n))
        mean *= rng.choice([-1.0, 1.0], n)
        var = 0.02 * 2.0 ** (-rng.uniform(1, 3) * lev) * np.exp(0.1 * rng.standard_normal(n))
        a, b, bias = hm.henry_mlmc_rates(mean, var, 1)
        assert a == pytest.approx(-np.polyfit(lev[1:], np.log2(np.abs(mean[1:])), 1)[0], rel=1e-12, abs=1e-12)
        assert b == pytest.approx(-np.polyfit(lev[1:], np.log2(var[1:]), 1)[0], rel=1e-12, abs=1e-12)
        assert bias == pytest.approx(abs(mean[-1]) / (2.0 ** a - 1.0), rel=1e-12)


def test_rates_of_exact_geometric_levels(L):
    lev = np.arange(6)
    a, b, bias = hm.henry_mlmc_rates(0.5 * 2.0 ** (-lev), 0.1 * 4.0 ** (-lev), 1)
    assert a == pytest.approx(1.0, abs=1e-13) and b == pytest.approx(2.0, abs=1e-13)
    # E[Y_l] = 0.5 * 2^-l: the levels beyond 5 add 0.5 * 2^-5 in all
    assert bias == pytest.approx(0.5 * 2.0 ** -5, rel=1e-12)


def test_planning_rejects_bad_arguments(L):
    with pytest.raises(hm.HenryError):
        hm.henry_mlmc_allocate([1e-5, -1e-6], [1.0, 2.0], 1e-6)
    with pytest.raises(hm.HenryError):
        hm.henry_mlmc_allocate([1e-5], [0.0], 1e-6)
    with pytest.raises(hm.HenryError):
        hm.henry_mlmc_allocate([1e-5], [1.0], 0.0)
    with pytest.raises(hm.HenryError):
        hm.henry_mlmc_rates([1.0, 0.5], [1.0, 0.5], 1)  # one level in the fit
    with pytest.raises(hm.HenryError):
        hm.henry_mlmc_rates([1.0, 0.5, 0.0], [1.0, 0.5, 0.2], 1)  # zero mean in the fit


def test_allocation_meets_the_variance_target_at_near_optimal_cost(L):
    """eq:M_ell is the minimiser of the cost sum m_l s_l subject to the
    estimator variance sum V_l / m_l = eps^2: rounded up, the counts meet
    the target and cost at most one sample per level more than the
    continuous optimum, and every randomly perturbed integer allocation
    that still meets the target costs at least that optimum."""
    rng = np.random.default_rng(12)
    for _ in range(200):
        n = int(rng.integers(1, 7))
        V = 10.0 ** rng.uniform(-9, -3, n)
        s = 10.0 ** rng.uniform(-2, 3, n)
        eps2 = 10.0 ** rng.uniform(-9, -5)
        m, cost = hm.henry_mlmc_allocate(V, s, eps2)
        assert (V / m).sum() <= eps2 * (1 + 1e-12)
        assert cost <= (m * s).sum() <= cost + s.sum() * (1 + 1e-12)
        # any other integer allocation that meets the target costs at least the continuous optimum
        for _ in range(5):
            mm = np.maximum(1, np.round(m * 10.0 ** rng.uniform(-0.3, 0.3, n))).astype(np.int64)
            if (V / mm).sum() <= eps2:
                assert (mm * s).sum() >= cost * (1 - 1e-12)
