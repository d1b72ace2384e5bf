"""Pins of the oracle's Karhunen-Loeve fields against facts fixed outside it.

  * 1D eigenvalues     -- the trace identity sum(lam) = |I| (C(x,x) = 1) and
                          the Hilbert-Schmidt identity sum(lam^2) =
                          int int C^2, which has a closed form with erf;
                          an independent midpoint-rule discretisation;
  * eigenfunctions     -- the eigen-equation and orthonormality checked off
                          the Nystrom nodes with scipy's adaptive quadrature;
                          even/odd symmetry about the interval midpoint;
  * 2D basis           -- products of 1D pairs, descending eigenvalues,
                          orthonormality under the cell-centre rule;
  * Gaussian sampler   -- normal moments and a Kolmogorov-Smirnov test of the
                          Box-Muller map, uncorrelated components;
  * field map          -- special values at xi = 0, the pointwise variance
                          sum lam_k e_k(x)^2 against a sample variance;
  * KL gradient        -- central finite differences of the oracle solve.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import henry_inputs as hi
import oracle
from oracle import kl


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


@pytest.mark.parametrize("a,b", [(0.0, 2.0), (-1.0, 0.0)])
def test_trace_and_hilbert_schmidt_identities(a, b):
    lam, _, _, _ = kl.nystrom_1d(a, b)
    L, l = b - a, kl.CORR_LEN
    assert abs(lam.sum() - L) < 1e-12 * L
    # int_0^L int_0^L exp(-(s-t)^2 / l^2) ds dt
    hs = L * l * math.sqrt(math.pi) * math.erf(L / l) - l * l * (1.0 - math.exp(-(L / l) ** 2))
    assert abs((lam ** 2).sum() - hs) < 1e-12 * hs


def test_eigenvalues_match_independent_midpoint_discretisation():
    lam, _, _, _ = kl.nystrom_1d(0.0, 2.0)

    def midpoint(N):
        t = (np.arange(N) + 0.5) * (2.0 / N)
        C = np.exp(-(t[:, None] - t[None, :]) ** 2 / (2 * kl.CORR_LEN ** 2)) * (2.0 / N)
        return np.sort(np.linalg.eigvalsh(C))[::-1][:12]

    # the midpoint rule is O(h^2): Richardson extrapolation of two levels
    m1, m2 = midpoint(1500), midpoint(3000)
    np.testing.assert_allclose(lam[:12], (4.0 * m2 - m1) / 3.0, rtol=1e-8)


def test_eigen_equation_and_orthonormality_off_nodes():
    lam, X, W, E = kl.nystrom_1d(0.0, 2.0)
    l = kl.CORR_LEN
    e = lambda k, s: kl.eval_1d(lam, X, W, E, np.atleast_1d(s))[k, 0]
    for k in (0, 3, 7):
        for x in (0.013, 0.7, 1.91):
            lhs = integrate.quad(lambda t: math.exp(-(x - t) ** 2 / (2 * l * l)) * e(k, t), 0.0, 2.0,
                                 epsabs=1e-13, epsrel=1e-12, limit=200)[0]
            assert abs(lhs - lam[k] * e(k, x)) < 1e-9 * max(1.0, abs(lam[k] * e(k, x)))
    for k in (0, 2, 5):
        for m in (0, 2, 5, 6):
            ip = integrate.quad(lambda t: e(k, t) * e(m, t), 0.0, 2.0, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
            assert abs(ip - (1.0 if k == m else 0.0)) < 1e-9


def test_eigenfunctions_alternate_even_odd_about_midpoint():
    lam, X, W, E = kl.nystrom_1d(0.0, 2.0)
    s = np.linspace(0.05, 0.95, 7)
    f = kl.eval_1d(lam, X, W, E, s)
    g = kl.eval_1d(lam, X, W, E, 2.0 - s)
    for k in range(10):
        np.testing.assert_allclose(g[k], (-1) ** k * f[k], atol=1e-10)


def test_2d_basis_products_ordering_orthonormality():
    nx, ny = 256, 128
    lam, modes = kl.basis(nx, ny)
    assert np.all(np.diff(lam) <= 0)
    lx = kl.nystrom_1d(0.0, 2.0)[0]
    ly = kl.nystrom_1d(-1.0, 0.0)[0]
    prods = np.sort(np.outer(lx[:20], ly[:20]).ravel())[::-1][:20]
    np.testing.assert_allclose(lam, prods, rtol=1e-13)
    h = 1.0 / ny
    G = np.tensordot(modes, modes, axes=([1, 2], [1, 2])) * h * h
    assert np.abs(G - np.eye(20)).max() < 2e-3     # midpoint rule, O(h^2)
    # each 2D mode separates: rank-1 as a [ny][nx] matrix
    for k in range(20):
        sv = np.linalg.svd(modes[k], compute_uv=False)
        assert sv[1] < 1e-12 * sv[0]


def test_box_muller_normals():
    x = kl.sample_xi41(hi.SEED, 1, 0, 1500)
    z = x[:, :40].ravel()
    n = z.size
    assert abs(z.mean()) < 4.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    R = np.corrcoef(x[:, :40].T)
    assert np.abs(R - np.eye(40)).max() < 5.0 / math.sqrt(x.shape[0])
    u = x[:, 40]
    assert u.min() >= -1.0 and u.max() < 1.0
    assert stats.kstest((u + 1.0) / 2.0, "uniform").pvalue > 1e-3


def test_field_map_special_values_and_variance(phys):
    nx, ny = 32, 16
    lam, modes = kl.basis(nx, ny)
    phi, K, q = kl.fields(phys, lam, modes, np.zeros(41))
    assert np.all(phi == phys["phi0"]) and np.allclose(K, phys["k0"], rtol=1e-15) and q == phys["q_in"]
    x = kl.sample_xi41(hi.SEED, 0, 0, 3000)
    logk = np.array([np.log(kl.fields(phys, lam, modes, xi)[1]) for xi in x])
    var_pred = kl.SIGMA_LOGK ** 2 * np.tensordot(lam, modes ** 2, axes=1)
    var_mc = logk.var(axis=0, ddof=1)
    # chi-square: relative sd of a sample variance is sqrt(2/(n-1))
    assert np.abs(var_mc / var_pred - 1.0).max() < 5.0 * math.sqrt(2.0 / 2999)
    # captured fraction of the pointwise variance of a unit field
    frac = np.tensordot(lam, modes ** 2, axes=1)
    assert 0.5 < frac.min() and frac.max() <= 1.0 + 1e-12


def test_kl_gradient_matches_central_differences(phys):
    nx, ny, r = 16, 8, 20
    lam, modes = kl.basis(nx, ny)
    xi = kl.sample_xi41(hi.SEED, 2, 7, 1)[0]
    Q, g = kl.adjoint_kl(phys, r, xi, lam, modes)
    rng = np.random.default_rng(5)
    for _ in range(2):
        v = rng.standard_normal(41)
        eps = 1e-4
        qp = kl.solve_kl(phys, nx, ny, r, xi + eps * v, lam, modes)[0]
        qm = kl.solve_kl(phys, nx, ny, r, xi - eps * v, lam, modes)[0]
        fd = (qp - qm) / (2 * eps)
        assert abs(fd - g @ v) < 1e-6 * abs(fd) + 1e-12 * abs(Q)
    # one coefficient of each kind on its own
    for k in (0, 25, 40):
        e = np.zeros(41); e[k] = 1e-4
        fd = (kl.solve_kl(phys, nx, ny, r, xi + e, lam, modes)[0]
              - kl.solve_kl(phys, nx, ny, r, xi - e, lam, modes)[0]) / 2e-4
        assert abs(fd - g[k]) < 1e-5 * abs(g).max()
