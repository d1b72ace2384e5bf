"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test names what pins which part:
  * sample generator   -- published Philox4x32-10 known answers; exactness
                          and moments of the uniform map;
  * random fields      -- special values and symmetries of the closed forms;
  * banded LU          -- numpy's dense LAPACK solve (plain and transposed);
  * Jacobian           -- central finite differences of the residual;
  * conservation       -- interior fluxes cancel; the accumulation equals the
                          change of the total fluid/salt mass;
  * buoyancy, right BC -- the hydrostatic seawater state has zero Darcy flux;
  * diffusion, BCs,
    time stepping      -- the exact discrete sine-series solution of 1D
                          diffusion between c = 0 and c = 1;
  * harmonic K / phi   -- series-resistance exactness for cellwise-constant
                          coefficients (continuum integrals);
  * upwind advection,
    inflow BC          -- the steady upwind recurrence for uniform flow;
  * convergence order  -- first-order self-convergence (Sec. 2.3);
  * MLMC statistics    -- telescoping identity, numpy's unbiased variance,
                          Table 3 of the paper (eq:M_ell);
  * QMC                -- radical-inverse values; Halton vs MC mean;
  * adjoint            -- tangent-linear/adjoint duality and central FD.
"""
import math
import os

import numpy as np
import pytest

import henry_inputs as hi
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def phys_with(**kw):
    p = dict(hi.PHYS)
    p.update(kw)
    return p


# ---------------------------------------------------------------- generator
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert oracle.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])


def test_xi_exact_and_uniform():
    xi = oracle.sample_xi(0, 0, 0, 200000, 3)
    assert xi.min() >= -1.0 and xi.max() < 1.0
    k = (xi + 1.0) * 2.0 ** 52
    assert np.all(k == np.floor(k))                      # 53-bit lattice, exact
    assert abs(xi.mean()) < 5e-3
    assert abs(xi.var() - 1.0 / 3.0) < 5e-3
    # components and samples are distinct streams
    assert abs(np.corrcoef(xi[:, 0], xi[:, 1])[0, 1]) < 1e-2
    # keys: (seed, level, index) -> the same value however the batch is cut
    a = oracle.sample_xi(0, 3, 10, 5, 3)
    b = oracle.sample_xi(0, 3, 0, 20, 3)
    assert np.array_equal(a, b[10:15])
    assert not np.array_equal(oracle.sample_xi(0, 2, 0, 4, 3), oracle.sample_xi(0, 3, 0, 4, 3))


def test_xi_from_words():
    """A component is the top 53 bits of two Philox words, mapped to [-1,1)."""
    w = oracle.philox4x32_10((0, 0, 7, 0), (0, 0))
    x0 = (((w[1] << 32) | w[0]) >> 11)
    x1 = (((w[3] << 32) | w[2]) >> 11)
    xi = oracle.sample_xi(0, 0, 7, 1, 2)[0]
    assert xi[0] == x0 * 2.0 ** -52 - 1.0 and xi[1] == x1 * 2.0 ** -52 - 1.0


# ---------------------------------------------------------------- fields
def test_fields_special_values(phys):
    phi, K, q = oracle.fields_closed(phys, 16, 8, [0.0, 0.0, 0.0])
    assert np.all(phi == phys["phi0"]) and np.all(K == phys["k0"]) and q == phys["q_in"]
    phi1, K1, q1 = oracle.fields_closed(phys, 16, 8, [0.7, 0.4, -1.0])
    phi2, K2, q2 = oracle.fields_closed(phys, 16, 8, [-0.7, -0.4, 1.0])
    np.testing.assert_allclose(phi1 + phi2, 2 * phys["phi0"], rtol=1e-15)     # odd in xi1
    np.testing.assert_allclose(K1 * K2, phys["k0"] ** 2, rtol=1e-14)           # log K odd in xi2
    assert q1 == pytest.approx(0.8 * phys["q_in"]) and q2 == pytest.approx(1.2 * phys["q_in"])
    # porosity varies along both axes, permeability only along x
    assert np.ptp(phi1, axis=0).max() > 0 and np.ptp(phi1, axis=1).max() > 0
    assert np.ptp(K1, axis=0).max() == 0
    # K grows to the right for xi2 > 0 (sin(pi x/2) > 0 on (0, 2))
    assert np.all(np.diff(K1[0, :8]) > 0)
    phiw, _, _ = oracle.fields_closed(phys, 16, 8, [1.0, 0.0, 0.0])
    assert 0.28 - 1e-12 <= phiw.min() and phiw.max() <= 0.42 + 1e-12


# ---------------------------------------------------------------- banded LU
@pytest.mark.parametrize("n,kl,ku", [(12, 2, 3), (40, 5, 5), (33, 7, 4)])
def test_band_lu_vs_dense(n, kl, ku):
    rng = np.random.default_rng(n)
    A = np.zeros((n, n))
    for r in range(n):
        for c in range(max(0, r - kl), min(n, r + ku + 1)):
            A[r, c] = rng.normal()
    b = rng.normal(size=n)
    x = oracle.band_solve_dense(A, b, kl, ku)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    xt = oracle.band_solve_dense(A, b, kl, ku, trans=True)
    np.testing.assert_allclose(xt, np.linalg.solve(A.T, b), rtol=1e-10, atol=1e-12)


def test_band_lu_on_jacobian(phys):
    nx, ny = 8, 4
    p, c, cn, phi, K, q = hi.random_state(nx, ny, 3)
    J = oracle.jacobian_dense(phys, 50, phi, K, q, p, c, cn)
    kl = 2 * ny + 1
    # the interleaved y-fastest ordering keeps J inside the band
    rr, cc = np.nonzero(J)
    assert np.max(np.abs(rr - cc)) <= kl
    b = np.random.default_rng(0).normal(size=J.shape[0])
    np.testing.assert_allclose(oracle.band_solve_dense(J, b, kl, kl), np.linalg.solve(J, b), rtol=1e-9)
    np.testing.assert_allclose(oracle.band_solve_dense(J, b, kl, kl, trans=True), np.linalg.solve(J.T, b),
                               rtol=1e-9)


# ---------------------------------------------------------------- Jacobian
@pytest.mark.parametrize("nx,ny,seed", [(4, 2, 0), (6, 3, 1), (8, 4, 2)])
def test_jacobian_matches_central_fd(phys, nx, ny, seed):
    p, c, cn, phi, K, q = hi.random_state(nx, ny, seed)
    J = oracle.jacobian_dense(phys, 50, phi, K, q, p, c, cn)
    band = oracle.cell_to_band(nx, ny)
    Jfd = np.zeros_like(J)
    for j in range(ny):
        for i in range(nx):
            u = band[j, i]
            for v, (arr, step) in enumerate(((p, 1e-3), (c, 1e-7))):
                a1 = arr.copy(); a1[j, i] += step
                a2 = arr.copy(); a2[j, i] -= step
                args1 = (a1, c, cn) if v == 0 else (p, a1, cn)
                args2 = (a2, c, cn) if v == 0 else (p, a2, cn)
                R1 = oracle.residual(phys, 50, phi, K, q, *args1)
                R2 = oracle.residual(phys, 50, phi, K, q, *args2)
                col = 2 * u + v
                for w in range(2):
                    d = (R1[w] - R2[w]) / (2 * step)
                    Jfd[2 * band.ravel() + w, col] = d.ravel()
    scale = np.abs(J).max(axis=1, keepdims=True)
    assert np.max(np.abs(J - Jfd) / scale) < 1e-6


# ---------------------------------------------------------------- conservation
def _salt_mass(phys, phi, c, h):
    rho = phys["rho0"] + (phys["rho1"] - phys["rho0"]) * c
    return h * h * np.sum(phi * rho * c)


def _fluid_mass(phys, phi, c, h):
    rho = phys["rho0"] + (phys["rho1"] - phys["rho0"]) * c
    return h * h * np.sum(phi * rho)


def test_interior_fluxes_cancel(phys):
    """Changing p or c in a cell away from the left/right boundaries changes
    the domain totals of R^p and R^c only through the stored mass: every
    interior face flux enters two cells with opposite signs."""
    nx, ny, r = 12, 6, 40
    tau = phys["T"] / r
    h = 1.0 / ny
    p, c, cn, phi, K, q = hi.random_state(nx, ny, 11)
    Rp0, Rc0 = oracle.residual(phys, r, phi, K, q, p, c, cn)
    for (j, i) in [(0, 3), (2, 5), (5, 10), (3, 1)]:
        p1 = p.copy(); p1[j, i] += 37.0
        Rp1, Rc1 = oracle.residual(phys, r, phi, K, q, p1, c, cn)
        assert abs(Rp1.sum() - Rp0.sum()) <= 1e-13 * np.abs(Rp0).sum()
        assert abs(Rc1.sum() - Rc0.sum()) <= 1e-13 * np.abs(Rc0).sum()
        c1 = c.copy(); c1[j, i] = min(1.0, c1[j, i] + 0.3)
        Rp2, Rc2 = oracle.residual(phys, r, phi, K, q, p, c1, cn)
        dsalt = (_salt_mass(phys, phi, c1, h) - _salt_mass(phys, phi, c, h)) / tau
        dfluid = (_fluid_mass(phys, phi, c1, h) - _fluid_mass(phys, phi, c, h)) / tau
        assert abs((Rc2.sum() - Rc0.sum()) - dsalt) <= 1e-12 * np.abs(Rc0).sum()
        assert abs((Rp2.sum() - Rp0.sum()) - dfluid) <= 1e-12 * np.abs(Rp0).sum()


# ---------------------------------------------------------------- hydrostatic
@pytest.mark.parametrize("seed", [0, 1])
def test_hydrostatic_seawater_is_exact(phys, seed):
    """c = 1 everywhere, no recharge, no diffusion: p = -rho1 g y carries no
    Darcy flux (Sec. 2.1, e_Darcy_vel with gravity (0,-g)), so c stays 1."""
    ph = phys_with(D=0.0, q_in=0.0)
    nx, ny, r = 16, 8, 10
    _, _, _, phi, K, _ = hi.random_state(nx, ny, seed)
    h = 1.0 / ny
    y = -1.0 + (np.arange(ny) + 0.5) * h
    p_exact = np.repeat((-ph["rho1"] * ph["g"] * y)[:, None], nx, axis=1)
    one = np.ones((ny, nx))
    Rp, Rc = oracle.residual(ph, r, phi, K, 0.0, p_exact, one, one)
    lam = ph["rho1"] * K.max() / ph["mu"]
    assert np.abs(Rp).max() <= 1e-13 * lam * ph["rho1"] * ph["g"] * h
    assert np.abs(Rc).max() <= 1e-13 * lam * ph["rho1"] * ph["g"] * h
    out = oracle.solve(ph, r, phi, K, 0.0, c0=one)
    assert np.abs(out["c"] - 1.0).max() <= 1e-15
    np.testing.assert_allclose(out["p"], p_exact, rtol=1e-13)


# ---------------------------------------------------------------- 1D diffusion
def test_1d_diffusion_exact_discrete_solution(phys):
    """rho1 = rho0, no recharge, uniform phi and K: p stays hydrostatic, the
    Darcy flux vanishes and c solves implicit-Euler diffusion between c = 0 at
    x = 0 and c = 1 at x = 2 (Sec. 2.1).  The cell-centred Dirichlet
    Laplacian has the discrete sines sin(k pi x_i / 2) as exact eigenvectors
    with eigenvalues (4/h^2) sin^2(k pi h / 4), and x/2 is its exact steady
    state, so c_i^n = x_i/2 - sum_k b_k (1 + tau D mu_k)^-n sin(k pi x_i/2)."""
    ph = phys_with(rho1=phys["rho0"], q_in=0.0)
    nx, ny, r = 16, 8, 25
    h = 1.0 / ny
    tau = ph["T"] / r
    phi = np.full((ny, nx), 0.31)
    K = np.full((ny, nx), 2e-9)
    out = oracle.solve(ph, r, phi, K, 0.0, trajectory=True)
    x = (np.arange(nx) + 0.5) * h
    k = np.arange(1, nx + 1)
    S = np.sin(np.outer(x, k) * np.pi / 2)
    b = np.linalg.solve(S, x / 2)
    D = ph["D"] * 0.31 / 0.31          # diffusion coefficient phi D over storage phi
    mu = 4.0 / h ** 2 * np.sin(k * np.pi * h / 4) ** 2
    for n in (1, 5, r):
        exact = x / 2 - S @ (b * (1 + tau * D * mu) ** (-n))
        np.testing.assert_allclose(out["c_traj"][n], np.broadcast_to(exact, (ny, nx)), atol=2e-14)
    y = -1.0 + (np.arange(ny) + 0.5) * h
    np.testing.assert_allclose(out["p"], np.repeat((-ph["rho0"] * ph["g"] * y)[:, None], nx, 1), rtol=1e-13)


def test_1d_diffusion_continuum_limit(phys):
    """Against the continuum series c = x/2 - sum 2(-1)^(k+1)/(k pi)
    exp(-D (k pi/2)^2 t) sin(k pi x/2): the error falls as h^2 + tau."""
    ph = phys_with(rho1=phys["rho0"], q_in=0.0, T=2000.0)
    errs = []
    for lev in range(3):
        nx, ny, r = 16 << lev, 8 << lev, 10 << (2 * lev)
        phi = np.full((ny, nx), 0.35); K = np.full((ny, nx), 1e-9)
        # only one row is needed for the comparison; keep the full grid
        out = oracle.solve(ph, r, phi, K, 0.0)
        x = (np.arange(nx) + 0.5) / ny
        kk = np.arange(1, 2000)
        ex = x / 2 - (2 * (-1.0) ** (kk + 1) / (kk * np.pi) * np.exp(-ph["D"] * (kk * np.pi / 2) ** 2 * ph["T"])
                      ) @ np.sin(np.outer(kk, x) * np.pi / 2)
        errs.append(np.abs(out["c"][0] - ex).max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


# ---------------------------------------------------------------- harmonic means
def test_series_resistance_diffusion(phys):
    """Steady diffusion through cellwise-constant porosity phi(x): the exact
    flux of the continuous problem is 1 / integral(dx / (rho0 phi D)); the
    harmonic face mean reproduces it, and c at each centre equals the
    continuum value there."""
    ph = phys_with(rho1=phys["rho0"], q_in=0.0, T=1e12)
    nx, ny = 16, 8
    h = 1.0 / ny
    phix = 0.25 + 0.2 * np.random.default_rng(5).uniform(size=nx)
    phi = np.repeat(phix[None, :], ny, 0)
    out = oracle.solve(ph, 3, phi, np.full((ny, nx), 1e-9), 0.0)
    res = h / (ph["rho0"] * phix * ph["D"])             # resistance of each cell (per unit depth)
    F = 1.0 / res.sum() * 1.0                           # (c_right - c_left) / total resistance; face length 1/ny... per row
    c_centre = F * (np.cumsum(res) - res / 2)
    np.testing.assert_allclose(out["c"][3], c_centre, rtol=1e-9, atol=1e-12)


def test_series_resistance_darcy(phys):
    """Uniform recharge through cellwise-constant K(x), rho1 = rho0: the flux
    is rho0 q everywhere and the pressure at each centre is the seawater
    value plus the Darcy drop mu q integral_x^2 dx / K, exactly."""
    ph = phys_with(rho1=phys["rho0"], D=0.0)
    nx, ny = 16, 8
    h = 1.0 / ny
    Kx = 1e-9 * np.exp(np.random.default_rng(9).uniform(-1, 1, size=nx))
    K = np.repeat(Kx[None, :], ny, 0)
    q = ph["q_in"]
    out = oracle.solve(ph, 2, np.full((ny, nx), 0.35), K, q)
    y = -1.0 + (np.arange(ny) + 0.5) * h
    drop_cells = ph["mu"] * q * h / Kx                    # drop across each full cell
    right = drop_cells[::-1].cumsum()[::-1] - drop_cells / 2
    p_exact = (-ph["rho0"] * ph["g"] * y)[:, None] + right[None, :]
    np.testing.assert_allclose(out["p"], p_exact, rtol=1e-12)


def test_upwind_steady_state(phys):
    """Uniform flow to the right (rho1 = rho0, uniform coefficients): at
    steady state the donor-cell flux F = M c_i - delta (c_{i+1} - c_i) is the
    same on every face, with F = -2 delta c_0 at the fresh inflow face and
    F = M c_last - 2 delta (1 - c_last) at the seawater face."""
    ph = phys_with(rho1=phys["rho0"], T=1e13)
    nx, ny = 16, 8
    h = 1.0 / ny
    phi0 = 0.3
    q = ph["q_in"] * 0.3
    out = oracle.solve(ph, 4, np.full((ny, nx), phi0), np.full((ny, nx), 1e-9), q)
    M = ph["rho0"] * q * h
    dl = ph["rho0"] * phi0 * ph["D"]
    alpha = [-1.0 / (2 * dl)]
    for _ in range(nx - 1):
        alpha.append(alpha[-1] * (1 + M / dl) - 1.0 / dl)
    F = -2 * dl / (1 - (M + 2 * dl) * alpha[-1])
    np.testing.assert_allclose(out["c"][2], np.array(alpha) * F, rtol=1e-9, atol=1e-13)


# ---------------------------------------------------------------- Newton / order
def test_newton_solution_has_zero_residual(phys):
    xi = oracle.sample_xi(0, 0, 0, 1, 3)[0]
    phi, K, q = oracle.fields_closed(phys, 16, 8, xi)
    out = oracle.solve(phys, 50, phi, K, q, trajectory=True)
    for n in (1, 25, 50):
        Rp, Rc = oracle.residual(phys, 50, phi, K, q, out["p_traj"][n], out["c_traj"][n], out["c_traj"][n - 1])
        scale = phys["rho1"] * phys["k0"] / phys["mu"] * phys["rho1"] * phys["g"] / 8   # lambda rho g h
        assert np.abs(Rc).max() < 1e-13 * scale and np.abs(Rp).max() < 1e-13 * scale
    assert 0.0 <= out["c"].min() and out["c"].max() <= 1.0
    # salt enters along the bottom of the seawater side (Sec. 2.1, Fig. 1)
    assert out["c"][0, -1] > out["c"][-1, -1] and out["c"][0, -1] > out["c"][0, 0]


@pytest.mark.slow
def test_first_order_self_convergence(phys):
    """Sec. 2.3: first-order behaviour under joint refinement of h and tau."""
    Q = []
    for lev in range(3):
        nx, ny, r = hi.level_grid(lev)
        phi, K, q = oracle.fields_closed(phys, nx, ny, [0.0, 0.0, 0.0])
        Q.append(oracle.solve(phys, r, phi, K, q)["qoi"])
    ratio = (Q[1] - Q[0]) / (Q[2] - Q[1])
    assert 1.3 < ratio < 3.0


# ---------------------------------------------------------------- MLMC statistics
def test_level_stats_unbiased_variance():
    rng = np.random.default_rng(1)
    f = rng.normal(size=(17, 8, 16)); c = rng.normal(size=(17, 4, 8))
    mean, var = oracle.level_stats(f, c)
    Y = f - np.kron(c, np.ones((1, 2, 2)))
    np.testing.assert_allclose(mean, Y.mean(axis=0), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(var, Y.var(axis=0, ddof=1), rtol=1e-13)
    qm, qv = oracle.level_stats(rng.normal(size=9), None)
    assert qv.shape == ()


def test_telescoping_identity_on_shared_samples():
    """With the same samples on every level, sum_l mean(g_l - g_{l-1}) equals
    mean(g_L) (eq:EgL); injection composes across levels."""
    rng = np.random.default_rng(2)
    m = 11
    g = [rng.uniform(size=(m, 4 << l, 8 << l)) for l in range(4)]
    means = [oracle.level_stats(g[0])[0]] + [oracle.level_stats(g[l], g[l - 1])[0] for l in range(1, 4)]
    E, _ = oracle.mlmc_estimate(means, [np.zeros_like(x) for x in means], [m] * 4)
    np.testing.assert_allclose(E, g[3].mean(axis=0), rtol=1e-13, atol=1e-14)
    np.testing.assert_array_equal(oracle.inject(oracle.inject(g[0][0], 2), 2), oracle.inject(g[0][0], 4))
    qs = [rng.uniform(size=m) for _ in range(4)]
    qm = [oracle.level_stats(qs[0])[0]] + [oracle.level_stats(qs[l], qs[l - 1])[0] for l in range(1, 4)]
    Eq, _ = oracle.mlmc_estimate(qm, [0.0] * 4, [m] * 4)
    assert Eq == pytest.approx(qs[3].mean(), rel=1e-13)


def test_table3_sample_counts():
    """eq:M_ell with ceil reproduces every entry of Table 3 of the paper."""
    lines = [l.split() for l in open(os.path.join(GOLDEN, "table3_mlmc_samples.txt")) if not l.startswith("#")]
    s = [float(x) for x in lines[0][1:]]
    V = [float(x) for x in lines[1][1:]]
    for row in lines[2:]:
        eps2 = float(row[1])
        m, S = oracle.optimal_samples(V, s, eps2)
        assert list(m) == [int(x) for x in row[2:]]
        assert S == pytest.approx(sum(math.sqrt(v * w) for v, w in zip(V, s)) ** 2 / eps2)


# ---------------------------------------------------------------- QMC
def test_radical_inverse_values():
    assert [oracle.radical_inverse(k, 2) for k in range(1, 8)] == [0.5, 0.25, 0.75, 0.125, 0.625, 0.375, 0.875]
    assert oracle.radical_inverse(5, 3) == pytest.approx(2 / 3 + 1 / 9)
    h = oracle.halton(4, 3)
    np.testing.assert_allclose(h[0], [0.5, 1 / 3, 1 / 5])


def test_qmc_mean_agrees_with_mc(phys):
    """E[Q] on 16x8 with 10 steps: a Halton rule (the abstract names QMC as the
    paper's reference) and plain MC must agree within MC error."""
    n = 256
    hal = 2.0 * oracle.halton(n, 3) - 1.0
    mc = oracle.sample_xi(0, 0, 0, n, 3)
    jobs_h = [(16, 8, 10, x) for x in hal]
    jobs_m = [(16, 8, 10, x) for x in mc]
    qh = np.array([r["qoi"] for r in oracle.solve_many(phys, jobs_h)])
    qm = np.array([r["qoi"] for r in oracle.solve_many(phys, jobs_m)])
    sig = qm.std(ddof=1)
    assert abs(qh.mean() - qm.mean()) <= 4 * sig / math.sqrt(n)


# ---------------------------------------------------------------- adjoint
@pytest.mark.parametrize("nx,ny,r", [(8, 4, 10), (16, 8, 20)])
def test_adjoint_tangent_duality(phys, nx, ny, r):
    xi = oracle.sample_xi(0, 0, 3, 1, 3)[0]
    phi, K, q = oracle.fields_closed(phys, nx, ny, xi)
    Q, gphi, gK, gq = oracle.adjoint(phys, r, phi, K, q)
    rng = np.random.default_rng(4)
    vphi = rng.normal(size=phi.shape) * 0.01
    vK = rng.normal(size=K.shape) * 1e-10
    vq = 1e-6
    Q2, dQ = oracle.tangent(phys, r, phi, K, q, vphi, vK, vq)
    assert Q2 == Q
    lhs = (gphi * vphi).sum() + (gK * vK).sum() + gq * vq
    assert abs(lhs - dQ) <= 1e-10 * (abs(dQ) + abs((gphi * vphi)).sum())


def test_adjoint_vs_central_fd_xi(phys):
    nx, ny, r = 16, 8, 20
    xi = oracle.sample_xi(0, 3, 0, 1, 3)[0]
    Q, g, glogk = oracle.adjoint_xi(phys, nx, ny, r, xi)
    hfd = 1e-6
    for d in range(3):
        e = np.zeros(3); e[d] = hfd
        Qp = oracle.solve_xi(phys, nx, ny, r, xi + e)["qoi"]
        Qm = oracle.solve_xi(phys, nx, ny, r, xi - e)["qoi"]
        fd = (Qp - Qm) / (2 * hfd)
        assert abs(fd - g[d]) <= 1e-5 * max(abs(g).max(), 1e-12)
    # a random direction in per-cell log K
    phi, K, q = oracle.fields_closed(phys, nx, ny, xi)
    v = np.random.default_rng(7).normal(size=K.shape)
    Qp = oracle.solve(phys, r, phi, K * np.exp(hfd * v), q)["qoi"]
    Qm = oracle.solve(phys, r, phi, K * np.exp(-hfd * v), q)["qoi"]
    fd = (Qp - Qm) / (2 * hfd)
    assert abs(fd - (glogk * v).sum()) <= 1e-5 * np.abs(glogk * v).sum()
