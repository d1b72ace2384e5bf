"""The paper's own random input model in the oracle (Sec. 4:
eq:poro_2levels, eq:poro_2levels_C; Sec. 2.2: e_perm_Kozeny_Carman; the
recharge with a +-50 % amplitude) and its derivatives, pinned without
retyping the formulas:
  * at xi = 0 the model is the homogeneous medium, the closed-form fields'
    value at xi = 0 (a different function);
  * with xi2 = 0 the porosity of two cells of one column on either side of
    y = -0.75 differs exactly by the layer factor (1 + 0.2 xi1) / (1 - 0.2 xi1),
    and the lower layer holds the bottom quarter of the rows;
  * Fig. 2's printed maximum over the domain at xi* (tests/golden);
  * the recharge's +-50 % range;
  * the stated bounds of phi over random xi;
  * the xi-derivatives against central differences of the fields, and the
    oracle's dQ/dxi through them against central differences of Q."""
import os

import numpy as np
import pytest

import henry_inputs as hi
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PH = hi.PHYS_TABLE1


def test_zero_xi_is_the_homogeneous_medium():
    phi, K, q = oracle.fields_two_layer(PH, 32, 16, [0.0, 0.0, 0.0])
    phc, Kc, qc = oracle.fields_closed(PH, 32, 16, np.zeros(3))
    np.testing.assert_array_equal(phi, phc)
    np.testing.assert_allclose(K, Kc, rtol=4e-16)
    assert q == qc == PH["q_in"]


@pytest.mark.parametrize("ny", [4, 8, 64])
def test_layer_factor_across_the_split(ny):
    nx = 2 * ny
    x1 = 0.6
    phi, _, _ = oracle.fields_two_layer(PH, nx, ny, [x1, 0.0, 0.0])
    jb = ny // 4  # rows 0 .. ny/4 - 1 have centres below y = -0.75
    ratio = phi[jb - 1] / phi[jb]
    np.testing.assert_allclose(ratio, (1 + 0.2 * x1) / (1 - 0.2 * x1), rtol=1e-15)
    # within a layer, with xi2 = 0, the porosity does not depend on y
    np.testing.assert_array_equal(phi[:jb], np.broadcast_to(phi[0], (jb, nx)))
    np.testing.assert_array_equal(phi[jb:], np.broadcast_to(phi[jb], (ny - jb, nx)))


def test_fig2_maximum():
    rows = {l.split()[0]: l.split()[1:] for l in open(os.path.join(ROOT, "tests", "golden", "fig2_porosity_range.txt"))
            if not l.startswith("#")}
    xi = [float(v) for v in rows["xi"]]
    phi, _, _ = oracle.fields_two_layer(PH, 2048, 1024, xi)
    assert round(phi.max(), 3) == float(rows["max"][0])


def test_recharge_amplitude():
    for x3, f in ((1.0, 1.5), (-1.0, 0.5), (0.0, 1.0)):
        assert oracle.fields_two_layer(PH, 4, 2, [0.0, 0.0, x3])[2] == pytest.approx(f * PH["q_in"], rel=1e-15)


def test_porosity_bounds_and_positive_permeability():
    rng = np.random.default_rng(8)
    lo, hi_ = np.inf, -np.inf
    for xi in rng.uniform(-1, 1, (200, 3)):
        phi, K, _ = oracle.fields_two_layer(PH, 64, 32, xi)
        lo, hi_ = min(lo, phi.min()), max(hi_, phi.max())
        assert (K > 0).all() and np.isfinite(K).all()
    assert 0.44 * PH["phi0"] <= lo and hi_ <= 1.74 * PH["phi0"]
    # the corner values: all terms aligned
    phi, _, _ = oracle.fields_two_layer(PH, 2048, 1024, [1.0, 1.0, 0.0])
    assert phi.max() == pytest.approx(1.74 * PH["phi0"], rel=1e-3)


def test_field_derivatives_against_central_differences():
    xi = np.array([0.3, -0.7, 0.2])
    dphi, dK, dq = oracle.field_derivs_two_layer(PH, 16, 8, xi)
    for k in range(2):
        e = np.zeros(3)
        e[k] = 1e-6
        pp, Kp, _ = oracle.fields_two_layer(PH, 16, 8, xi + e)
        pm, Km, _ = oracle.fields_two_layer(PH, 16, 8, xi - e)
        np.testing.assert_allclose(dphi[k], (pp - pm) / 2e-6, rtol=1e-7, atol=1e-12)
        np.testing.assert_allclose(dK[k], (Kp - Km) / 2e-6, rtol=1e-7, atol=1e-22)
    qp = oracle.fields_two_layer(PH, 16, 8, xi + [0, 0, 1e-6])[2]
    qm = oracle.fields_two_layer(PH, 16, 8, xi - [0, 0, 1e-6])[2]
    assert dq == pytest.approx((qp - qm) / 2e-6, rel=1e-8)


def test_adjoint_gradient_against_central_differences():
    xi = np.array([-0.5898, -0.7257, -0.9616])
    nx, ny, r = 8, 4, 12
    Q, g, _ = oracle.adjoint_xi(PH, nx, ny, r, xi, model="two_layer")
    assert Q == pytest.approx(oracle.solve_xi(PH, nx, ny, r, xi, model="two_layer")["qoi"], rel=1e-14)
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1e-5
        qp = oracle.solve_xi(PH, nx, ny, r, xi + e, model="two_layer")["qoi"]
        qm = oracle.solve_xi(PH, nx, ny, r, xi - e, model="two_layer")["qoi"]
        assert g[k] == pytest.approx((qp - qm) / 2e-5, rel=1e-5), k


def test_paper_hierarchy_matches_table2():
    """The paper's hierarchy (henry_inputs.paper_level_grid with T = 6016 s)
    against Table 2: level l has 32 2^l x 16 2^l cells, i.e. the paper's
    quadrilaterals, whose (nx + 1)(ny + 1) vertices carry two unknowns each
    (n_l), r_l steps and tau_l = T / r_l."""
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    rows = [l.split() for l in open(os.path.join(root, "tests", "golden", "table2_hierarchy.txt"))
            if not l.startswith("#")]
    for lev, n, r, tau, _ in rows:
        nx, ny, steps = hi.paper_level_grid(int(lev))
        assert 2 * (nx + 1) * (ny + 1) == int(n)
        assert steps == int(r)
        assert PH["T"] / steps == float(tau)
    assert PH["T"] == 6016.0
