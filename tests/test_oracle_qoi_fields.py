"""Pins of the oracle's quantity of interest and of its closed-form random
fields, against values worked out by hand (exact trigonometric values,
midpoint sums), not against the oracle's own formulas.

  * The QoI, the salt mass in x < 1 at T (the physical mass of salt per
    metre of depth, h^2 sum over the cells of x < 1 of phi rho(c) c,
    rho(c) = rho0 + (rho1 - rho0) c; Sec. 2.1, e_lin_density): on fields of
    known cell values.  c = 1 everywhere gives phi0 rho1 times the 1 m^2 of
    the left half; c = 1 on the right half only gives 0; c = 1/2 on the left
    half gives phi0 rho(1/2) / 2; c = x gives the midpoint sums
    h sum x_i = 1/2 and h sum x_i^2 = 1/3 - h^2/12 in closed form; a
    porosity linear in y gives its column mean.  A sum over the wrong half,
    a dropped rho(c), a dropped phi or a wrong h power fails one of them.
  * The closed-form fields of the uncertain inputs (Sec. 2.2 in the
    workload's forms: phi = phi0 (1 + 0.2 xi1 cos(pi x/2) cos(pi y)),
    K = k0 exp(0.5 xi2 sin(pi x/2)), q = q_in (1 + 0.2 xi3)) at cell
    centres of a 6 x 3 grid, where x in {1/6, 1/2, 5/6, 7/6, 3/2, 11/6}
    and y in {-5/6, -1/2, -1/6} give exact values: cos(pi/12) =
    (sqrt 6 + sqrt 2)/4, sin(pi/12) = (sqrt 6 - sqrt 2)/4, cos(pi/4) =
    sqrt 2/2, cos(pi/6) = sqrt 3/2, cos(pi/2) = 0.  A swapped sine and
    cosine, a lost half angle or a coefficient attached to the wrong xi
    fails one of them.
"""
import math

import numpy as np
import pytest

import henry_inputs as hi
import oracle

PH = hi.PHYS
PHI0, RHO0, RHO1 = PH["phi0"], PH["rho0"], PH["rho1"]
S2, S3, S6 = math.sqrt(2.0), math.sqrt(3.0), math.sqrt(6.0)


def grid(ny):
    nx = 2 * ny
    h = 1.0 / ny
    x = (np.arange(nx) + 0.5) * h
    y = -1.0 + (np.arange(ny) + 0.5) * h
    return nx, h, np.meshgrid(x, y, indexing="xy")


@pytest.mark.parametrize("ny", [1, 3, 8, 32])
def test_qoi_of_uniform_salt(ny):
    nx, h, (X, Y) = grid(ny)
    phi = np.full((ny, nx), PHI0)
    # c = 1 everywhere: phi0 rho1 over the 1 m^2 of x < 1
    assert oracle.qoi(PH, phi, np.ones((ny, nx))) == pytest.approx(PHI0 * RHO1, rel=1e-14)
    # salt only where x > 1: nothing in the region
    assert oracle.qoi(PH, phi, np.where(X > 1.0, 1.0, 0.0)) == 0.0
    # c = 1/2 where x < 1: phi0 rho(1/2) / 2
    half = np.where(X < 1.0, 0.5, 0.0)
    assert oracle.qoi(PH, phi, half) == pytest.approx(PHI0 * (RHO0 + RHO1) / 2.0 * 0.5, rel=1e-14)


@pytest.mark.parametrize("ny", [1, 3, 8, 32])
def test_qoi_of_salt_linear_in_x(ny):
    """c = x at the cell centres (on the whole domain): per column of height
    1, h sum_{x_i < 1} x_i = 1/2 and h sum x_i^2 = 1/3 - h^2/12 (midpoint
    sums), so Q = phi0 (rho0 / 2 + (rho1 - rho0)(1/3 - h^2/12))."""
    nx, h, (X, Y) = grid(ny)
    phi = np.full((ny, nx), PHI0)
    want = PHI0 * (RHO0 * 0.5 + (RHO1 - RHO0) * (1.0 / 3.0 - h * h / 12.0))
    assert oracle.qoi(PH, phi, X) == pytest.approx(want, rel=1e-13)


def test_qoi_weights_each_cell_by_its_porosity():
    """phi linear in y on the left half (mean over a column 0.25), anything
    on the right half, c = 1: Q = rho1 * 0.25 * 1 m."""
    ny = 8
    nx, h, (X, Y) = grid(ny)
    phi = np.where(X < 1.0, 0.3 + 0.1 * Y, 0.9)
    assert oracle.qoi(PH, phi, np.ones((ny, nx))) == pytest.approx(RHO1 * 0.25, rel=1e-14)


XI = np.array([0.7, 0.4, -1.0])


def test_closed_form_porosity_at_exact_points():
    phi, K, q = oracle.fields_closed(PH, 6, 3, XI)
    a = 0.2 * XI[0]
    # rows j = 0, 1, 2 are y = -5/6, -1/2, -1/6; columns i = 0..5 are x = 1/6, 1/2, .., 11/6
    assert phi[2, 1] == pytest.approx(PHI0 * (1.0 + a * (S2 / 2) * (S3 / 2)), rel=1e-14)   # x 1/2, y -1/6
    assert phi[0, 4] == pytest.approx(PHI0 * (1.0 + a * (-S2 / 2) * (-S3 / 2)), rel=1e-14)  # x 3/2, y -5/6
    assert phi[2, 0] == pytest.approx(PHI0 * (1.0 + a * (S6 + S2) / 4 * (S3 / 2)), rel=1e-14)  # x 1/6
    assert phi[0, 5] == pytest.approx(PHI0 * (1.0 + a * (-(S6 + S2) / 4) * (-S3 / 2)), rel=1e-14)  # x 11/6
    # y = -1/2: cos(-pi/2) = 0, the porosity is phi0 along the whole row
    assert np.allclose(phi[1], PHI0, rtol=1e-15, atol=0.0)


def test_closed_form_permeability_and_recharge_at_exact_points():
    phi, K, q = oracle.fields_closed(PH, 6, 3, XI)
    b = 0.5 * XI[1]
    sin_x = [(S6 - S2) / 4, S2 / 2, (S6 + S2) / 4, (S6 + S2) / 4, S2 / 2, (S6 - S2) / 4]  # sin(pi x / 2)
    for i, s in enumerate(sin_x):
        assert np.allclose(K[:, i], PH["k0"] * math.exp(b * s), rtol=1e-14, atol=0.0), i
    assert q == pytest.approx(PH["q_in"] * 0.8, rel=1e-15)


def test_each_field_follows_its_own_coefficient():
    phi, K, q = oracle.fields_closed(PH, 16, 8, [0.7, 0.0, 0.0])
    assert np.all(K == PH["k0"]) and q == PH["q_in"]
    phi, K, q = oracle.fields_closed(PH, 16, 8, [0.0, 0.4, 0.0])
    assert np.all(phi == PHI0) and q == PH["q_in"]
    phi, K, q = oracle.fields_closed(PH, 16, 8, [0.0, 0.0, 1.0])
    assert np.all(phi == PHI0) and np.all(K == PH["k0"]) and q == pytest.approx(1.2 * PH["q_in"], rel=1e-15)
