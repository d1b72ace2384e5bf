"""The oracle's multigrid smoothers and level operators (the relaxations the
GPU solves run in every V-cycle), pinned without retyping them:
  * the pressure operator by hand on a 2x1 grid, its symmetry, and its row
    sums (interior faces cancel; only the seawater faces remain);
  * the transport operator without flow equals the pressure operator of
    its diffusion coefficients plus the accumulation; with flow it keeps
    the row sums acc + boundary terms and couples a cell only to upwind
    neighbours (an M-matrix);
  * red-black Gauss-Seidel by hand on 2x1, and both smoothers converge to
    the sparse direct solution;
  * one x-line sweep on a one-row grid is the exact solve."""
import numpy as np
import scipy.sparse.linalg as spla

import oracle


def rand_pressure(rng, nx, ny):
    return rng.uniform(0.5, 1.5, (ny, nx)), rng.uniform(0.5, 1.5, (ny, nx))


def rand_transport(rng, nx, ny):
    return (rng.uniform(0.1, 1.0, (ny, nx)), rng.uniform(-1, 1, (ny, nx)), rng.uniform(-1, 1, (ny, nx)),
            rng.uniform(0.05, 0.5, (ny, nx)), rng.uniform(0.05, 0.5, (ny, nx)), rng.uniform(-1, 1, ny),
            rng.uniform(0.05, 0.5, ny), rng.uniform(0.05, 0.5, ny), rng.uniform(0.0, 1.0, ny))


def test_pressure_operator_by_hand_and_invariants():
    te = np.array([[2.0, 3.0]])
    tn = np.array([[7.0, 7.0]])  # no face above the only row: unused
    A = oracle.pressure_operator(te, tn).toarray()
    np.testing.assert_array_equal(A, [[2.0, -2.0], [-2.0, 5.0]])
    rng = np.random.default_rng(1)
    te, tn = rand_pressure(rng, 16, 8)
    A = oracle.pressure_operator(te, tn)
    assert abs(A - A.T).max() == 0
    rs = np.asarray(A.sum(axis=1)).ravel().reshape(8, 16)
    want = np.zeros((8, 16))
    want[:, -1] = te[:, -1]
    np.testing.assert_allclose(rs, want, atol=1e-14)


def test_transport_operator_reduces_and_is_upwind():
    rng = np.random.default_rng(2)
    nx, ny = 16, 8
    acc, mx, my, dx, dy, mr, dr, dl, ml = rand_transport(rng, nx, ny)
    z = np.zeros((ny, nx))
    # no flow, no recharge-side terms: diffusion like the pressure operator
    te = dx.copy()
    te[:, -1] = dr
    A = oracle.transport_operator(acc, z, z, dx, dy, np.zeros(ny), dr, np.zeros(ny), np.zeros(ny))
    B = oracle.pressure_operator(te, dy) + __import__("scipy").sparse.diags(acc.ravel())
    assert abs(A - B).max() < 1e-15
    # with flow: row sums are the accumulation plus the boundary terms, and
    # every off-diagonal is <= 0 (M-matrix), nonzero only towards inflow or diffusion
    A = oracle.transport_operator(acc, mx, my, dx, dy, mr, dr, dl, ml).toarray()
    rs = A.sum(axis=1).reshape(ny, nx)
    bnd = np.zeros((ny, nx))
    bnd[:, -1] += np.maximum(-mr, 0) + dr
    bnd[:, 0] += dl + ml
    np.testing.assert_allclose(rs, acc + bnd, atol=1e-13)
    off = A - np.diag(np.diag(A))
    assert (off <= 0).all()
    P, E = 3 * nx + 5, 3 * nx + 6
    assert -A[P, E] == max(-mx[3, 5], 0) + dx[3, 5]
    assert -A[E, P] == max(mx[3, 5], 0) + dx[3, 5]


def test_red_black_gauss_seidel_by_hand():
    te = np.array([[2.0, 3.0]])
    A = oracle.pressure_operator(te, np.zeros((1, 2)))
    b, x0 = np.array([1.0, 4.0]), np.array([0.5, -1.0])
    red = (b[0] + 2.0 * x0[1]) / 2.0
    black = (b[1] + 2.0 * red) / 5.0
    np.testing.assert_allclose(oracle.gauss_seidel_rb(A, b, x0, 2, 1, 1).ravel(), [red, black], rtol=1e-15)


def test_smoothers_converge_to_the_direct_solution():
    rng = np.random.default_rng(3)
    nx, ny = 8, 4  # Dirichlet on one side only: Gauss-Seidel converges slowly
    te, tn = rand_pressure(rng, nx, ny)
    A = oracle.pressure_operator(te, tn)
    b = rng.normal(size=nx * ny)
    xs = spla.spsolve(A.tocsc(), b)
    x = oracle.gauss_seidel_rb(A, b, np.zeros(nx * ny), nx, ny, 2000)
    np.testing.assert_allclose(x.ravel(), xs, rtol=0, atol=1e-8 * np.abs(xs).max())
    nx, ny = 16, 8
    b = rng.normal(size=nx * ny)
    T = oracle.transport_operator(*rand_transport(rng, nx, ny))
    xs = spla.spsolve(T.tocsc(), b)
    for ylines in (False, True):
        x = oracle.zebra_lines(T, b, np.zeros(nx * ny), nx, ny, 60, ylines)
        np.testing.assert_allclose(x.ravel(), xs, rtol=0, atol=1e-10 * np.abs(xs).max())


def test_one_line_sweep_solves_a_one_row_grid():
    rng = np.random.default_rng(4)
    nx, ny = 32, 1
    T = oracle.transport_operator(*rand_transport(rng, nx, ny))
    b = rng.normal(size=nx)
    x = oracle.zebra_lines(T, b, rng.normal(size=nx), nx, ny, 1)
    np.testing.assert_allclose(x.ravel(), spla.spsolve(T.tocsc(), b), rtol=1e-12)
