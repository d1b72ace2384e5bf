"""The oracle's time-series functions (Sec. 4: eq:integral_fw, the points of
eq:12points, the quantiles of Figs. 4 and 6, the first-passage times of
Figs. 5 and 7), pinned without retyping them:
  * the fresh-water area is the area of D (2) for c = 0, 0 for c = 1, and a
    counted multiple of h^2 on a field with a known number of fresh cells;
  * point values on a field with known cell values: inside a cell, on a
    vertical and a horizontal face, at a corner, on the boundary, and the
    paper's 12 points on 32x16 (rows y = -0.75 and -0.5 lie on faces);
  * record steps: the last record is the last step, records are strictly
    increasing, and nrec = nsteps takes every step;
  * type-7 quantiles against numpy's "linear" method and the order
    statistics they must return at p = 0, 1 and on exact grid points;
  * first-passage times by hand on short series;
  * a trace's last record equals the fresh area and point values of the
    solve's final state."""
import numpy as np
import pytest

import henry_inputs as hi
import oracle

PTS12 = [(1.10, -0.95), (1.35, -0.95), (1.60, -0.95), (1.85, -0.95), (1.10, -0.75), (1.35, -0.75),
         (1.60, -0.75), (1.85, -0.75), (1.10, -0.50), (1.35, -0.50), (1.60, -0.50), (1.85, -0.50)]


def test_fresh_area():
    assert oracle.fresh_area(np.zeros((16, 32))) == 2.0
    assert oracle.fresh_area(np.ones((16, 32))) == 0.0
    c = np.ones((8, 16))
    c[0, :5] = 0.0
    c[3, 7] = oracle.FRESH  # on the threshold: fresh
    c[4, 7] = np.nextafter(oracle.FRESH, 1.0)
    assert oracle.fresh_area(c) == 6 / 64


def test_point_values_on_a_known_field():
    ny, nx = 8, 16
    c = np.add.outer(100.0 * np.arange(ny), np.arange(nx))  # c[j, i] = i + 100 j
    h = 1.0 / ny
    assert oracle.point_value(c, 1.3, -0.9) == 10 + 0  # u = 10.4, v = 0.8
    assert oracle.point_value(c, 1.0, -0.9) == 7.5  # the face x = 1 between columns 7 and 8
    assert oracle.point_value(c, 1.3, -0.5) == 10 + 350  # the face y = -0.5 between rows 3 and 4
    assert oracle.point_value(c, 1.0, -0.5) == 7.5 + 350  # a corner of four
    assert oracle.point_value(c, 0.0, -1.0) == 0.0  # the domain's corner: one cell
    assert oracle.point_value(c, 2.0, 0.0) == 15 + 700
    assert oracle.point_value(c, 2.0, -1.0 + 3 * h) == 15 + 250
    # the paper's 12 points on 32 x 16: rows y = -0.75 and -0.5 take two rows of cells
    ny, nx = 16, 32
    c = np.add.outer(100.0 * np.arange(ny), np.arange(nx))
    got = [oracle.point_value(c, x, y) for x, y in PTS12]
    cols = [17, 21, 25, 29]  # floor(x * 16) for x = 1.10, 1.35, 1.60, 1.85
    want = [cc + 0 for cc in cols] + [cc + 350 for cc in cols] + [cc + 750 for cc in cols]
    assert got == want


def test_record_steps():
    for n, r in ((50, 10), (50, 7), (188, 48), (188, 188), (3, 1)):
        st = oracle.record_steps(n, r)
        assert len(st) == r and st[-1] == n and all(b > a for a, b in zip(st, st[1:]))
        for k, s in enumerate(st, start=1):
            assert (s - 1) * r < k * n <= s * r  # the first step at or after k T / nrec
    assert oracle.record_steps(188, 188) == list(range(1, 189))


def test_quantile7():
    rng = np.random.default_rng(5)
    for n in (1, 2, 3, 10, 600):
        x = rng.normal(size=n)
        for p in (0.0, 0.025, 0.25, 0.5, 0.75, 0.975, 1.0):
            assert oracle.quantile7(x, p) == pytest.approx(np.quantile(x, p, method="linear"), abs=1e-15)
        assert oracle.quantile7(x, 0.0) == x.min() and oracle.quantile7(x, 1.0) == x.max()
    x = np.array([4.0, 1.0, 3.0, 2.0, 5.0])
    assert oracle.quantile7(x, 0.5) == 3.0 and oracle.quantile7(x, 0.25) == 2.0
    assert oracle.quantile7(x, 0.125) == 1.5
    assert oracle.quantile7(np.array([2.0, 2.0, 2.0]), 0.3) == 2.0


def test_first_passage():
    s = [2.0, 1.9, 1.6, 1.3, 1.1, 1.0]
    assert oracle.first_passage(s, 1.7) == 3
    assert oracle.first_passage(s, 1.2) == 5
    assert oracle.first_passage(s, 0.5) == 0
    assert oracle.first_passage(s, 1.6) == 4  # strictly below
    assert oracle.first_passage([0.1, 0.5, 0.95, 0.99], 0.9, below=False) == 3


def test_trace_last_record_is_the_final_state():
    phi, K, q = oracle.fields_two_layer(hi.PHYS_TABLE1, 16, 8, [0.3, -0.4, 0.5])
    tr, out = oracle.trace(hi.PHYS_TABLE1, 20, phi, K, q, 6, PTS12)
    assert tr.shape == (6, 13)
    assert tr[-1, 0] == oracle.fresh_area(out["c"])
    assert list(tr[-1, 1:]) == [oracle.point_value(out["c"], x, y) for x, y in PTS12]
    assert tr[0, 0] <= 2.0 and (tr[:, 1:] >= -1e-12).all() and (tr[:, 1:] <= 1 + 1e-12).all()
