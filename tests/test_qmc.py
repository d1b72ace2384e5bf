"""Quasi-Monte Carlo points (the reference of the abstract and of Sec. 4,
Fig. 11; the paper's set-up names Halton points).

Pins of the oracle's rule that do not retype it: the stratification of a
van der Corput sequence (its first b^m points are exactly the grid
{j / b^m}), its digit recurrence phi_b(b k + d) = (d + phi_b(k)) / b, the
prime base of every coordinate, and what a Cranley-Patterson rotation keeps
(one point per interval of length b^-m, shifted by the rotation).  The
library's henry_qmc_points (host code, no GPU) is checked against the oracle
within rounding and against the exact rationals of the digit reversal, of
which it must take the correctly rounded value before the map 2u - 1."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import paper_2302_07804_amd as hm

PRIMES = [2, 3, 5, 7, 11, 13]


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(hm.LIB_PATH):
        pytest.fail("libhenry.so is not built (run __graft_entry__.build())")
    return hm.lib()


# ---------------------------------------------------------------- oracle pins
@pytest.mark.parametrize("b,m", [(2, 10), (3, 6), (5, 4), (7, 3), (13, 2)])
def test_van_der_corput_is_stratified(b, m):
    n = b ** m
    u = np.array([oracle.radical_inverse(k, b) for k in range(n)])
    scaled = u * n
    assert np.allclose(scaled, np.round(scaled), atol=1e-9)
    assert sorted(np.round(scaled).astype(int)) == list(range(n))


@pytest.mark.parametrize("b", [2, 3, 5, 7])
def test_van_der_corput_digit_recurrence(b):
    for k in range(0, 300):
        for d in range(b):
            assert oracle.radical_inverse(b * k + d, b) == pytest.approx((d + oracle.radical_inverse(k, b)) / b,
                                                                      abs=1e-15)


def test_halton_coordinates_use_successive_primes():
    for dim in (1, 3, 6):
        h = oracle.halton(2 * 3 * 5 * 7 * 11 * 13, dim, skip=0)
        for d in range(dim):
            b = PRIMES[d]
            m = int(math.log(h.shape[0], b))
            col = h[: b ** m, d] * b ** m
            assert sorted(np.round(col).astype(int)) == list(range(b ** m)), (dim, d)


def test_shifted_rule_keeps_one_point_per_interval():
    shift = np.array([0.3141, 0.2718, 0.6931])
    n = 3 ** 5
    xi = oracle.qmc_xi(n, 3, skip=0, shift=shift)
    assert xi.min() >= -1.0 and xi.max() < 1.0
    u = (xi[:, 1] + 1.0) / 2.0  # base-3 coordinate
    # each point of the rotated grid {frac(j / n + s)}: one per interval
    g = np.mod(u - shift[1], 1.0) * n
    assert np.allclose(g, np.round(g), atol=1e-8)
    assert sorted(np.mod(np.round(g).astype(int), n)) == list(range(n))
    # with no shift the map is 2u - 1 of the plain Halton points
    assert np.array_equal(oracle.qmc_xi(8, 3), 2.0 * oracle.halton(8, 3) - 1.0)


# ---------------------------------------------------------------- library
def _exact(k, b):
    num, den = 0, 1
    while k > 0:
        num, den, k = num * b + k % b, den * b, k // b
    return Fraction(num, den)


def test_library_points_match_oracle(L):
    for first, n in ((1, 512), (0, 7), (1000, 300), (123456, 64)):
        got = hm.henry_qmc_points(first, n, 3)
        ref = oracle.qmc_xi(n, 3, skip=first)
        np.testing.assert_allclose(got, ref, rtol=0, atol=2e-15)
    rng = np.random.default_rng(3)
    for _ in range(5):
        sh = rng.random(3)
        np.testing.assert_allclose(hm.henry_qmc_points(1, 400, 3, sh), oracle.qmc_xi(400, 3, 1, sh), rtol=0,
                                   atol=4e-15)


def test_library_points_are_correctly_rounded(L):
    for dim in (3, 16):
        pts = hm.henry_qmc_points(1, 200, dim)
        primes = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53][:dim]
        for k in range(200):
            for d, b in enumerate(primes):
                assert pts[k, d] == 2.0 * float(_exact(k + 1, b)) - 1.0, (k, d)
    # large indices, near the documented limit
    first = 2 ** 31 - 5
    pts = hm.henry_qmc_points(first, 5, 3)
    for k in range(5):
        for d, b in enumerate((2, 3, 5)):
            assert pts[k, d] == 2.0 * float(_exact(first + k, b)) - 1.0


def test_library_points_reject_bad_arguments(L):
    ok = hm.henry_qmc_points(1, 0, 3)
    assert ok.shape == (0, 3)
    for first, count, dim in ((-1, 4, 3), (1, -1, 3), (1, 4, 0), (1, 4, 17), (2 ** 31 - 2, 4, 3)):
        with pytest.raises(hm.HenryError):
            hm.henry_qmc_points(first, count, dim)
    for bad in ([1.0, 0.0, 0.0], [-0.1, 0.0, 0.0], [float("nan"), 0.0, 0.0]):
        with pytest.raises(hm.HenryError):
            hm.henry_qmc_points(1, 4, 3, bad)


def test_point_cell():
    for nx in (16, 32, 256, 512):
        ny = nx // 2
        h = 1.0 / ny
        for x, y in ((1.60, -0.95), (1.35, -0.95), (0.01, -0.99), (1.99, -0.01)):
            k = hm.point_cell((nx, ny, 1), x, y)
            i, j = k % nx, k // nx
            assert i * h < x < (i + 1) * h and -1 + j * h < y < -1 + (j + 1) * h
    with pytest.raises(ValueError):
        hm.point_cell((16, 8, 1), 1.0, -0.5)  # a face at every level
    with pytest.raises(ValueError):
        hm.point_cell((256, 128, 1), 1.10, -0.75)  # y = -0.75 is a face for ny >= 4
    with pytest.raises(ValueError):
        hm.point_cell((16, 8, 1), 2.5, -0.5)
