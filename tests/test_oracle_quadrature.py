"""Pins for the oracle's velocity sets (quadrature requirement of Sec. 2.2,
1-D rule of eq. weight): brute-force monomial exactness against the moments
of the Gaussian weight function, exactness failing one degree higher, and the
1-D rule against numpy's Gauss-HermiteE routine."""

from itertools import product

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

from oracle import quadrature


def gaussian_moment(powers):
    """E[prod z_i^{p_i}] for independent standard normals (brute force from
    the 1-D double factorials)."""
    out = 1.0
    for p in powers:
        if p % 2:
            return 0.0
        out *= np.prod(np.arange(p - 1, 0, -2, dtype=float)) if p > 0 else 1.0
    return out


def max_error_at_degree(vs, degree):
    err = 0.0
    for p in product(range(degree + 1), repeat=vs.D):
        if sum(p) != degree:
            continue
        got = np.sum(vs.w * np.prod(vs.c ** np.array(p)[None, :], axis=1))
        err = max(err, abs(got - gaussian_moment(p)))
    return err


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_1d_rule_matches_library_and_is_exact_to_2n_minus_1(n):
    c, w = quadrature.hermite_rule_1d(n)
    xl, wl = He.hermegauss(n)                      # weight exp(-x^2/2), sum sqrt(2 pi)
    np.testing.assert_allclose(c, xl, rtol=0, atol=1e-13)
    np.testing.assert_allclose(w, wl / np.sqrt(2 * np.pi), rtol=1e-13)
    for k in range(2 * n):
        scale = np.sum(w * np.abs(c) ** k)
        assert abs(np.sum(w * c ** k) - gaussian_moment([k])) < 1e-13 * scale
    assert abs(np.sum(w * c ** (2 * n)) - gaussian_moment([2 * n])) > 1e-3


def test_six_point_rule_is_eleventh_order():
    # Sec. 4 uses an 11th-order set; the 6-point 1-D rule of eq. weight is
    # exact through degree 11.
    c, w = quadrature.hermite_rule_1d(6)
    assert max(abs(np.sum(w * c ** k) - gaussian_moment([k])) / np.sum(w * np.abs(c) ** k)
               for k in range(12)) < 1e-13
    assert abs(np.sum(w * c ** 12) - gaussian_moment([12])) > 1.0


@pytest.mark.parametrize("name,degree", [("D2Q37", 9), ("D3Q39", 7)])
def test_lattice_exact_to_stated_degree_and_not_beyond(name, degree):
    vs = quadrature.velocity_set(name)
    assert np.all(vs.w > 0)
    assert abs(vs.w.sum() - 1.0) < 1e-15
    for k in range(degree + 1):
        scale = max(1.0, max(gaussian_moment([k] + [0] * (vs.D - 1)), 1.0))
        assert max_error_at_degree(vs, k) < 2e-13 * scale, k
    assert max_error_at_degree(vs, degree + 1) > 1e-2


def test_d3q39_weights_are_the_known_rationals(d3q39):
    expected = {(0, 0, 0): 1 / 12, (1, 0, 0): 1 / 12, (1, 1, 1): 1 / 27,
                (2, 0, 0): 2 / 135, (2, 2, 0): 1 / 432, (3, 0, 0): 1 / 1620}
    for e, w in zip(d3q39.e, d3q39.w):
        key = tuple(sorted(np.abs(e).tolist(), reverse=True))
        assert w == pytest.approx(expected[key], rel=1e-15)
    assert d3q39.r ** 2 == pytest.approx(1.5, rel=1e-15)


def test_d2q37_scale_solves_its_degree_eight_conditions(d2q37):
    # Independent check of r: with the weights fixed, the x^8 moment is 105.
    assert np.sum(d2q37.w * d2q37.c[:, 0] ** 8) == pytest.approx(105.0, rel=1e-13)
    assert 1.19 < d2q37.r < 1.20


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_velocity_order_convention(name):
    vs = quadrature.velocity_set(name)
    P = (vs.Q - 1) // 2
    assert np.all(vs.e[0] == 0)
    np.testing.assert_array_equal(vs.e[1:P + 1], -vs.e[P + 1:])
    for v in vs.e[1:P + 1]:
        nz = v[v != 0]
        assert nz[0] > 0
    norms = np.sum(vs.e[1:P + 1] ** 2, axis=1)
    assert np.all(np.diff(norms) >= 0)
    assert len({tuple(v) for v in vs.e}) == vs.Q
    assert np.abs(vs.e).max() == 3
