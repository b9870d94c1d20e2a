"""Pins for the oracle of the paper's scheme on its 3-D set D3Q216 (the
tensor cube of the 6-point Gauss-Hermite rule; the paper's validation runs
use D = 3):

* The set integrates every monomial c_x^p c_y^q c_z^r with p, q, r <= 11
  exactly against the Gaussian weight and not p = 12; opposites at a + 108.
* Collision and flux form conserve mass, momentum and energy on a periodic
  grid; a uniform body force adds exactly dt rho g of momentum per step.
* A gas at rest at the walls' temperature is a fixed point; a flow uniform
  in x and y stays uniform; a channel mirror-symmetric in z stays symmetric.
* Quasi-steady Couette flow across z (the paper's 1-D setting) has an
  antisymmetric velocity, uniform shear stress and wall slip.
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import offlattice as O


@pytest.fixture(scope="module")
def gh3():
    return O.ProductSet(6, 3, 4)


def _gauss_moment(p):
    return 0.0 if p % 2 else float(np.prod(np.arange(p - 1, 0, -2))) if p else 1.0


def test_cube_set_exact_to_degree_eleven(gh3):
    assert gh3.Q == 216 and gh3.P == 108
    np.testing.assert_array_equal(gh3.c[108:], -gh3.c[:108])
    c, w = gh3.c, gh3.w
    for p in range(12):
        for q in range(12):
            for r in range(0, 12, 1):
                terms = w * c[:, 0] ** p * c[:, 1] ** q * c[:, 2] ** r
                exact = _gauss_moment(p) * _gauss_moment(q) * _gauss_moment(r)
                assert abs(terms.sum() - exact) < 1e-12 * np.abs(terms).sum()
    assert abs(np.sum(w * c[:, 2] ** 12) - _gauss_moment(12)) > 1.0


def _totals(f, prob):
    rho, u, T, s, q = O.macroscopic(f, prob)
    return np.array([rho.sum(), *(rho[:, None] * u).sum(0), (rho * (3 * T + (u ** 2).sum(1))).sum()])


def test_periodic_step_conserves_and_forces(gh3):
    rng = np.random.default_rng(41)
    g = (0.01, -0.005, 0.002)
    prob = O.TVDProblem(gh3, (4, 3, 5), Kn=0.05, Pr=2 / 3, g=g, cfl=0.5, n_ref=5)
    M = prob.M
    f = O.equilibrium_state(prob, 1 + 0.02 * rng.uniform(-1, 1, M), 0.02 * rng.uniform(-1, 1, (M, 3)),
                            1 + 0.02 * rng.uniform(-1, 1, M)) * (1 + 0.01 * rng.standard_normal((216, M)))
    t0 = _totals(f, prob)
    f1 = O.step(f, prob)
    t1 = _totals(f1, prob)
    assert abs(t1[0] - t0[0]) < 1e-12 * t0[0]
    np.testing.assert_allclose(t1[1:4] - t0[1:4], prob.dt * t0[0] * np.array(g), rtol=1e-10, atol=1e-14)
    # without the force, energy is conserved too
    prob0 = O.TVDProblem(gh3, (4, 3, 5), Kn=0.05, Pr=2 / 3, cfl=0.5, n_ref=5)
    f2 = O.run(f, prob0, 3)
    np.testing.assert_allclose(_totals(f2, prob0), t0, rtol=1e-12, atol=1e-13)


def _channel(gh3, dims, T=(1.0, 1.0), u=((0, 0, 0), (0, 0, 0)), Kn=0.1):
    return O.TVDProblem(gh3, dims, Kn=Kn, Pr=2 / 3, cfl=0.8, walls=True,
                        wall_lo=L.Wall(T[0], tuple(u[0])), wall_hi=L.Wall(T[1], tuple(u[1])))


def test_rest_fixed_point_and_xy_uniform_flow(gh3):
    prob = _channel(gh3, (2, 2, 7), T=(1.05, 1.05))
    M = prob.M
    f0 = O.equilibrium_state(prob, np.ones(M), np.zeros((M, 3)), np.full(M, 1.05))
    np.testing.assert_allclose(O.run(f0, prob, 3), f0, rtol=1e-14, atol=0)
    # moving walls, a start uniform in x and y: every (x, y) column stays equal
    prob = _channel(gh3, (3, 2, 7), T=(0.97, 1.04), u=((-0.05, 0.02, 0), (0.04, 0, 0)))
    rng = np.random.default_rng(42)
    col = O.equilibrium_state(_channel(gh3, (1, 1, 7)), np.ones(7), np.zeros((7, 3)), np.ones(7))
    col = col * (1 + 0.01 * rng.standard_normal(col.shape))
    f = np.repeat(col[:, :, None], prob.dims[0] * prob.dims[1], axis=2).reshape(216, -1)
    f = O.run(f, prob, 4)
    g = prob.grid(f)                                  # (Q, nz, ny, nx)
    # equal up to the rounding of numpy's blocked products across columns
    np.testing.assert_allclose(g, np.broadcast_to(g[:, :, :1, :1], g.shape), rtol=1e-14, atol=0)


def test_mirror_symmetric_channel_stays_symmetric(gh3):
    rng = np.random.default_rng(43)
    prob = _channel(gh3, (1, 1, 9), T=(1.03, 1.03))
    mirror = np.array([int(np.flatnonzero((gh3.c[:, 0] == c[0]) & (gh3.c[:, 1] == c[1]) & (gh3.c[:, 2] == -c[2]))[0])
                       for c in gh3.c])
    M = prob.M
    f = O.equilibrium_state(prob, np.ones(M), np.zeros((M, 3)), np.ones(M)) * rng.uniform(0.95, 1.05, (216, M))
    f = 0.5 * (f + f[mirror][:, ::-1])
    f = O.run(f, prob, 5)
    np.testing.assert_allclose(f, f[mirror][:, ::-1], rtol=1e-13, atol=1e-17)


@pytest.mark.slow
def test_couette_across_z(gh3):
    prob = _channel(gh3, (1, 1, 11), u=((-0.05, 0, 0), (0.05, 0, 0)), Kn=0.2)
    M = prob.M
    f = O.equilibrium_state(prob, np.ones(M), np.zeros((M, 3)), np.ones(M))
    f = O.run(f, prob, 600)
    rho, u, T, sigma, q = O.macroscopic(f, prob)
    ux = u[:, 0]
    np.testing.assert_allclose(ux, -ux[::-1], atol=1e-14)
    assert np.all(np.diff(ux) > 0)
    sxz = sigma[1:-1, 0, 2]
    np.testing.assert_allclose(sxz, sxz.mean(), rtol=0.03)
    assert sxz.mean() < 0
    assert 0 < 0.05 - ux[-1] < 0.05
