"""Pins for the diffuse walls of the paper's own scheme (Sec. 3.2, the first
version of the boundary conditions of Sofonea et al.): wall nodes on the
walls, ghost nodes that copy them, and re-emission of the wall node's
populations that move into the gas as rho_W S(T_W, u_W).

* A gas at rest in equilibrium at the walls' temperature is a fixed point.
* The ghost copies make the wall faces first-order upwind: a unit value on
  the wall node flows into the first node at exactly |nu| per step (the
  ghosts refill the wall node) or, moving toward the wall, out through it;
  a unit value on the first node flows into the wall node at exactly |nu|.
* After a step the wall emits, column by column, the normal particle flux
  that the first interior node sends toward it, with the shape of
  S(T_W, u_W).
* The walls are mirror images: a mirror-symmetric channel stays symmetric.
* Steady Couette flow has an antisymmetric velocity, a uniform shear
  stress and a slip at the walls that grows with Kn; steady heat conduction
  has a uniform heat flux and temperature jumps at the walls.
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import model
from oracle import offlattice as O


@pytest.fixture(scope="module")
def gh():
    return O.ProductSet(6, 2, 4)


def _channel(gh, dims, T=(1.0, 1.0), uw=(0.0, 0.0), Kn=0.1, Pr=2 / 3, cfl=0.8, g=(0.0, 0.0, 0.0)):
    return O.TVDProblem(gh, dims, Kn=Kn, Pr=Pr, cfl=cfl, g=g, walls=True,
                        wall_lo=L.Wall(T[0], (uw[0], 0.0, 0.0)), wall_hi=L.Wall(T[1], (uw[1], 0.0, 0.0)))


def _rest(prob, T=1.0):
    M = prob.M
    return O.equilibrium_state(prob, np.ones(M), np.zeros((M, 2)), np.full(M, T))


def test_rest_at_wall_temperature_is_a_fixed_point(gh):
    prob = _channel(gh, (3, 9), T=(1.1, 1.1))
    f0 = _rest(prob, 1.1)
    f = O.run(f0, prob, 5)
    np.testing.assert_allclose(f, f0, rtol=1e-14, atol=0)


def test_wall_face_is_first_order_upwind(gh):
    prob = _channel(gh, (1, 8))
    ny = prob.dims[-1]
    for a in range(gh.Q):
        nu = gh.c[a, 1] * prob.dt / prob.dx
        for side, j_wall, j_in in ((0, 0, 1), (1, ny - 1, ny - 2)):
            into_gas = nu > 0 if side == 0 else nu < 0
            # unit value on the wall node: if the velocity points into the
            # gas it flows into the first node at |nu| while the ghost copies
            # refill the wall node; otherwise it leaves through the wall at
            # |nu| and the first node sees nothing
            f = np.zeros((gh.Q, prob.M))
            f[a, j_wall] = 1.0
            adv = O.advection(f, prob)
            expect = np.zeros(prob.M)                   # f_new = f - adv
            if into_gas:
                expect[j_in] = -abs(nu)
            else:
                expect[j_wall] = abs(nu)
            np.testing.assert_allclose(adv[a], expect, rtol=1e-14, atol=1e-16)
            # unit value on the first node moving toward the wall: the wall
            # node gains |nu| (its ghost copies keep the face upwind)
            f = np.zeros((gh.Q, prob.M))
            f[a, j_in] = 1.0
            adv = O.advection(f, prob)
            if not into_gas:
                assert adv[a, j_wall] == pytest.approx(-abs(nu), rel=1e-14)
                assert adv[a, j_in] == pytest.approx(abs(nu), rel=1e-14)


def test_wall_emits_the_incoming_flux_with_the_wall_maxwellian(gh):
    rng = np.random.default_rng(31)
    T, uw = (0.95, 1.08), (-0.04, 0.06)
    prob = _channel(gh, (6, 10), T=T, uw=uw)
    f = _rest(prob) * rng.uniform(0.9, 1.1, (gh.Q, prob.M))
    f1 = O.step(f, prob)
    g1 = prob.grid(f1)
    ny = prob.dims[-1]
    for side, jw, ji in ((0, 0, 1), (1, ny - 1, ny - 2)):
        # the wall's Maxwellian from its own temperature and speed (eq. feq0)
        S = model.truncated_maxwellian(np.ones(1), np.array([[uw[side], 0.0]]), np.array([T[side]]),
                                       gh.c, gh.w, gh.N)[:, 0]
        cn = gh.c[:, 1] if side == 0 else -gh.c[:, 1]          # inward normal
        out, inc = cn > 0, cn < 0
        emitted = cn[out] @ g1[out, jw]
        arriving = np.abs(cn[inc]) @ g1[inc, ji]
        np.testing.assert_allclose(emitted, arriving, rtol=1e-14)
        # the emitted populations are S(T_W, u_W) times one density per column
        ratio = g1[out, jw] / S[out][:, None]
        np.testing.assert_allclose(ratio, np.broadcast_to(ratio[:1], ratio.shape), rtol=1e-13)


def test_mirror_symmetric_channel_stays_symmetric(gh):
    rng = np.random.default_rng(32)
    prob = _channel(gh, (4, 11), T=(1.05, 1.05), Kn=0.05)
    ny = prob.dims[-1]
    # mirror in y: velocity (cx, cy) -> (cx, -cy), node j -> ny - 1 - j
    mirror = np.array([int(np.flatnonzero((gh.c[:, 0] == c[0]) & (gh.c[:, 1] == -c[1]))[0]) for c in gh.c])
    f = _rest(prob) * rng.uniform(0.95, 1.05, (gh.Q, prob.M))
    g = prob.grid(f)
    g = 0.5 * (g + g[mirror][:, ::-1, :])
    f = g.reshape(f.shape)
    f = O.run(f, prob, 6)
    g = prob.grid(f)
    np.testing.assert_allclose(g, g[mirror][:, ::-1, :], rtol=1e-13, atol=1e-17)


@pytest.mark.slow
def test_couette_quasi_steady_state(gh):
    # the scheme drains a little mass at walls with a shear flow beside
    # them, so the profiles are taken once they have settled (1000 steps,
    # about twenty viscous times of the 13-node channel)
    slips = []
    for Kn in (0.1, 0.3):
        prob = _channel(gh, (1, 13), uw=(-0.05, 0.05), Kn=Kn, cfl=0.9)
        f = O.run(_rest(prob), prob, 1000)
        rho, u, T, sigma, q = O.macroscopic(f, prob)
        ux = u[:, 0]
        np.testing.assert_allclose(ux, -ux[::-1], atol=1e-14)
        assert np.all(np.diff(ux) > 0)
        sxy = sigma[1:-1, 0, 1]
        np.testing.assert_allclose(sxy, sxy.mean(), rtol=0.03)
        assert sxy.mean() < 0                      # momentum flows from the upper wall down
        assert abs(rho.sum() / prob.M - 1) < 1e-3
        slips.append(0.05 - ux[-1])
    assert 0 < slips[0] < slips[1]


@pytest.mark.slow
def test_heat_conduction_quasi_steady_state(gh):
    prob = _channel(gh, (1, 13), T=(1.0, 1.1), Kn=0.1, cfl=0.9)
    f = O.run(_rest(prob, 1.05), prob, 1000)
    rho, u, T, sigma, q = O.macroscopic(f, prob)
    qy = q[1:-1, 1]
    np.testing.assert_allclose(qy, qy.mean(), rtol=0.03)
    assert qy.mean() < 0                           # heat flows from the hot upper wall down
    assert np.all(np.diff(T) > 0)
    assert 1.0 < T[0] and T[-1] < 1.1              # temperature jumps at both walls
    np.testing.assert_allclose(u[:, 0], 0.0, atol=1e-14)
    # the wall treatment is not exactly conservative: a normal drift of a
    # few 1e-3 thermal speeds remains (it does not change over the run)
    assert np.abs(u[:, 1]).max() < 3e-3
