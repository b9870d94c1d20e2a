"""Pins for the oracle's unsteady boundary heating (Sec. 4.2): wall
temperatures T_W(t) = T + A sin(theta t), with t in units of L/sqrt(R T0).

* The step from stored level n to n + 1 re-emits S(T_W((n + 1/2) dt), u_W).
* No amplitude reproduces the static wall exactly.
* Heating both walls alike keeps the mirror symmetry of the channel (u_y
  odd, T and rho even, u_x zero) and conserves mass.
* Small amplitudes give a linear response, as the paper assumes: doubling A
  doubles the deviation from rest up to O(A^2).
* Heating first warms the gas at the walls and adds energy; cooling removes
  it.
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import model
from oracle import quadrature


def _channel(name, A, theta=np.pi / 2, ny=12, T=1.0):
    vs = quadrature.velocity_set(name)
    dims = (1, ny) if vs.D == 2 else (1, 1, ny)
    wall = L.Wall(T, (0.0, 0.0, 0.0), 1.0, A, theta)
    return L.Problem(vs, dims, Kn=0.1, Pr=2 / 3, walls=True, wall_lo=wall, wall_hi=wall)


def _rest(prob):
    M = prob.M
    return L.equilibrium_state(prob, np.ones(M), np.zeros((M, prob.D)), np.ones(M))


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_emission_uses_the_midpoint_wall_temperature(name):
    prob = _channel(name, 0.01, theta=2.0)
    for n in (0, 3, 17):
        t = (n + 0.5) * prob.dt
        Tw = 1.0 + 0.01 * np.sin(2.0 * t)
        expect = model.truncated_maxwellian(np.ones(1), np.zeros((1, prob.D)), np.array([Tw]),
                                            prob.vs.c, prob.vs.w, prob.N)[:, 0]
        lo, hi = prob.wall_emission(n)
        np.testing.assert_allclose(lo, expect, rtol=1e-15, atol=0)
        np.testing.assert_allclose(hi, expect, rtol=1e-15, atol=0)


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_zero_amplitude_is_the_static_wall(name):
    heated = _channel(name, 0.0, theta=3.0, T=1.02)
    static = L.Problem(heated.vs, heated.dims, Kn=0.1, Pr=2 / 3, walls=True,
                       wall_lo=L.Wall(1.02), wall_hi=L.Wall(1.02))
    f0 = _rest(static)
    np.testing.assert_array_equal(L.run(f0, heated, 5), L.run(f0, static, 5))


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_symmetric_heating_keeps_the_mirror_symmetry_and_mass(name):
    prob = _channel(name, 0.01)
    f = _rest(prob)
    m0 = f.sum()
    for n in range(40):
        f = L.step(f, prob, n)
        assert abs(f.sum() / m0 - 1.0) < 1e-14
    rho, u, T, s, q = L.macroscopic(f, prob, n=40)
    np.testing.assert_allclose(u[:, -1], -u[::-1, -1], atol=1e-15)
    np.testing.assert_allclose(T, T[::-1], atol=1e-15)
    np.testing.assert_allclose(rho, rho[::-1], atol=1e-15)
    assert np.abs(u[:, 0]).max() < 1e-15
    assert np.abs(u[:, -1]).max() > 1e-6                  # the gas does move


def test_small_amplitude_response_is_linear_and_heats_first(d2q37):
    A, steps = 1e-3, 30
    dev = []
    for amp in (A, 2 * A):
        prob = _channel("D2Q37", amp)
        f = L.run(_rest(prob), prob, steps)
        rho, u, T, s, q = L.macroscopic(f, prob, n=steps)
        dev.append(np.concatenate([rho - 1.0, u[:, 1], T - 1.0]))
        if amp == A:
            # sin > 0 over the first steps: the walls warm the gas (and the
            # compression waves they launch meet and heat the middle too)
            assert T.min() > 1.0
    d1, d2 = dev
    assert np.abs(d2 - 2 * d1).max() < 1e-2 * np.abs(d2).max()


def test_heating_adds_and_cooling_removes_energy(d2q37):
    def energy(f, prob):
        return 0.5 * (f * (prob.vs.c ** 2).sum(1)[:, None]).sum()
    for sign in (1.0, -1.0):
        prob = _channel("D2Q37", sign * 0.01)
        f0 = _rest(prob)
        f = L.run(f0, prob, 20)
        assert sign * (energy(f, prob) - energy(f0, prob)) > 0
