"""Pins for the oracle's FP64 reductions (mass, energy, momentum, mass flow
rate, steady-state residual) against closed forms of prescribed states.

The reductions are taken over the current time level: the stored
post-collision state is streamed (pull) and the physical distribution is
recovered from it, as for every moment read-out. On a periodic lattice
streaming permutes each velocity's values among the cells, so the sums over
all cells of sum_alpha fbar_alpha psi(c_alpha) are those of the stored state
for any psi. For a stored state made of truncated Maxwellians rho_k S(T_k, u_k)
(eq. feq0; its moments through the second order are exact on a set of
degree >= N + 2) the recovery of the physical f (Sec. 2.2, the trapezoidal
change of variable) then gives, with hs = dt/2 (trapezoid) or 0 (Euler):

  sum rho        = sum_k rho_k
  sum rho u      = sum_k rho_k u_k + hs g sum_k rho_k          (rho u = j + hs rho g)
  sum 1/2 f c^2  = 1/2 sum_k rho_k (u_k^2 + D T_k)
                   + hs g . sum_k rho_k u_k + hs^2 |g|^2 sum_k rho_k
                   (tr M2 = tr Mbar2 + 2 hs rho g . u)

The mass flow rate through a plane normal to x is the integral of rho u_x over
the cross-section, averaged over the nx planes: dx^(D-1)/nx sum rho u_x. For a
parabolic u_x across a channel of height 1 sampled at cell centres, the
midpoint rule is exact up to its known error term: sum_j dx u(y_j) =
2U/3 + U dx^2/3 for u = 4U y(1 - y). Planted mistakes (a wrong power of dx,
no division by nx, no half-step force shift) move each value by far more than
the tolerance.
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import quadrature

TOL = 1e-12


def _state(prob, rho, u, T):
    """Stored truncated-Maxwellian state of prescribed fields (no noise)."""
    return L.equilibrium_state(prob, rho, u, T)


def _fields(prob, rng):
    M, D = prob.M, prob.D
    rho = 1.0 + 0.1 * rng.uniform(-1, 1, M)
    u = 0.08 * rng.uniform(-1, 1, (M, D))
    T = 1.0 + 0.1 * rng.uniform(-1, 1, M)
    return rho, u, T


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
@pytest.mark.parametrize("scheme", ["trapezoid", "euler"])
@pytest.mark.parametrize("force", [False, True])
def test_mass_momentum_energy_of_prescribed_fields(name, scheme, force):
    vs = quadrature.velocity_set(name)
    dims = (7, 5) if vs.D == 2 else (5, 4, 3)
    g = (0.03, -0.02, 0.01) if force else (0.0, 0.0, 0.0)
    prob = L.Problem(vs, dims, Kn=0.07, Pr=0.8, scheme=scheme, g=g, n_ref=9)
    rho, u, T = _fields(prob, np.random.default_rng(3))
    red = L.reductions(_state(prob, rho, u, T), prob)
    gv = prob.gvec
    hs = prob.hs
    mass = rho.sum()
    mom = (rho[:, None] * u).sum(axis=0) + hs * gv * mass
    energy = (0.5 * np.sum(rho * (np.sum(u * u, axis=1) + prob.D * T))
              + hs * gv @ (rho[:, None] * u).sum(axis=0) + hs ** 2 * (gv @ gv) * mass)
    assert abs(red["mass"] - mass) <= TOL * mass
    np.testing.assert_allclose(red["mom"], mom, rtol=0, atol=TOL * mass)
    assert abs(red["energy"] - energy) <= TOL * energy
    if force and scheme == "trapezoid":
        # a dropped half-step shift of the force would be visible
        assert np.max(np.abs(red["mom"] - (rho[:, None] * u).sum(axis=0))) > 1e3 * TOL * mass
        e_no_shift = 0.5 * np.sum(rho * (np.sum(u * u, axis=1) + prob.D * T))
        assert abs(red["energy"] - e_no_shift) > 1e3 * TOL * energy


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_mass_of_uniform_state_with_walls(name):
    """A uniform rest state at the walls' temperature is a fixed point of the
    step (the diffuse walls re-emit exactly what arrives), so the mass of the
    current level is M rho0 and its momentum zero."""
    vs = quadrature.velocity_set(name)
    dims = (5, 8) if vs.D == 2 else (3, 4, 7)
    Tw = 1.1
    prob = L.Problem(vs, dims, Kn=0.1, Pr=2 / 3, walls=True, wall_lo=L.Wall(Tw), wall_hi=L.Wall(Tw))
    rho0 = 1.3
    M = prob.M
    f = _state(prob, np.full(M, rho0), np.zeros((M, vs.D)), np.full(M, Tw))
    red = L.reductions(f, prob)
    assert abs(red["mass"] - M * rho0) <= TOL * M * rho0
    assert np.max(np.abs(red["mom"])) <= TOL * M
    assert abs(red["energy"] - 0.5 * M * rho0 * vs.D * Tw) <= TOL * M
    assert red["mdot"] == pytest.approx(0.0, abs=TOL)


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
@pytest.mark.parametrize("scheme", ["trapezoid", "euler"])
def test_mass_flow_rate_of_parabolic_profile(name, scheme):
    """u_x = 4U eta(1 - eta) across the last axis (eta = (j + 1/2)/n, height
    1 with n_ref = n), rho = T = 1, a force g_x: the mass flow rate through a
    plane normal to x is the midpoint-rule integral of u_x + hs g_x over the
    cross-section."""
    vs = quadrature.velocity_set(name)
    n = 12
    dims = (5, n) if vs.D == 2 else (4, 3, n)
    gx = 0.02
    prob = L.Problem(vs, dims, Kn=0.1, Pr=2 / 3, scheme=scheme, g=(gx, 0.0, 0.0), n_ref=n)
    U = 0.06
    eta = (prob.coords[:, -1] + 0.5) / n
    M = prob.M
    u = np.zeros((M, vs.D))
    u[:, 0] = 4.0 * U * eta * (1.0 - eta)
    red = L.reductions(_state(prob, np.ones(M), u, np.ones(M)), prob)
    dx = 1.0 / n
    width = 1.0 if vs.D == 2 else dims[1] * dx          # extent of the cross-section along y (3-D)
    exact = width * (2.0 * U / 3.0 + U * dx * dx / 3.0 + prob.hs * gx)
    assert abs(red["mdot"] - exact) <= TOL
    # planted mistakes: dx^D instead of dx^(D-1), no average over the nx planes, no force shift
    assert abs(red["mdot"] * dx - exact) > 1e6 * TOL
    assert abs(red["mdot"] * dims[0] - exact) > 1e6 * TOL
    if scheme == "trapezoid":
        assert abs((red["mdot"] - width * prob.hs * gx) - exact) > 1e6 * TOL


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_residual_closed_form(name):
    """From a uniform periodic state with velocity U the current level has
    u = U + hs g in every cell; against a prescribed previous field V the
    residual is ||U' - V||_2 / ||U'||_2 over all cells and components, and 0
    against itself."""
    vs = quadrature.velocity_set(name)
    dims = (6, 5) if vs.D == 2 else (4, 3, 5)
    g = (0.01, 0.02, -0.01)
    prob = L.Problem(vs, dims, Kn=0.1, Pr=1.0, g=g, n_ref=10)
    M, D = prob.M, vs.D
    U = np.array([0.05, -0.03, 0.02])[:D]
    f = _state(prob, np.ones(M), np.tile(U, (M, 1)), np.ones(M))
    Up = U + prob.hs * prob.gvec
    rng = np.random.default_rng(5)
    V = Up[None, :] + 0.01 * rng.standard_normal((M, D))
    red = L.reductions(f, prob, u_prev=V)
    exact = np.sqrt(np.sum((Up[None, :] - V) ** 2)) / np.sqrt(M * np.sum(Up ** 2))
    assert abs(red["residual"] - exact) <= 1e-12 * exact
    np.testing.assert_allclose(red["u"], np.tile(Up, (M, 1)), rtol=0, atol=1e-14)
    assert L.reductions(f, prob, u_prev=red["u"])["residual"] == 0.0
    assert L.reductions(f, prob)["residual"] == 0.0
    # the norm is the 2-norm over all cells, not a per-cell maximum or mean
    assert abs(np.max(np.linalg.norm(Up[None, :] - V, axis=1)) / np.linalg.norm(Up) - exact) > 1e-3 * exact
