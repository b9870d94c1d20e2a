"""Pins for the oracle's Maxwell wall model (Sec. 3.2): a fraction gamma of
the particles that reach a wall is re-emitted diffusely, 1 - gamma is
reflected specularly.

* A specularly reflected particle keeps its tangential velocity, reverses
  the normal one and lands where a straight flight mirrored in the wall plane
  ends: checked particle by particle from the geometry of the flight.
* Specular walls only move populations between mirror-paired velocities, so
  each pair's values are permuted; mass, energy and tangential momentum are
  conserved by the full step while diffuse walls at other temperatures change
  the energy.
* The pull is affine in gamma: gamma times the diffuse pull plus 1 - gamma
  times the specular one.
* Less accommodation means more slip in Couette flow (Maxwell's slip length
  grows like (2 - gamma)/gamma).
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import quadrature


def _problem(name, gam_lo, gam_hi, T=(1.0, 1.0), uw=0.0, dims=None, **kw):
    vs = quadrature.velocity_set(name)
    if dims is None:
        dims = (5, 9) if vs.D == 2 else (4, 3, 9)
    u_lo = (-uw, 0.0, 0.0)
    u_hi = (uw, 0.0, 0.0)
    return L.Problem(vs, dims, Kn=kw.pop("Kn", 0.1), Pr=2 / 3, walls=True,
                     wall_lo=L.Wall(T[0], u_lo, gam_lo), wall_hi=L.Wall(T[1], u_hi, gam_hi), **kw)


def _flight_end(p, e, dims):
    """Where a particle at integer cell p with velocity e is one step later,
    and with which velocity: straight flight, periodic in every axis but the
    last, mirrored in the wall planes at -1/2 and n - 1/2 of the last axis."""
    q = [p[k] + e[k] for k in range(len(p))]
    v = list(e)
    n = dims[-1]
    if q[-1] < 0:                       # crossed the plane y = -1/2
        q[-1] = -1 - q[-1]
        v[-1] = -v[-1]
    elif q[-1] > n - 1:                 # crossed the plane y = n - 1/2
        q[-1] = 2 * n - 1 - q[-1]
        v[-1] = -v[-1]
    for k in range(len(p) - 1):
        q[k] %= dims[k]
    return tuple(q), tuple(v)


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_specular_particle_lands_where_the_mirrored_flight_ends(name):
    prob = _problem(name, 0.0, 0.0)
    e = prob.vs.e
    vel = {tuple(v): a for a, v in enumerate(e)}
    dims = prob.dims
    n = dims[-1]
    checked = 0
    for a in range(prob.vs.Q):
        if e[a, -1] == 0:
            continue
        # a particle next to the wall it flies towards, off every periodic edge
        p = [min(2, d - 1) for d in dims[:-1]]
        p.append(0 if e[a, -1] < 0 else n - 1)
        f = np.zeros((prob.vs.Q, prob.M))
        src = prob.flat(np.array(p))
        f[a, src] = 1.0
        out = L.gather(f, prob)
        q, v = _flight_end(p, tuple(e[a]), dims)
        expect = np.zeros_like(out)
        expect[vel[v], prob.flat(np.array(q))] = 1.0
        np.testing.assert_array_equal(out, expect)
        checked += 1
    assert checked == np.count_nonzero(e[:, -1])


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_specular_pull_permutes_each_mirror_pair(name):
    rng = np.random.default_rng(21)
    prob = _problem(name, 0.0, 0.0, T=(0.9, 1.1))
    f = rng.uniform(0.5, 1.5, (prob.vs.Q, prob.M))
    out = L.gather(f, prob)
    for a in range(prob.vs.Q):
        pair = sorted({a, int(prob.mirror[a])})
        np.testing.assert_array_equal(np.sort(out[pair].ravel()), np.sort(f[pair].ravel()))
    # no trace of the wall state: the same pull with other wall temperatures
    other = _problem(name, 0.0, 0.0, T=(1.3, 0.8))
    np.testing.assert_array_equal(L.gather(f, other), out)


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_pull_is_affine_in_accommodation(name):
    rng = np.random.default_rng(22)
    T = (0.97, 1.04)
    diffuse = _problem(name, 1.0, 1.0, T=T, uw=0.03)
    specular = _problem(name, 0.0, 0.0, T=T, uw=0.03)
    mixed = _problem(name, 0.3, 0.8, T=T, uw=0.03)
    f = diffuse.vs.w[:, None] * rng.uniform(0.9, 1.1, (diffuse.vs.Q, diffuse.M))
    g1, g0, gm = L.gather(f, diffuse), L.gather(f, specular), L.gather(f, mixed)
    e_n = diffuse.vs.e[:, -1][:, None]
    t = diffuse.coords[:, -1][None, :]
    lo = np.broadcast_to(t - e_n < 0, f.shape)
    hi = np.broadcast_to(t - e_n >= diffuse.dims[-1], f.shape)
    expect = g1.copy()
    expect[lo] = 0.3 * g1[lo] + 0.7 * g0[lo]
    expect[hi] = 0.8 * g1[hi] + 0.2 * g0[hi]
    np.testing.assert_allclose(gm, expect, rtol=1e-15, atol=0)
    assert not np.allclose(g1[lo], g0[lo])


def _moments(f, prob):
    """Total mass, energy, tangential (x) and normal momentum of a state."""
    c = prob.vs.c
    return (f.sum(), 0.5 * (f * (c ** 2).sum(1)[:, None]).sum(), (f * c[:, :1]).sum(),
            (f * c[:, -1:]).sum())


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_specular_walls_conserve_mass_energy_and_tangential_momentum(name):
    rng = np.random.default_rng(23)
    T = (0.9, 1.1)
    spec = _problem(name, 0.0, 0.0, T=T, uw=0.05)
    M, D = spec.M, spec.D
    rho = 1.0 + 0.05 * rng.uniform(-1, 1, M)
    u = 0.05 * rng.uniform(-1, 1, (M, D))
    Tc = 1.0 + 0.05 * rng.uniform(-1, 1, M)
    f0 = L.equilibrium_state(spec, rho, u, Tc)
    m0, E0, px0, _ = _moments(f0, spec)
    f = f0
    for _ in range(6):
        f = L.step(f, spec)
        m, E, px, _ = _moments(f, spec)
        assert abs(m / m0 - 1) < 1e-14
        assert abs(E / E0 - 1) < 1e-14
        assert abs(px - px0) < 1e-14 * m0
    # diffuse walls at other temperatures do exchange energy (and moving
    # diffuse walls exchange tangential momentum)
    diff = _problem(name, 1.0, 1.0, T=T, uw=0.05)
    g = L.run(f0, diff, 6)
    m, E, px, _ = _moments(g, diff)
    assert abs(m / m0 - 1) < 1e-14
    assert abs(E / E0 - 1) > 1e-6
    assert abs(px - px0) > 1e-6 * m0


@pytest.mark.slow
def test_less_accommodation_more_couette_slip(d2q37):
    slip = []
    uw = 0.05 * d2q37.r
    for gam in (1.0, 0.6):
        prob = _problem("D2Q37", gam, gam, uw=uw, dims=(1, 12), Kn=0.1)
        M = prob.M
        f = L.equilibrium_state(prob, np.ones(M), np.zeros((M, 2)), np.ones(M))
        f = L.run(f, prob, 700)
        rho, u, T, s, q = L.macroscopic(f, prob)
        ux = u[:, 0]
        np.testing.assert_allclose(ux, -ux[::-1], atol=1e-14)
        slip.append(uw - ux[-1])
    assert 0.0 < slip[0] < slip[1]
