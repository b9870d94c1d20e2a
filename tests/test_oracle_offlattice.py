"""Pins for the oracle of the paper's own scheme (Sec. 3.1): the 6-point
Gauss-Hermite product set with forward Euler in time and TVD minmod fluxes.

* The product set integrates every monomial c_x^p c_y^q with p, q <= 11
  against the Gaussian weight exactly (eq. weight per axis), not p = 12; its
  N = 4 ES projection carries the anisotropic Gaussian's moments to order 4.
* The flux form conserves each velocity's total on a periodic grid; a
  uniform equilibrium is a fixed point of the whole step.
* At |nu| = 1 the TVD update is the exact shift by one cell; for |nu| < 1 it
  does not increase the total variation, and smooth profiles converge at
  close to second order (the minmod limiter clips extrema).
* Shear waves decay at nu k^2 (Newtonian viscosity Kn T^varpi) up to the
  scheme's numerical diffusion, which shrinks under refinement.
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import model
from oracle import offlattice as O


@pytest.fixture(scope="module")
def gh():
    return O.ProductSet(6, 2, 4)


def _gauss_moment(p):
    return 0.0 if p % 2 else float(np.prod(np.arange(p - 1, 0, -2))) if p else 1.0


def test_product_set_exact_to_degree_eleven_per_axis(gh):
    c, w = gh.c, gh.w
    for p in range(12):
        for q in range(12):
            terms = w * c[:, 0] ** p * c[:, 1] ** q
            scale = np.abs(terms).sum()
            assert abs(terms.sum() - _gauss_moment(p) * _gauss_moment(q)) < 1e-13 * scale
    got = np.sum(w * c[:, 0] ** 12)
    assert abs(got - _gauss_moment(12)) > 1.0


def test_product_set_order_and_opposites(gh):
    assert gh.Q == 36 and gh.P == 18
    np.testing.assert_array_equal(gh.c[gh.P:], -gh.c[:gh.P])
    assert np.all(gh.c[:gh.P, 0] > 0)
    assert abs(gh.w.sum() - 1.0) < 1e-14
    np.testing.assert_allclose(np.sort(np.unique(np.round(np.abs(gh.c), 12))),
                               [0.616706590193, 1.889175877754, 3.324257433552], rtol=1e-11)


def test_es_projection_on_the_product_set(gh):
    rng = np.random.default_rng(5)
    M = 6
    rho = 1.0 + 0.1 * rng.uniform(-1, 1, M)
    u = 0.2 * rng.uniform(-1, 1, (M, 2))
    T = 1.0 + 0.1 * rng.uniform(-1, 1, M)
    sig = 0.05 * rng.uniform(-1, 1, (M, 2, 2))
    sig = 0.5 * (sig + sig.transpose(0, 2, 1))
    sig -= np.einsum("mii->m", sig)[:, None, None] / 2 * np.eye(2)
    lam = model.es_tensor(T, sig, rho, model.b_from_prandtl(2 / 3))
    a = model.es_coefficients(rho, u, lam, 4)
    f = model.hermite_projection(a, gh.c, gh.w)
    m0, m1, m2, m3 = model.raw_moments(f, gh.c, 3)
    np.testing.assert_allclose(m0, rho, rtol=1e-13)
    np.testing.assert_allclose(m1, rho[:, None] * u, atol=1e-13)
    np.testing.assert_allclose(m2, rho[:, None, None] * (np.einsum("mi,mj->mij", u, u) + lam), atol=1e-13)
    uuu = np.einsum("mi,mj,mk->mijk", u, u, u)
    sym = (np.einsum("mij,mk->mijk", lam, u) + np.einsum("mik,mj->mijk", lam, u)
           + np.einsum("mjk,mi->mijk", lam, u))
    np.testing.assert_allclose(m3, rho[:, None, None, None] * (uuu + sym), atol=1e-13)


def _problem(gh, dims=(8, 6), **kw):
    return O.TVDProblem(gh, dims, Kn=kw.pop("Kn", 0.1), Pr=kw.pop("Pr", 2 / 3), **kw)


def test_flux_form_conserves_each_velocity(gh):
    prob = _problem(gh)
    rng = np.random.default_rng(6)
    f = rng.uniform(0.5, 1.5, (gh.Q, prob.M))
    adv = O.advection(f, prob)
    assert np.abs(adv.sum(axis=1)).max() < 1e-13 * f.sum(axis=1).max()
    assert np.abs(adv).max() > 1e-3


def test_uniform_equilibrium_is_a_fixed_point(gh):
    prob = _problem(gh, g=(0.0, 0.0, 0.0))
    M = prob.M
    f0 = O.equilibrium_state(prob, 1.1 * np.ones(M), np.tile([0.1, -0.05], (M, 1)), 1.05 * np.ones(M))
    np.testing.assert_allclose(O.step(f0, prob), f0, rtol=1e-14, atol=1e-16)


def _advect_only(f, prob, steps):
    for _ in range(steps):
        f = f - O.advection(f, prob)
    return f


def test_unit_courant_is_the_exact_shift(gh):
    """On a one-row grid the x-flux of the fastest velocities (|c_x| the
    largest root) at CFL = 1 moves them exactly one cell per step."""
    prob = O.TVDProblem(gh, (16, 1), Kn=0.1, Pr=2 / 3, cfl=1.0)
    rng = np.random.default_rng(7)
    f = rng.uniform(0.5, 1.5, (gh.Q, 16))
    out = f - O.advection(f, prob)
    fast = np.nonzero(np.isclose(np.abs(gh.c[:, 0]), np.abs(gh.c).max()))[0]
    assert len(fast) == 12
    for a in fast:
        assert abs(abs(gh.c[a, 0]) * prob.dt / prob.dx - 1.0) < 1e-14
        np.testing.assert_allclose(out[a], np.roll(f[a], int(np.sign(gh.c[a, 0]))), rtol=1e-14)


def _total_variation(x):
    return np.abs(np.diff(np.concatenate([x, x[:1]]))).sum()


def test_tvd_does_not_increase_total_variation(gh):
    prob = O.TVDProblem(gh, (40, 1), Kn=0.1, Pr=2 / 3, cfl=0.8)
    rng = np.random.default_rng(8)
    f = np.where(rng.uniform(size=(gh.Q, 40)) > 0.5, 1.0, 0.2) + 0.05 * rng.standard_normal((gh.Q, 40))
    tv = [_total_variation(f[a]) for a in range(gh.Q)]
    for _ in range(30):
        f = f - O.advection(f, prob)
        tv_new = [_total_variation(f[a]) for a in range(gh.Q)]
        assert all(b <= t + 1e-12 for b, t in zip(tv_new, tv))
        tv = tv_new


def test_smooth_advection_converges_at_about_second_order(gh):
    a = 0                                   # slowest velocity, c_x > 0
    errs = []
    for n in (32, 64, 128):
        prob = O.TVDProblem(gh, (n, 1), Kn=0.1, Pr=2 / 3, cfl=0.5)
        x = (np.arange(n) + 0.5) / n
        f = np.ones((gh.Q, n)) + 0.3 * np.sin(2 * np.pi * x)[None, :]
        steps = int(round(0.5 / (gh.c[a, 0] * prob.dt)))     # travel half the box
        t = steps * prob.dt
        g = _advect_only(f, prob, steps)
        exact = 1.0 + 0.3 * np.sin(2 * np.pi * (x - gh.c[a, 0] * t))
        errs.append(np.abs(g[a] - exact).mean())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.5), rates


@pytest.mark.slow
def test_shear_wave_decays_at_the_viscous_rate(gh):
    rates = []
    for ny in (24, 48):
        Kn = 0.02
        prob = O.TVDProblem(gh, (1, ny), Kn=Kn, Pr=2 / 3, cfl=0.5, n_ref=ny)
        y = (np.arange(ny) + 0.5) / ny
        M = prob.M
        amp = 1e-3
        ux = amp * np.sin(2 * np.pi * y)
        f = O.equilibrium_state(prob, np.ones(M), np.stack([ux, np.zeros(M)], 1), np.ones(M))
        steps = int(round(0.3 / prob.dt))
        f = O.run(f, prob, steps)
        rho, u, T, s, q = O.macroscopic(f, prob)
        a_end = 2 * np.mean(u[:, 0] * np.sin(2 * np.pi * y))
        rates.append(-np.log(a_end / amp) / (steps * prob.dt))
    k2 = (2 * np.pi) ** 2
    nu = 0.02                                  # Kn T^varpi / rho at rest
    err = [abs(r / (nu * k2) - 1.0) for r in rates]
    assert err[1] < 0.1 and err[1] < err[0]


def test_unsplit_euler_stability_bound():
    """The scheme of Sec. 3.1 applies forward Euler to the collision and the
    advection together. With w = dt/tau, one step is a convex combination of
    the equilibrium (weight w) and a TVD advection step whose Courant number
    is sum|nu| / (1 - w), the sum taken over the axes along which the field
    varies. So it stays bounded while sum|nu| <= 1 - w. Collision-free
    advection is bounded up to sum|nu| = 1; with collisions the bound moves
    in by w, and beyond it the noise grows without bound."""
    gh4 = O.ProductSet(4, 2, 3)
    Kn, Pr = 0.05, 2 / 3

    def run(dims, cfl, kn, steps=400):
        prob = O.TVDProblem(gh4, dims, Kn=kn, Pr=Pr, cfl=cfl, n_ref=max(dims), g=(0.0, 0.0, 0.0))
        rng = np.random.default_rng(3)
        M = prob.M
        f = O.equilibrium_state(prob, np.ones(M), np.zeros((M, 2)), np.ones(M),
                                rng.standard_normal((gh4.Q, M)), 0.02)
        with np.errstate(all="ignore"):
            g = O.run(f, prob, steps)
        w = prob.dt * Pr / kn               # dt / tau at rho = T = 1
        grew = not np.isfinite(g).all() or np.abs(g).max() > 10 * np.abs(f).max()
        return w, grew, np.abs(f).max(), np.abs(g).max()

    # collision-free: no new extrema up to a unit Courant number
    w, grew, m0, m1 = run((1, 48), 1.0, 1e3)
    assert w < 1e-4 and m1 <= m0
    # 1-D field with collisions (w ~ 0.1)
    w, grew, m0, m1 = run((1, 48), 0.85, Kn)
    assert 0.85 <= 1 - w and m1 <= m0
    w, grew, _, _ = run((1, 48), 0.95, Kn)
    assert 0.95 > 1 - w and grew
    # 2-D field: the two axes' Courant numbers add up
    w, grew, m0, m1 = run((24, 24), 0.44, Kn)
    assert 2 * 0.44 <= 1 - w and m1 <= m0
    w, grew, _, _ = run((24, 24), 0.5, Kn)
    assert 2 * 0.5 > 1 - w and grew
