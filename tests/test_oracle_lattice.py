"""Pins for the oracle's time step (streaming, diffuse walls, collision, force)
against invariants and closed forms that the paper's model fixes:

* the collision conserves mass, momentum and energy (Sec. 2.1); the body force
  adds dt rho g of momentum and dt rho g.u of energy per step (Sec. 2.2);
* homogeneous relaxation: the stress relaxes at 1/(Pr tau) and the heat flux
  at 1/tau, so Pr = 1/(1-b) is recovered exactly (Sec. 2.1);
* Newtonian closures in the slip regime: sigma_xy = -mu du/dy with
  mu = Kn T^varpi and q_y = -kappa dT/dy with kappa = (D+2)/2 mu/Pr
  (Sec. 2.1 transport coefficients, Sec. 2.2 scaling);
* the diffuse wall of Sec. 3.2 conserves mass and leaves a wall-temperature
  rest equilibrium unchanged;
* shear and thermal waves decay at nu k^2 and nu k^2/Pr.
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import model


def _near_equilibrium(prob, rng, amp=0.02, u_amp=0.05):
    M, D = prob.M, prob.D
    rho = 1.0 + 0.05 * rng.uniform(-1, 1, M)
    u = u_amp * rng.uniform(-1, 1, (M, D))
    T = 1.0 + 0.05 * rng.uniform(-1, 1, M)
    f = L.equilibrium_state(prob, rho, u, T)
    return f * (1.0 + amp * rng.standard_normal(f.shape))


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
@pytest.mark.parametrize("scheme", ["trapezoid", "euler"])
def test_collision_conserves_mass_momentum_energy(name, scheme):
    from oracle import quadrature
    vs = quadrature.velocity_set(name)
    dims = (6,) * vs.D
    prob = L.Problem(vs, dims, Kn=0.05, Pr=2 / 3, scheme=scheme, n_ref=8)
    fbar = _near_equilibrium(prob, np.random.default_rng(0))
    fs = L.collide(fbar, prob)
    c2 = np.sum(vs.c ** 2, axis=1)
    np.testing.assert_allclose(fs.sum(0), fbar.sum(0), rtol=1e-14)
    np.testing.assert_allclose(fs.T @ vs.c, fbar.T @ vs.c, atol=1e-15)
    np.testing.assert_allclose(fs.T @ c2, fbar.T @ c2, rtol=1e-14)
    assert np.abs(fs - fbar).max() > 1e-4     # it did relax


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
@pytest.mark.parametrize("scheme", ["trapezoid", "euler"])
def test_body_force_momentum_and_energy_source(name, scheme):
    from oracle import quadrature
    vs = quadrature.velocity_set(name)
    g = (0.3, -0.2, 0.1)
    prob = L.Problem(vs, (5,) * vs.D, Kn=0.05, Pr=2 / 3, g=g, scheme=scheme, n_ref=8)
    fbar = _near_equilibrium(prob, np.random.default_rng(1))
    fs = L.collide(fbar, prob)
    st = L.physical_state(fbar, prob)
    rho = fbar.sum(0)
    gv = np.array(g[:vs.D])
    np.testing.assert_allclose(fs.T @ vs.c - fbar.T @ vs.c, prob.dt * rho[:, None] * gv[None],
                               atol=1e-15)
    c2 = np.sum(vs.c ** 2, axis=1)
    np.testing.assert_allclose(0.5 * (fs.T @ c2 - fbar.T @ c2), prob.dt * rho * (st.u @ gv),
                               atol=1e-15)


@pytest.mark.parametrize("scheme", ["trapezoid", "euler"])
@pytest.mark.parametrize("Pr", [2 / 3, 0.8, 1.0])
def test_homogeneous_relaxation_recovers_prandtl(d2q37, scheme, Pr):
    vs = d2q37
    # tau/dt chosen so that Euler is stable: dt/tau = Pr * 0.4
    prob = L.Problem(vs, (1, 1), Kn=0.1, Pr=Pr, varpi=0.5, scheme=scheme,
                     n_ref=int(round(1 / (0.1 * 0.4 * vs.r))))
    rho, u, T = np.array([1.1]), np.array([[0.05, -0.03]]), np.array([1.02])
    f = L.equilibrium_state(prob, rho, u, T)
    from oracle import hermite
    chi2 = hermite.chi(vs.c, 2)
    chi3 = hermite.chi(vs.c, 3)
    f = f + vs.w[:, None] * (0.01 * chi2[:, 0, 1] + 0.004 * (chi3[:, 0, 0, 0] + chi3[:, 0, 1, 1])
                             + 0.003 * chi3[:, 1, 1, 1])[:, None]
    hist = []
    for n in range(4):
        rho_n, u_n, T_n, s_n, q_n = L.macroscopic(f, prob)
        hist.append((rho_n[0], u_n[0], T_n[0], s_n[0], q_n[0]))
        f = L.step(f, prob)
    tau = model.relaxation_time(prob.Kn, Pr, 0.5, hist[0][0], hist[0][2])
    x = prob.dt / tau
    y = x / Pr
    if scheme == "euler":
        fs, fq = 1 - y, 1 - x
    else:
        fs, fq = (2 - y) / (2 + y), (2 - x) / (2 + x)
    for n in range(3):
        np.testing.assert_allclose(hist[n + 1][0], hist[0][0], rtol=1e-14)
        np.testing.assert_allclose(hist[n + 1][1], hist[0][1], atol=1e-15)
        np.testing.assert_allclose(hist[n + 1][2], hist[0][2], rtol=1e-14)
        np.testing.assert_allclose(hist[n + 1][3], fs * hist[n][3], atol=1e-15)
        np.testing.assert_allclose(hist[n + 1][4], fq * hist[n][4], atol=1e-15)
    # invert the measured factors: x/y = Pr
    ms = hist[1][3][0, 1] / hist[0][3][0, 1]
    mq = hist[1][4][0] / hist[0][4][0]
    if scheme == "euler":
        y_m, x_m = 1 - ms, 1 - mq
    else:
        y_m, x_m = 2 * (1 - ms) / (1 + ms), 2 * (1 - mq) / (1 + mq)
    assert x_m / y_m == pytest.approx(Pr, rel=1e-10)


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_recovered_distribution_has_the_reconstructed_moments(name):
    from oracle import quadrature
    vs = quadrature.velocity_set(name)
    prob = L.Problem(vs, (4,) * vs.D, Kn=0.05, Pr=2 / 3, g=(0.2, 0.1, -0.1), n_ref=6)
    fbar = _near_equilibrium(prob, np.random.default_rng(2))
    f, st = L.physical_distribution(fbar, prob)
    rho, u, T, sigma, q = model.macroscopic(f, vs.c)
    np.testing.assert_allclose(rho, st.rho, rtol=1e-14)
    np.testing.assert_allclose(u, st.u, atol=1e-15)
    np.testing.assert_allclose(T, st.T, rtol=1e-14)
    np.testing.assert_allclose(sigma, st.sigma, atol=1e-15)
    np.testing.assert_allclose(model.raw_moments(f, vs.c, 3)[3], st.M3, atol=2e-15)


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_periodic_streaming_is_a_permutation(name):
    from oracle import quadrature
    vs = quadrature.velocity_set(name)
    dims = (5, 4) if vs.D == 2 else (4, 3, 5)
    prob = L.Problem(vs, dims, Kn=0.1, Pr=1.0)
    f = np.random.default_rng(3).uniform(size=(vs.Q, prob.M))
    fb = L.gather(f, prob)
    np.testing.assert_allclose(np.sort(fb, axis=1), np.sort(f, axis=1), rtol=0, atol=0)
    # a single marked cell moves by e_alpha
    f = np.zeros((vs.Q, prob.M))
    f[:, 0] = 1.0
    fb = L.gather(f, prob)
    for a in range(vs.Q):
        dest = np.mod(prob.coords[0] + vs.e[a], np.array(dims))
        assert fb[a, prob.flat(dest[None])[0]] == 1.0


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_wall_rest_equilibrium_is_a_fixed_point(name):
    from oracle import quadrature
    vs = quadrature.velocity_set(name)
    dims = (3, 8) if vs.D == 2 else (2, 3, 8)
    Tw = 1.03
    prob = L.Problem(vs, dims, Kn=0.1, Pr=2 / 3, walls=True,
                     wall_lo=L.Wall(Tw), wall_hi=L.Wall(Tw))
    M = prob.M
    f0 = L.equilibrium_state(prob, 1.2 * np.ones(M), np.zeros((M, vs.D)), Tw * np.ones(M))
    f = L.run(f0, prob, 5)
    np.testing.assert_allclose(f, f0, rtol=1e-13)


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_walls_conserve_mass_every_step(name):
    from oracle import quadrature
    vs = quadrature.velocity_set(name)
    dims = (4, 10) if vs.D == 2 else (3, 2, 10)
    uw = (0.08, 0.02, 0.0) if vs.D == 3 else (0.08, 0.0, 0.0)
    prob = L.Problem(vs, dims, Kn=0.1, Pr=2 / 3, walls=True, g=(0.05, 0.0, 0.0),
                     wall_lo=L.Wall(1.0, tuple(-a for a in uw)), wall_hi=L.Wall(1.05, uw))
    f = _near_equilibrium(prob, np.random.default_rng(4))
    m0 = f.sum()
    for _ in range(10):
        f = L.step(f, prob)
        assert abs(f.sum() / m0 - 1.0) < 1e-14


@pytest.mark.slow
def test_couette_antisymmetry_linear_bulk_and_viscosity(d2q37):
    vs, ny, uw, Kn = d2q37, 16, 0.05, 0.05
    prob = L.Problem(vs, (1, ny), Kn=Kn, Pr=2 / 3, walls=True,
                     wall_lo=L.Wall(1.0, (-uw, 0, 0)), wall_hi=L.Wall(1.0, (uw, 0, 0)))
    M = prob.M
    f = L.equilibrium_state(prob, np.ones(M), np.zeros((M, 2)), np.ones(M))
    f = L.run(f, prob, 1500)
    rho, u, T, s, q = L.macroscopic(f, prob)
    ux = u[:, 0]
    np.testing.assert_allclose(ux, -ux[::-1], atol=1e-14)
    np.testing.assert_allclose(T, T[::-1], atol=1e-14)
    y = (np.arange(ny) + 0.5) / ny
    bulk = slice(3, ny - 3)
    slope, icpt = np.polyfit(y[bulk], ux[bulk], 1)
    assert np.abs(ux[bulk] - (slope * y[bulk] + icpt)).max() < 2e-3 * uw
    assert 0.0 < slope < 2 * uw                       # slip reduces the shear rate
    mu = Kn * T[bulk] ** 0.5
    assert np.mean(s[bulk, 0, 1]) == pytest.approx(np.mean(-mu * slope), rel=1e-2)
    np.testing.assert_allclose(s[bulk, 0, 1], -mu * slope, rtol=2e-2)


@pytest.mark.slow
def test_fourier_flux_is_uniform_and_follows_conductivity(d2q37):
    vs, ny, Kn, Pr = d2q37, 16, 0.05, 2 / 3
    prob = L.Problem(vs, (1, ny), Kn=Kn, Pr=Pr, walls=True,
                     wall_lo=L.Wall(0.97), wall_hi=L.Wall(1.03))
    M = prob.M
    f = L.equilibrium_state(prob, np.ones(M), np.zeros((M, 2)), np.ones(M))
    f = L.run(f, prob, 2500)
    rho, u, T, s, q = L.macroscopic(f, prob)
    y = (np.arange(ny) + 0.5) / ny
    bulk = slice(3, ny - 3)
    dTdy = np.polyfit(y[bulk], T[bulk], 1)[0]
    assert dTdy > 0
    kappa = (prob.D + 2) / 2 * Kn * T[bulk] ** 0.5 / Pr
    assert np.mean(q[bulk, 1]) == pytest.approx(np.mean(-kappa * dTdy), rel=2e-2)
    np.testing.assert_allclose(q[bulk, 1], np.mean(q[bulk, 1]), rtol=2e-2)
    assert np.abs(u[:, 0]).max() < 1e-14          # nothing drives a flow along the walls


@pytest.mark.slow
def test_poiseuille_stress_gradient_balances_force(d2q37):
    vs, ny, Kn, gx = d2q37, 16, 0.1, 0.02
    prob = L.Problem(vs, (1, ny), Kn=Kn, Pr=2 / 3, walls=True, g=(gx, 0, 0))
    M = prob.M
    f = L.equilibrium_state(prob, np.ones(M), np.zeros((M, 2)), np.ones(M))
    f = L.run(f, prob, 1500)
    rho, u, T, s, q = L.macroscopic(f, prob)
    y = (np.arange(ny) + 0.5) / ny
    bulk = slice(3, ny - 3)
    # momentum balance d sigma_xy / dy = rho g_x
    slope = np.polyfit(y[bulk], s[bulk, 0, 1], 1)[0]
    assert slope == pytest.approx(np.mean(rho) * gx, rel=2e-2)
    np.testing.assert_allclose(u[:, 0], u[::-1, 0], atol=1e-13)
    assert u[ny // 2, 0] > u[0, 0] > 0


def _wave_rates(prob, nsteps, fit_from):
    nx = prob.dims[0]
    x = np.arange(nx)
    k = 2 * np.pi
    u = np.zeros((prob.M, prob.D))
    u[:, 1] = 1e-4 * np.sin(k * x / nx)
    T = 1.0 + 1e-3 * np.cos(k * x / nx)
    f = L.equilibrium_state(prob, 1.0 / T, u, T)
    su, sT = [], []
    for _ in range(nsteps):
        _, uu, TT, _, _ = L.macroscopic(f, prob)
        su.append(2 * np.mean(uu[:, 1] * np.sin(k * x / nx)))
        sT.append(2 * np.mean((TT - 1) * np.cos(k * x / nx)))
        f = L.step(f, prob)
    t = np.arange(nsteps) * prob.dt
    sl = slice(fit_from, nsteps)
    ru = -np.polyfit(t[sl], np.log(su[sl]), 1)[0]
    rT = -np.polyfit(t[sl], np.log(sT[sl]), 1)[0]
    return ru / (prob.Kn * k * k), rT / (prob.Kn / prob.Pr * k * k)


@pytest.mark.slow
@pytest.mark.parametrize("Pr", [2 / 3, 1.0])
def test_shear_and_thermal_waves_decay_at_nu_and_nu_over_pr(d2q37, Pr):
    coarse = _wave_rates(L.Problem(d2q37, (32, 1), Kn=0.02, Pr=Pr), 400, 100)
    fine = _wave_rates(L.Problem(d2q37, (64, 1), Kn=0.01, Pr=Pr), 800, 200)
    for c_, f_ in zip(coarse, fine):
        assert abs(f_ - 1) < 1.5e-2
        assert abs(c_ - 1) < 4e-2
        assert abs(f_ - 1) < 0.45 * abs(c_ - 1)      # second-order convergence in k Kn


@pytest.mark.slow
def test_euler_scheme_has_the_first_order_viscosity(d2q37):
    # forward Euler along characteristics at Courant number one: the effective
    # viscosity and conductivity are reduced by (1 - y/2) and (1 - x/2)
    prob = L.Problem(d2q37, (32, 1), Kn=0.02, Pr=2 / 3, scheme="euler")
    ru, rT = _wave_rates(prob, 400, 100)
    y = prob.dt / prob.Kn
    x = prob.Pr * y
    assert ru == pytest.approx(1 - y / 2, abs=0.02)
    assert rT == pytest.approx(1 - x / 2, abs=0.03)


@pytest.mark.slow
def test_d3q39_shear_wave_viscosity(d3q39):
    ru, rT = _wave_rates(L.Problem(d3q39, (32, 1, 1), Kn=0.02, Pr=2 / 3), 400, 100)
    assert abs(ru - 1) < 4e-2
    assert abs(rT - 1) < 6e-2
