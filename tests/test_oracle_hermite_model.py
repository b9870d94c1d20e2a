"""Pins for the oracle's Hermite basis and ES-BGK model pieces (Sec. 2.1-2.2,
eq. feq0 of Sec. 3.2). Every expected value comes from an independent route:
numpy's HermiteE polynomials, a 20-point-per-axis Gauss-Hermite integral of
the anisotropic Gaussian, finite differences of the continuous expansion, or
the other closed form printed in the paper."""

from itertools import product
from math import factorial

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

from oracle import hermite, model


def test_chi_reduces_to_he_n_along_each_axis():
    rng = np.random.default_rng(0)
    for D in (2, 3):
        c = rng.normal(size=(7, D)) * 1.5
        for n in range(5):
            x = hermite.chi(c, n)
            for a in range(D):
                idx = (slice(None),) + (a,) * n
                np.testing.assert_allclose(x[idx], He.hermeval(c[:, a], [0] * n + [1]),
                                           rtol=1e-13, atol=1e-12)


def test_chi_is_symmetric_and_satisfies_the_recurrence():
    # c_i chi^n_J = chi^(n+1)_{iJ} + sum_k delta_{i j_k} chi^(n-1)_{J without j_k}
    rng = np.random.default_rng(1)
    D = 3
    c = rng.normal(size=(5, D))
    d = np.eye(D)
    for n in range(1, 4):
        xn, xp, xm = hermite.chi(c, n), hermite.chi(c, n + 1), hermite.chi(c, n - 1)
        for J in product(range(D), repeat=n):
            for i in range(D):
                rhs = xp[(slice(None), i) + J].copy()
                for k in range(n):
                    if i == J[k]:
                        rest = J[:k] + J[k + 1:]
                        rhs += xm[(slice(None),) + rest]
                np.testing.assert_allclose(c[:, i] * xn[(slice(None),) + J], rhs, atol=1e-12)
        for J in product(range(D), repeat=n + 1):
            for perm in [J[::-1], J[1:] + J[:1]]:
                np.testing.assert_allclose(xp[(slice(None),) + J], xp[(slice(None),) + perm])


def _product_rule(D, npts=20):
    z, wz = He.hermegauss(npts)
    wz = wz / np.sqrt(2 * np.pi)
    pts = np.array(list(product(z, repeat=D)))
    wts = np.prod(np.array(list(product(wz, repeat=D))), axis=1)
    return pts, wts


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_chi_orthogonality_on_the_lattice(name):
    from oracle import quadrature
    vs = quadrature.velocity_set(name)
    pts, wts = _product_rule(vs.D, 8)          # exact to degree 15
    for m in range(5):
        for n in range(5):
            if m + n > vs.degree:
                continue
            lat = np.einsum("q,qa,qb->ab", vs.w, hermite.chi(vs.c, m).reshape(vs.Q, -1),
                            hermite.chi(vs.c, n).reshape(vs.Q, -1))
            ref = np.einsum("q,qa,qb->ab", wts, hermite.chi(pts, m).reshape(len(wts), -1),
                            hermite.chi(pts, n).reshape(len(wts), -1))
            np.testing.assert_allclose(lat, ref, atol=2e-12)


def _random_state(D, rng, M=4, amp=0.2):
    rho = 1.0 + 0.1 * rng.uniform(-1, 1, M)
    u = amp * rng.uniform(-1, 1, (M, D))
    T = 1.0 + 0.1 * rng.uniform(-1, 1, M)
    A = rng.uniform(-1, 1, (M, D, D)) * 0.1
    sigma = A + A.transpose(0, 2, 1)
    sigma -= np.trace(sigma, axis1=1, axis2=2)[:, None, None] / D * np.eye(D)
    return rho, u, T, sigma


def _gaussian_raw_moments(rho, u, lam, order):
    """Raw moments of rho N(u, lam) by a product Gauss-Hermite rule in the
    whitened variable (c = u + L z, lam = L L^T)."""
    D = u.shape[0]
    pts, wts = _product_rule(D, 20)
    L = np.linalg.cholesky(lam)
    c = u[None, :] + pts @ L.T
    out = []
    for n in range(order + 1):
        if n == 0:
            out.append(rho * wts.sum())
            continue
        letters = "ijkl"[:n]
        ops = ",".join(["p"] + [f"p{a}" for a in letters])
        out.append(rho * np.einsum(f"{ops}->{letters}", wts, *([c] * n)))
    return out


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_es_projection_reproduces_gaussian_moments_up_to_order_N(name):
    from oracle import quadrature
    vs = quadrature.velocity_set(name)
    rng = np.random.default_rng(2)
    rho, u, T, sigma = _random_state(vs.D, rng)
    for b in (-0.5, 0.0, 0.6):
        lam = model.es_tensor(T, sigma, rho, b)
        f = model.hermite_projection(model.es_coefficients(rho, u, lam, vs.N), vs.c, vs.w)
        mom = model.raw_moments(f, vs.c, min(vs.N, 3))
        for m in range(rho.shape[0]):
            ref = _gaussian_raw_moments(rho[m], u[m], lam[m], min(vs.N, 3))
            for n in range(len(ref)):
                np.testing.assert_allclose(mom[n][m], ref[n], atol=1e-12)
        if vs.N == 4:
            m4 = np.einsum("qm,qi,qj,qk,ql->mijkl", f, *([vs.c] * 4))
            for m in range(rho.shape[0]):
                pts, wts = _product_rule(vs.D, 20)
                Lc = np.linalg.cholesky(lam[m])
                c = u[m][None, :] + pts @ Lc.T
                ref4 = rho[m] * np.einsum("p,pi,pj,pk,pl->ijkl", wts, c, c, c, c)
                np.testing.assert_allclose(m4[m], ref4, atol=1e-11)


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_es_with_zero_stress_equals_truncated_maxwellian(name):
    from oracle import quadrature
    vs = quadrature.velocity_set(name)
    rng = np.random.default_rng(3)
    rho, u, T, sigma = _random_state(vs.D, rng)
    lam = model.es_tensor(T, 0.0 * sigma, rho, -0.5)
    f_es = model.hermite_projection(model.es_coefficients(rho, u, lam, vs.N), vs.c, vs.w)
    S = model.truncated_maxwellian(rho, u, T, vs.c, vs.w, vs.N)
    np.testing.assert_allclose(f_es, S, rtol=1e-13, atol=1e-15)
    # at rest and T = 1 it is w_alpha rho
    S0 = model.truncated_maxwellian(rho, 0 * u, np.ones_like(T), vs.c, vs.w, vs.N)
    np.testing.assert_allclose(S0, vs.w[:, None] * rho[None, :], rtol=1e-15)


def test_truncated_maxwellian_with_stress_differs(d2q37):
    # guards the test above against a projection that ignores sigma
    rng = np.random.default_rng(4)
    rho, u, T, sigma = _random_state(2, rng)
    lam = model.es_tensor(T, sigma, rho, -0.5)
    f_es = model.hermite_projection(model.es_coefficients(rho, u, lam, 4), d2q37.c, d2q37.w)
    S = model.truncated_maxwellian(rho, u, T, d2q37.c, d2q37.w, 4)
    assert np.abs(f_es - S).max() > 1e-4


def _continuous_expansion(a, c):
    """f(c)/omega(c) = sum_n (1/n!) a^(n) : chi^(n)(c), one cell."""
    total = np.zeros(c.shape[0])
    for n, an in enumerate(a):
        total += hermite.contract(an[None], hermite.chi(c, n))[:, 0] / factorial(n)
    return total


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_force_term_is_minus_g_dot_velocity_gradient(name):
    # F = -g . grad_c f for f = omega sum_{n<N} a^(n) chi^(n)/n!, checked by
    # central differences of the continuous expansion at the lattice nodes.
    from oracle import quadrature
    vs = quadrature.velocity_set(name)
    rng = np.random.default_rng(5)
    D, N = vs.D, vs.N
    a = [np.array(1.1)]
    for n in range(1, N):
        t = rng.normal(size=(D,) * n) * 0.3
        # symmetrise
        from itertools import permutations
        t = sum(np.transpose(t, p) for p in permutations(range(n))) / factorial(n)
        a.append(t)
    g = rng.normal(size=D)
    omega = lambda c: np.exp(-0.5 * np.sum(c * c, axis=1)) / (2 * np.pi) ** (D / 2)
    f = lambda c: omega(c) * _continuous_expansion(a, c)
    h = 1e-5
    grad = np.zeros((vs.Q, D))
    for i in range(D):
        dc = np.zeros(D)
        dc[i] = h
        grad[:, i] = (f(vs.c + dc) - f(vs.c - dc)) / (2 * h)
    F_cont = -(grad @ g)                                      # F(c_alpha)
    a_f = [np.atleast_1d(a[0])] + [x[None] for x in a[1:]]
    F_lat = model.force_term(g, a_f, vs.c, vs.w, N)[:, 0]     # w F / omega
    np.testing.assert_allclose(F_lat, vs.w * F_cont / omega(vs.c), rtol=1e-7, atol=1e-9)


def test_force_moments(d2q37):
    vs = d2q37
    rng = np.random.default_rng(6)
    rho, u, T, sigma = _random_state(2, rng)
    g = np.array([0.3, -0.2])
    lam = model.es_tensor(T, sigma, rho, -0.5)
    a = model.es_coefficients(rho, u, lam, 3)
    F = model.force_term(g, a, vs.c, vs.w, 4)
    np.testing.assert_allclose(F.sum(axis=0), 0, atol=1e-14)
    np.testing.assert_allclose(F.T @ vs.c, rho[:, None] * g[None, :], atol=1e-14)
    # energy source: sum F c^2 = 2 rho g.u (rate of change of rho |c|^2)
    np.testing.assert_allclose((F * np.sum(vs.c ** 2, axis=1)[:, None]).sum(axis=0),
                               2 * rho * (u @ g), atol=1e-13)


def test_macroscopic_of_a_maxwellian(d2q37, d3q39):
    for vs in (d2q37, d3q39):
        rng = np.random.default_rng(7)
        rho, u, T, _ = _random_state(vs.D, rng)
        S = model.truncated_maxwellian(rho, u, T, vs.c, vs.w, vs.N)
        r2, u2, T2, s2, q2 = model.macroscopic(S, vs.c)
        np.testing.assert_allclose(r2, rho, rtol=1e-14)
        np.testing.assert_allclose(u2, u, atol=1e-14)
        np.testing.assert_allclose(T2, T, rtol=1e-13)
        np.testing.assert_allclose(s2, 0, atol=1e-13)
        np.testing.assert_allclose(q2, 0, atol=1e-13)


def test_prandtl_relations():
    # Sec. 2.1: Pr = 1/(1-b); Sec. 4 prints Pr = 2/3 <-> b = -1/2, Pr = 1 <-> b = 0
    assert model.b_from_prandtl(2.0 / 3.0) == pytest.approx(-0.5, abs=1e-15)
    assert model.b_from_prandtl(1.0) == 0.0
    # tau = (Kn/Pr) mu/p with mu = T^varpi: Maxwell molecules (varpi = 1) give
    # a temperature-independent tau rho
    T = np.array([0.8, 1.0, 1.3])
    rho = np.array([1.0, 2.0, 0.5])
    tau = model.relaxation_time(0.1, 2.0 / 3.0, 1.0, rho, T)
    np.testing.assert_allclose(tau * rho, 0.15, rtol=1e-15)
    tau_hs = model.relaxation_time(0.1, 2.0 / 3.0, 0.5, rho, T)
    np.testing.assert_allclose(tau_hs, 0.15 / (rho * np.sqrt(T)), rtol=1e-15)
