"""ES-BGK model pieces in the paper's nondimensional units (test infrastructure
only). Arrays carry one leading cell axis M; velocities are rows of c (Q, D).

Units (Sec. 2.2): velocities in sqrt(R T0), temperature in T0, density in
rho0, so the state equation is p = rho T and the gas constant drops out.
"""

from math import factorial

import numpy as np

from . import hermite


def b_from_prandtl(Pr):
    """Sec. 2.1: Pr = 1/(1 - b), so b = 1 - 1/Pr; admissible -1/2 <= b <= 1."""
    return 1.0 - 1.0 / Pr


def relaxation_time(Kn, Pr, varpi, rho, T):
    """Sec. 2.2: tau = (Kn/Pr) mu/p with p = rho T and the viscosity law of
    Sec. 2.1, mu/mu0 = (T/T0)^varpi (nondimensional mu = T^varpi)."""
    mu = T ** varpi
    p = rho * T
    return (Kn / Pr) * mu / p


def es_tensor(T, sigma, rho, b):
    """Sec. 2.1, eq. cfeq: lambda_ij = R T delta_ij + b sigma_ij / rho, here
    with R T -> T (nondimensional)."""
    D = sigma.shape[-1]
    return T[:, None, None] * np.eye(D)[None] + b * sigma / rho[:, None, None]


def es_coefficients(rho, u, lam, N):
    """Closed-form Hermite coefficients a_ES^(n), n = 0..N, of the anisotropic
    Gaussian (Sec. 2.2, the equations following eq. approxfeq)."""
    D = u.shape[1]
    d = np.eye(D)
    L = lam - d[None]                                   # lambda - delta
    out = [rho.copy(), rho[:, None] * u]
    if N >= 2:
        a2 = np.einsum("mi,mj->mij", u, u) + L
        out.append(rho[:, None, None] * a2)
    if N >= 3:
        a3 = (np.einsum("mi,mj,mk->mijk", u, u, u)
              + np.einsum("mij,mk->mijk", lam, u)
              + np.einsum("mik,mj->mijk", lam, u)
              + np.einsum("mjk,mi->mijk", lam, u)
              - np.einsum("ij,mk->mijk", d, u)
              - np.einsum("ik,mj->mijk", d, u)
              - np.einsum("jk,mi->mijk", d, u))
        out.append(rho[:, None, None, None] * a3)
    if N >= 4:
        a4 = (np.einsum("mi,mj,ml,mk->mijkl", u, u, u, u)
              + np.einsum("mil,mj,mk->mijkl", L, u, u)
              + np.einsum("mij,ml,mk->mijkl", L, u, u)
              + np.einsum("mik,mj,ml->mijkl", L, u, u)
              + np.einsum("mjl,mi,mk->mijkl", L, u, u)
              + np.einsum("mjk,mi,ml->mijkl", L, u, u)
              + np.einsum("mkl,mi,mj->mijkl", L, u, u)
              + np.einsum("mij,mkl->mijkl", L, L)
              + np.einsum("mik,mjl->mijkl", L, L)
              + np.einsum("mil,mkj->mijkl", L, L))
        out.append(rho[:, None, None, None, None] * a4)
    if N >= 5:
        raise ValueError("closed forms are given up to n = 4")
    return out


def hermite_projection(coeffs, c, w):
    """eq. approxfeq evaluated at the quadrature nodes (the discrete form of
    eq. lbgk, f_alpha = w_alpha f(c_alpha)/omega(c_alpha)):
        f_alpha = w_alpha sum_n (1/n!) a^(n) : chi^(n)(c_alpha).
    Returns shape (Q, M)."""
    total = 0.0
    for n, a in enumerate(coeffs):
        total = total + hermite.contract(a, hermite.chi(c, n)) / factorial(n)
    return w[:, None] * total


def force_term(g, a_f, c, w, N):
    """Body-force expansion of Sec. 2.2,
        F = omega sum_{n=1}^{N} 1/(n-1)! (g a^(n-1)) : chi^(n),
    at the quadrature nodes (g_alpha = w_alpha F(c_alpha)/omega(c_alpha),
    eq. lbgk). a_f[k] is the k-th Hermite coefficient of the distribution
    (eq. an). Returns shape (Q, M)."""
    g = np.asarray(g, dtype=np.float64)
    total = 0.0
    for n in range(1, N + 1):
        a = a_f[n - 1]
        # (g a^(n-1))_{i j...} = g_i a^(n-1)_{j...}
        ga = np.multiply.outer(a, g)                   # (M, D^(n-1), D): index order j..., i
        ga = np.moveaxis(ga, -1, 1)                    # (M, D, D^(n-1)): i first
        total = total + hermite.contract(ga, hermite.chi(c, n)) / factorial(n - 1)
    return w[:, None] * total


def truncated_maxwellian(rho, u, T, c, w, N):
    """eq. feq0 (Sec. 3.2): f^0_alpha = rho S(T, u), written term by term.
    The first two lines are the n <= 3 Hermite terms; the last three lines are
    the n = 4 terms, kept only for N = 4. Returns shape (Q, M)."""
    D = c.shape[1]
    cu = c @ u.T                                        # (Q, M)
    uu = np.sum(u * u, axis=1)[None, :]                 # (1, M)
    cc = np.sum(c * c, axis=1)[:, None]                 # (Q, 1)
    th = (T - 1.0)[None, :]
    s = (1.0 + cu
         + 0.5 * (cu ** 2 - uu + th * (cc - D))
         + cu / 6.0 * (cu ** 2 - 3.0 * uu + 3.0 * th * (cc - D - 2)))
    if N >= 4:
        s = s + (1.0 / 24.0 * (cu ** 4 - 6.0 * cu ** 2 * uu + 3.0 * uu ** 2)
                 + th / 4.0 * ((cc - D - 2) * (cu ** 2 - uu) - 2.0 * cu ** 2)
                 + th ** 2 / 8.0 * (cc ** 2 - 2.0 * (D + 2) * cc + D * (D + 2)))
    return rho[None, :] * w[:, None] * s


def macroscopic(f, c):
    """eq. mac with the nondimensional temperature of Sec. 2.2 evaluated on the
    quadrature: rho, u, the trace-free stress sigma = sum f C_<i C_j>, the heat
    flux q = 1/2 sum f C_i C^2 and T from D rho T = sum f C^2 (C = c - u).
    f has shape (Q, M)."""
    D = c.shape[1]
    rho = f.sum(axis=0)
    u = (f.T @ c) / rho[:, None]
    C = c[:, None, :] - u[None, :, :]                   # (Q, M, D)
    CC = np.einsum("qmi,qmj->qmij", C, C)
    P = np.einsum("qm,qmij->mij", f, CC)
    trP = np.trace(P, axis1=1, axis2=2)
    T = trP / (D * rho)
    sigma = P - (trP / D)[:, None, None] * np.eye(D)[None]
    C2 = np.sum(C * C, axis=2)
    q = 0.5 * np.einsum("qm,qmi,qm->mi", f, C, C2)
    return rho, u, T, sigma, q


def raw_moments(f, c, order):
    """Raw velocity moments sum_alpha f_alpha c^n for n = 0..order; f (Q, M)."""
    out = [f.sum(axis=0), f.T @ c]
    if order >= 2:
        out.append(np.einsum("qm,qi,qj->mij", f, c, c))
    if order >= 3:
        out.append(np.einsum("qm,qi,qj,qk->mijk", f, c, c, c))
    return out

