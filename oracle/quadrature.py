"""Discrete velocity sets for the oracle (test infrastructure only).

The paper (Sec. 2.2) discretises velocity space with a Gauss-Hermite quadrature
for the weight function omega(c) = (2 pi)^(-D/2) exp(-c^2/2): the abscissae
c_alpha and weights w_alpha must integrate polynomials exactly up to a degree
of at least 2N for an N-th order Hermite expansion (9 or more for N = 4).
It gives the 1-D rule (roots of He_n, weights from eq. weight) and points to
other constructions for multi-dimensional sets without printing one.

This module provides

* ``hermite_rule_1d(n)`` - the 1-D rule of eq. weight;
* ``d2q37()`` / ``d3q39()`` - on-lattice sets c_alpha = r e_alpha with integer
  e_alpha. The velocity shells are fixed; the scale r and one weight per shell
  are found by matching every even velocity moment of the set to the moment of
  the Gaussian weight function up to the set's even degree (odd moments vanish
  by the symmetry of the shells). D2Q37 comes out exact to degree 9 (the
  minimum the paper requires for N = 4), D3Q39 to degree 7 (enough for N = 3).

Velocity order (an interface convention shared with the library's population
I/O): index 0 is the rest velocity; indices 1..P are the vectors whose first
non-zero component is positive, sorted by |e|^2 and then by descending tuple
order; index alpha + P holds -e_alpha.
"""

from fractions import Fraction
from itertools import permutations, product
from math import factorial

import mpmath as mp
import numpy as np
from numpy.polynomial import hermite_e as He


def hermite_rule_1d(n):
    """1-D Gauss-Hermite rule of Sec. 2.2: abscissae are the n roots of the
    probabilists' Hermite polynomial He_n, weights from eq. weight,
    w_alpha = n! / [n He_{n-1}(c_alpha)]^2 (normalised to the weight function
    exp(-c^2/2)/sqrt(2 pi), so the weights sum to one).

    The library root finder's roots are refined by Newton's method on He_n in
    50-digit arithmetic and both formulas are evaluated there, so abscissae
    and weights are the correctly rounded doubles (in plain double precision
    the outer weight of n = 6 would carry a relative error near 2e-14)."""

    def he(k, x):                                   # He_{k+1} = x He_k - k He_{k-1}
        p0, p1 = mp.mpf(1), x
        if k == 0:
            return p0
        for j in range(1, k):
            p0, p1 = p1, x * p1 - j * p0
        return p1

    start = np.sort(He.hermeroots([0] * n + [1]))
    roots, w = np.empty(n), np.empty(n)
    with mp.workdps(50):
        for i, x0 in enumerate(start):
            x = mp.mpf(float(x0))
            for _ in range(8):                      # He_n' = n He_{n-1}
                x = x - he(n, x) / (n * he(n - 1, x))
            roots[i] = float(x)
            w[i] = float(mp.factorial(n) / (n * he(n - 1, x)) ** 2)
    return roots, w


def _orbit(v):
    """All distinct vectors obtained from v by permuting and sign-flipping its
    components (the hypercubic orbit of one shell)."""
    out = set()
    for p in permutations(v):
        for s in product((1, -1), repeat=len(v)):
            out.add(tuple(int(a * b) for a, b in zip(p, s)))
    return sorted(out)


def _canonical_order(vectors):
    """Rest first, then the representatives (first non-zero component
    positive) sorted by |e|^2 then descending tuple order, then their
    opposites in the same order."""
    D = len(vectors[0])
    rest = tuple([0] * D)
    reps = []
    for v in vectors:
        nz = [a for a in v if a != 0]
        if nz and nz[0] > 0:
            reps.append(v)
    reps.sort(key=lambda v: (sum(a * a for a in v), tuple(-a for a in v)))
    opp = [tuple(-a for a in v) for v in reps]
    return [rest] + reps + opp


def _double_factorial_odd(k):
    """(k-1)!! for even k: the k-th moment of the 1-D standard Gaussian."""
    out = 1
    for m in range(k - 1, 0, -2):
        out *= m
    return out


def _even_multi_indices(D, max_degree):
    """Sorted multi-indices (a_1 >= ... >= a_D >= 0) with 2*sum(a) <= max_degree;
    by the hypercubic symmetry of the shells these are the independent
    even-moment conditions."""
    out = []
    for total in range(0, max_degree // 2 + 1):
        for a in product(range(total + 1), repeat=D):
            if sum(a) == total and list(a) == sorted(a, reverse=True):
                out.append(a)
    return out


def moment_matched_set(shells, degree):
    """Solve for the scale r and the shell weights of a symmetric on-lattice
    set so that sum_alpha w_alpha c_alpha^m equals the Gaussian moment for every
    even monomial of degree <= degree (odd ones vanish by symmetry).

    With c = r e the conditions read  A W = G * t^{|a|},  t = r^{-2}, where A
    holds the integer shell sums of e^{2a}. There is one more condition than
    shell weights, so the right-hand side has to lie in the column space of A:
    projecting onto the (exact, rational) left null vector of A gives a
    polynomial in t whose real positive roots are the candidate scales; the
    accepted root is the one whose weights are all positive. Roots and weights
    are computed with 40 significant digits (mpmath) and then rounded to
    float64.
    """
    mp.mp.dps = 40
    D = len(shells[0])
    orbits = [_orbit(s) for s in shells]
    conds = _even_multi_indices(D, degree - (degree % 2))
    nc, ns = len(conds), len(shells)
    if nc != ns + 1:
        raise ValueError("moment matching expects one more condition than shells")
    A = [[0] * ns for _ in range(nc)]
    G = [0] * nc
    deg = [0] * nc
    for k, a in enumerate(conds):
        G[k] = int(np.prod([_double_factorial_odd(2 * ai) for ai in a]))
        deg[k] = sum(a)
        for s, orb in enumerate(orbits):
            A[k][s] = sum(int(np.prod([e[i] ** (2 * a[i]) for i in range(D)]))
                          for e in orb)
    # exact left null vector n (n^T A = 0) by rational elimination of A^T
    M = [[Fraction(A[k][s]) for k in range(nc)] for s in range(ns)]
    piv_cols, row = [], 0
    for col in range(nc):
        p = next((i for i in range(row, ns) if M[i][col] != 0), None)
        if p is None:
            continue
        M[row], M[p] = M[p], M[row]
        pv = M[row][col]
        M[row] = [x / pv for x in M[row]]
        for i in range(ns):
            if i != row and M[i][col] != 0:
                fct = M[i][col]
                M[i] = [x - fct * y for x, y in zip(M[i], M[row])]
        piv_cols.append(col)
        row += 1
    free = [c for c in range(nc) if c not in piv_cols]
    if len(free) != 1:
        raise ValueError("moment matrix does not have a one-dimensional left null space")
    nvec = [Fraction(0)] * nc
    nvec[free[0]] = Fraction(1)
    for i, c in enumerate(piv_cols):
        nvec[c] = -M[i][free[0]]
    poly = [Fraction(0)] * (max(deg) + 1)          # coefficients of t^k
    for k in range(nc):
        poly[deg[k]] += nvec[k] * G[k]
    coeffs = [mp.mpf(x.numerator) / x.denominator for x in poly[::-1]]
    roots = mp.polyroots(coeffs, maxsteps=200, extraprec=200)
    # ns linearly independent conditions (greedy, exact rank test)
    rows, basis = [], []
    for k in range(nc):
        v = [Fraction(x) for x in A[k]]
        for bv, pc in basis:
            if v[pc] != 0:
                f = v[pc] / bv[pc]
                v = [x - f * y for x, y in zip(v, bv)]
        pc = next((i for i in range(ns) if v[i] != 0), None)
        if pc is not None:
            basis.append((v, pc))
            rows.append(k)
    if len(rows) != ns:
        raise ValueError("shell weights are not determined by the moment conditions")
    Am = mp.matrix([[A[k][s] for s in range(ns)] for k in rows])
    found = []
    for t in roots:
        if abs(mp.im(t)) > mp.mpf("1e-25") or mp.re(t) <= 0:
            continue
        t = mp.re(t)
        W = mp.lu_solve(Am, mp.matrix([G[k] * t ** deg[k] for k in rows]))
        resid = max(abs(sum(A[k][s] * W[s] for s in range(ns)) - G[k] * t ** deg[k])
                    for k in range(nc))
        if all(W[s] > 0 for s in range(ns)) and resid < mp.mpf("1e-25"):
            found.append((1 / mp.sqrt(t), W))
    if len(found) != 1:
        raise ValueError(f"expected one admissible root, found {len(found)}")
    r, W = found[0]
    vectors = [v for orb in orbits for v in orb]
    weight_of = {}
    for orb, ws in zip(orbits, W):
        for v in orb:
            weight_of[v] = float(ws)
    order = _canonical_order(vectors)
    e = np.array(order, dtype=np.int64)
    w = np.array([weight_of[v] for v in order])
    return float(r), e, w


SHELLS_D2Q37 = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1)]
SHELLS_D3Q39 = [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 0, 0), (2, 2, 0), (3, 0, 0)]


class VelocitySet:
    """c_alpha = r e_alpha, weights w_alpha, exactness degree, Hermite order N."""

    def __init__(self, name, r, e, w, degree, order_N):
        self.name = name
        self.r = float(r)
        self.e = e                      # (Q, D) int64
        self.w = w                      # (Q,) float64
        self.c = r * e.astype(np.float64)
        self.Q, self.D = e.shape
        self.degree = degree
        self.N = order_N
        P = (self.Q - 1) // 2
        self.opposite = np.concatenate([[0], np.arange(P + 1, self.Q),
                                        np.arange(1, P + 1)])


def d2q37():
    """37-velocity 2-D set, exact to degree 9; carries the N = 4 expansion."""
    r, e, w = moment_matched_set(SHELLS_D2Q37, 9)
    return VelocitySet("D2Q37", r, e, w, 9, 4)


def d3q39():
    """39-velocity 3-D set, exact to degree 7; carries the N = 3 expansion."""
    r, e, w = moment_matched_set(SHELLS_D3Q39, 7)
    return VelocitySet("D3Q39", r, e, w, 7, 3)


def velocity_set(name):
    return {"D2Q37": d2q37, "D3Q39": d3q39}[name]()
