"""Pins for the velocity-set convergence study of the paper's own scheme:
the n-point Gauss-Hermite product sets (n = 4, 6, 8, 10) and the
self-convergence of a rarefied flow as the set grows.

* Each product set integrates every monomial c_x^p c_y^q with p, q <= 2n - 1
  against the Gaussian weight exactly (eq. weight per axis) and not
  p = 2n; the roots of the 4- and 8-point rules equal their closed forms
  (He_4: x^2 = 3 -+ sqrt 6; He_8 from its quartic in x^2 solved here by
  numpy's polynomial roots, a different method than the oracle's).
* Couette flow at Kn = 0.5 between diffuse walls (Sec. 3.2), run to the same
  time t = 10 with each set: the wall slip and the shear stress change by
  less with every richer set, roughly geometrically.
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import offlattice as O


def _gauss_moment(p):
    return 0.0 if p % 2 else float(np.prod(np.arange(p - 1, 0, -2))) if p else 1.0


@pytest.mark.parametrize("n", [4, 6, 8, 10])
def test_product_set_exact_to_degree_2n_minus_1(n):
    vs = O.ProductSet(n, 2, 3 if n == 4 else 4)
    assert vs.Q == n * n and vs.P == n * n // 2
    np.testing.assert_array_equal(vs.c[vs.P:], -vs.c[:vs.P])
    c, w = vs.c, vs.w
    for p in range(2 * n):
        for q in range(2 * n):
            terms = w * c[:, 0] ** p * c[:, 1] ** q
            scale = np.abs(terms).sum()
            assert abs(terms.sum() - _gauss_moment(p) * _gauss_moment(q)) < 1e-13 * scale
    got = np.sum(w * c[:, 0] ** (2 * n))
    assert abs(got - _gauss_moment(2 * n)) > 1e-3 * _gauss_moment(2 * n)


def test_roots_of_the_four_and_eight_point_rules():
    r4 = np.unique(np.round(np.abs(O.ProductSet(4, 2, 3).c), 14))
    np.testing.assert_allclose(r4, np.sqrt([3 - np.sqrt(6), 3 + np.sqrt(6)]), rtol=1e-14)
    # He_8 = x^8 - 28 x^6 + 210 x^4 - 420 x^2 + 105
    z = np.sort(np.roots([1.0, -28.0, 210.0, -420.0, 105.0]).real)
    r8 = np.unique(np.round(np.abs(O.ProductSet(8, 2, 4).c), 13))
    np.testing.assert_allclose(r8, np.sqrt(z), rtol=1e-12)


@pytest.mark.slow
def test_couette_converges_with_the_velocity_set():
    slip, sxy = [], []
    for n in (4, 6, 8, 10):
        vs = O.ProductSet(n, 2, 3 if n == 4 else 4)
        prob = O.TVDProblem(vs, (1, 13), Kn=0.5, Pr=2 / 3, cfl=0.9, walls=True,
                            wall_lo=L.Wall(1.0, (-0.05, 0.0, 0.0)), wall_hi=L.Wall(1.0, (0.05, 0.0, 0.0)))
        M = prob.M
        f = O.equilibrium_state(prob, np.ones(M), np.zeros((M, 2)), np.ones(M))
        f = O.run(f, prob, int(round(10.0 / prob.dt)))
        rho, u, T, sigma, q = O.macroscopic(f, prob)
        slip.append(0.05 - u[-1, 0])
        sxy.append(sigma[1:-1, 0, 1].mean())
    for seq in (slip, sxy):
        d = np.abs(np.diff(seq))
        assert np.all(d[1:] < 0.7 * d[:-1]), (seq, d)
    # the paper's set (n = 6) is within 4 % (slip) and 2 % (shear stress) of the richest one
    assert abs(slip[1] / slip[3] - 1) < 0.04 and abs(sxy[1] / sxy[3] - 1) < 0.02
