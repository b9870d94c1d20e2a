"""GPU parity of the paper's scheme on its 3-D set D3Q216 (Sec. 3.1 with
the diffuse walls of Sec. 3.2 across z) through the C ABI against the FP64
oracle (oracle/offlattice.py) on the same seeded inputs: the 14 moment
fields with the gates of tests/helpers.py, and FP64 populations element by
element.
"""

import numpy as np
import pytest

from oracle import lattice as OL
from oracle import offlattice as OF
from tests import helpers as H

pytestmark = pytest.mark.gpu

CUBE = OF.ProductSet(6, 3, 4)
WALLS = dict(T=(0.97, 1.04), u=((-0.04, 0.02, 0.0), (0.05, -0.01, 0.0)))

# (nx, ny, nz): a slice of 48 cells (one wavefront, idle lanes), a ragged
# slice of 210 cells (4 wavefronts), rows of one cell; rows of 64 and 128
# cells (whole wavefronts: the x neighbours by lane shifts, the halo wrapping
# to the other end of the row)
CASES = [(8, 6, 5), (70, 3, 4), (1, 1, 9), (64, 5, 4), (128, 2, 3)]


def _fields(f, prob):
    rho, u, T, sigma, q = OF.macroscopic(f, prob)
    sig = np.array([sigma[:, i, j] for i in range(3) for j in range(i, 3)])
    return {"rho": rho, "u": u.T.copy(), "T": T, "sigma": sig, "q": q.T.copy()}


def _pair(dims, storage, walls=None, Kn=0.02, g=(0.02, -0.01, 0.005), seed=13, amp=0.02, cfl=0.3):
    from paper_1209_6548_amd import TVDLattice
    n_ref = max(dims)
    kw = {}
    if walls:
        kw = dict(walls=True, wall_lo=OL.Wall(walls["T"][0], walls["u"][0]),
                  wall_hi=OL.Wall(walls["T"][1], walls["u"][1]))
    prob = OF.TVDProblem(CUBE, dims, Kn=Kn, Pr=2 / 3, g=g, cfl=cfl, n_ref=n_ref, **kw)
    lat = TVDLattice(dims[0], dims[1], nz=dims[2], storage=storage, cfl=cfl, n_ref=n_ref, walls=bool(walls),
                     velset="D3Q216GH")
    assert lat.dt == pytest.approx(prob.dt, rel=1e-14)
    lat.set_gas(Kn, 2 / 3)
    lat.set_body_force(g)
    if walls:
        for side in (0, 1):
            lat.set_wall(side, walls["T"][side], walls["u"][side])
    rho, u, T, xi, amp = H.init_fields(None, prob.M, 3, CUBE.Q, seed=seed, amp=amp)
    lat.init_equilibrium(rho, u, T, xi, amp)
    f = OF.equilibrium_state(prob, rho, u.T, T, xi, amp)
    return lat, prob, f


@pytest.mark.parametrize("dims", CASES)
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_tvd3_parity(dims, walls, storage):
    lat, prob, f = _pair(dims, storage, walls=WALLS if walls else None)
    h0 = lat.get_populations()
    np.testing.assert_allclose(h0, f / CUBE.w[:, None] - 1.0,
                               atol={"f64": 1e-14, "f32": 1e-7, "f16": 1e-3}[storage], rtol=0)
    steps = 8
    lat.step(steps)
    f = OF.run(f, prob, steps)
    ea, er = H.assert_parity(lat.read_moments(), _fields(f, prob), storage)
    print(dims, walls, storage, "scale", max(ea.values()), "signal", max(er.values()))
    if storage == "f64":
        h, ho = lat.get_populations(), f / CUBE.w[:, None] - 1.0
        assert np.abs(h - ho).max() / np.abs(ho).max() < 1e-12


def test_tvd3_slab_order_fp64():
    # more than 8 bands of 8 slices (65 slices: the last band holds one), so
    # the tiles go in groups of ceil(9 / 8) = 2 of the slice's 9 chunks (552
    # cells) through all bands, the last group one chunk wide: every cell is
    # stepped once, against the oracle population by population
    dims = (23, 24, 65)
    lat, prob, f = _pair(dims, "f64", walls=WALLS)
    steps = 2
    lat.step(steps)
    f = OF.run(f, prob, steps)
    h, ho = lat.get_populations(), f / CUBE.w[:, None] - 1.0
    assert np.abs(h - ho).max() / np.abs(ho).max() < 1e-12
    H.assert_parity(lat.read_moments(), _fields(f, prob), "f64")
    lat.close()


def test_tvd3_couette_across_z_fp64():
    # the paper's 1-D setting: walls moving in x, the flow varies along z only
    walls = dict(T=(1.0, 1.0), u=((-0.05, 0.0, 0.0), (0.05, 0.0, 0.0)))
    lat, prob, _ = _pair((1, 1, 11), "f64", walls=walls, Kn=0.2, g=(0.0, 0.0, 0.0), amp=0.0, cfl=0.8)
    M = prob.M
    lat.init_equilibrium()
    f = OF.equilibrium_state(prob, np.ones(M), np.zeros((M, 3)), np.ones(M))
    lat.step(150)
    f = OF.run(f, prob, 150)
    g = lat.read_moments()
    H.assert_parity(g, _fields(f, prob), "f64")
    ux = g["u"][0]
    np.testing.assert_allclose(ux, -ux[::-1], atol=1e-14)


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_tvd3_restart_is_bit_identical(storage, walls):
    """Each level carries its cells' moment sums, formed while the step (and
    the walls' re-emission) stores it; a level set from outside gets them
    from a separate pass over the stored populations. Both must give the same
    bits: a run continued from the carried sums equals one restarted from the
    same populations, also when the body force (and with it the third
    moments) is switched off and on again between the calls."""
    lat, prob, _ = _pair((70, 3, 4), storage, walls=WALLS if walls else None)
    lat.step(3)
    h = lat.get_populations()
    lat.step(2)
    lat.set_body_force((0.0, 0.0, 0.0))
    lat.step(2)
    lat.set_body_force((0.02, -0.01, 0.005))
    lat.step(1)
    a = lat.get_populations()
    lat.set_populations(h)
    lat.step(2)
    lat.set_body_force((0.0, 0.0, 0.0))
    h2 = lat.get_populations()
    lat.set_populations(h2)
    lat.step(2)
    lat.set_body_force((0.02, -0.01, 0.005))
    lat.step(1)
    np.testing.assert_array_equal(lat.get_populations(), a)


def test_tvd3_rejects_bad_arguments():
    from paper_1209_6548_amd import EsbgkError, TVDLattice
    with pytest.raises(EsbgkError):
        TVDLattice(4, 4, nz=2, storage="f32", walls=True, velset="D3Q216GH")   # two planes across
    lat = TVDLattice(4, 4, nz=5, storage="f32", walls=True, velset="D3Q216GH")
    with pytest.raises(EsbgkError):
        lat.set_wall(0, 1.0, (0.0, 0.0, 0.1))          # across the channel
    lat.set_wall(0, 1.0, (0.0, 0.1, 0.0))              # in its plane
    with pytest.raises(EsbgkError):
        TVDLattice(4, 4, nz=2, storage="f32", velset="D2Q36GH")                # a 2-D set in 3-D
