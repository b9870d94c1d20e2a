"""GPU parity of the paper's own scheme (Sec. 3.1): forward Euler with TVD
minmod flux differences on the 6-point Gauss-Hermite product set D2Q36,
periodic in x and y, through the C ABI against the FP64 oracle
(oracle/offlattice.py) on the same seeded inputs.

Gates: the moment fields use the scale- and signal-relative metrics of the
on-lattice parity tests (tests/helpers.py); FP64 populations are compared
element by element. The flux limiter is continuous in its arguments, so a
limiter branch taken differently by FP32 or FP16 rounding moves a flux by a
rounding-sized amount only.
"""

import numpy as np
import pytest

from oracle import lattice as OL
from oracle import offlattice as OF
from tests import helpers as H

pytestmark = pytest.mark.gpu

SETS = {"D2Q16GH": OF.ProductSet(4, 2, 3), "D2Q36GH": OF.ProductSet(6, 2, 4), "D2Q64GH": OF.ProductSet(8, 2, 4)}
GH = SETS["D2Q36GH"]                     # the paper's set

# (nx, ny): idle slots in every row, several wavefronts per row, a thin
# periodic strip (x wraps inside every wavefront), one-cell rows (1-D in y)
CASES = [(70, 9), (200, 12), (5, 40), (1, 33)]


def _fields(f, prob):
    rho, u, T, sigma, q = OF.macroscopic(f, prob)
    return {"rho": rho, "u": u.T.copy(), "T": T,
            "sigma": np.array([sigma[:, 0, 0], sigma[:, 0, 1], sigma[:, 1, 1]]), "q": q.T.copy()}


WALLS = dict(T=(0.98, 1.04), u=(-0.04, 0.05))


def _pair(dims, storage, cfl=0.5, Kn=0.005, Pr=2 / 3, g=(0.02, -0.01), seed=5, amp=0.02, walls=None,
          velset="D2Q36GH"):
    """GPU lattice and oracle problem with the same seeded start; walls =
    dict(T=(T_lo, T_hi), u=(u_lo, u_hi)) puts diffuse walls on the first
    and last rows."""
    from paper_1209_6548_amd import TVDLattice
    # N_L is the longer extent, so that dt = CFL dx / max|c| keeps the
    # forward-Euler collision stable on thin strips too
    n_ref = max(dims)
    kw = {}
    if walls:
        kw = dict(walls=True, wall_lo=OL.Wall(walls["T"][0], (walls["u"][0], 0.0, 0.0)),
                  wall_hi=OL.Wall(walls["T"][1], (walls["u"][1], 0.0, 0.0)))
    vs = SETS[velset]
    prob = OF.TVDProblem(vs, dims, Kn=Kn, Pr=Pr, g=g + (0.0,), cfl=cfl, n_ref=n_ref, **kw)
    lat = TVDLattice(dims[0], dims[1], storage=storage, cfl=cfl, n_ref=n_ref, walls=bool(walls), velset=velset)
    assert lat.dt == pytest.approx(prob.dt, rel=1e-14)
    lat.set_gas(Kn, Pr)
    lat.set_body_force(g)
    if walls:
        for side in (0, 1):
            lat.set_wall(side, walls["T"][side], (walls["u"][side], 0.0, 0.0))
    rho, u, T, xi, amp = H.init_fields(None, prob.M, 2, vs.Q, seed=seed, amp=amp)
    lat.init_equilibrium(rho, u, T, xi, amp)
    f = OF.equilibrium_state(prob, rho, u.T, T, xi, amp)
    return lat, prob, f


@pytest.mark.parametrize("dims", CASES)
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_tvd_step_parity(dims, storage):
    lat, prob, f = _pair(dims, storage)
    h0 = lat.get_populations()
    # |h| reaches ~10 at the outer velocities (small weights): FP64 rounding
    # of the start is ~1e-15 there
    np.testing.assert_allclose(h0, f / GH.w[:, None] - 1.0,
                               atol={"f64": 1e-14, "f32": 1e-7, "f16": 1e-3}[storage], rtol=0)
    steps = 12
    lat.step(steps)
    f = OF.run(f, prob, steps)
    assert lat.steps_done == steps
    ea, er = H.assert_parity(lat.read_moments(), _fields(f, prob), storage)
    print(dims, storage, "scale", max(ea.values()), "signal", max(er.values()))
    if storage == "f64":
        h, ho = lat.get_populations(), f / GH.w[:, None] - 1.0
        assert np.abs(h - ho).max() / np.abs(ho).max() < 1e-12


@pytest.mark.parametrize("dims", CASES)
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_tvd_walls_parity(dims, storage):
    """Sec. 3.2 walls on rows 0 and ny - 1 (moving, at different
    temperatures): ghost rows, re-emission after every step."""
    if dims[1] < 3:
        pytest.skip("a channel needs three rows")
    lat, prob, f = _pair(dims, storage, walls=WALLS)
    lat.step(12)
    f = OF.run(f, prob, 12)
    ea, er = H.assert_parity(lat.read_moments(), _fields(f, prob), storage)
    print(dims, storage, "walls: scale", max(ea.values()), "signal", max(er.values()))
    if storage == "f64":
        h, ho = lat.get_populations(), f / GH.w[:, None] - 1.0
        assert np.abs(h - ho).max() / np.abs(ho).max() < 1e-12


@pytest.mark.parametrize("case", ["couette", "fourier"])
def test_tvd_walls_long_run_fp64(case):
    # 300 steps of a 1 x 13 channel from rest: the profiles of Sec. 4
    # build up through the walls alone
    walls = dict(T=(1.0, 1.0), u=(-0.05, 0.05)) if case == "couette" else dict(T=(1.0, 1.1), u=(0.0, 0.0))
    lat, prob, _ = _pair((1, 13), "f64", cfl=0.9, Kn=0.1, g=(0.0, 0.0), amp=0.0, walls=walls)
    lat.init_equilibrium()
    M = prob.M
    f = OF.equilibrium_state(prob, np.ones(M), np.zeros((M, 2)), np.ones(M))
    lat.step(300)
    f = OF.run(f, prob, 300)
    H.assert_parity(lat.read_moments(), _fields(f, prob), "f64")
    h, ho = lat.get_populations(), f / GH.w[:, None] - 1.0
    assert np.abs(h - ho).max() / np.abs(ho).max() < 1e-12


def test_tvd_walls_wider_channel_fp32():
    # several wavefronts per row, a ragged row end, 3 steps
    lat, prob, f = _pair((520, 40), "f32", walls=WALLS, seed=7)
    lat.step(3)
    f = OF.run(f, prob, 3)
    H.assert_parity(lat.read_moments(), _fields(f, prob), "f32")


@pytest.mark.parametrize("velset", ["D2Q16GH", "D2Q64GH"])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_tvd_other_sets_parity(velset, walls, storage):
    """The 4- and 8-point product sets (N = 3 and 4) through the same
    kernels: 12 steps on a ragged 70 x 9 grid, periodic or walled."""
    lat, prob, f = _pair((70, 9), storage, walls=WALLS if walls else None, velset=velset)
    lat.step(12)
    f = OF.run(f, prob, 12)
    ea, er = H.assert_parity(lat.read_moments(), _fields(f, prob), storage)
    print(velset, walls, storage, "scale", max(ea.values()), "signal", max(er.values()))
    if storage == "f64":
        h, ho = lat.get_populations(), f / prob.vs.w[:, None] - 1.0
        assert np.abs(h - ho).max() / np.abs(ho).max() < 1e-12


def test_tvd_velocity_set_study():
    """The velocity-set convergence study on the GPU: Couette flow at
    Kn = 0.5 to t = 10 with the 4-, 6- and 8-point sets in FP64. Each run
    matches the oracle's, and the slip and shear stress change by less with
    the richer set."""
    slip, sxy = [], []
    for velset in ("D2Q16GH", "D2Q36GH", "D2Q64GH"):
        walls = dict(T=(1.0, 1.0), u=(-0.05, 0.05))
        lat, prob, _ = _pair((1, 13), "f64", cfl=0.9, Kn=0.5, g=(0.0, 0.0), amp=0.0, walls=walls, velset=velset)
        M = prob.M
        lat.init_equilibrium()
        f = OF.equilibrium_state(prob, np.ones(M), np.zeros((M, 2)), np.ones(M))
        steps = int(round(10.0 / prob.dt))
        lat.step(steps)
        f = OF.run(f, prob, steps)
        g = lat.read_moments()
        H.assert_parity(g, _fields(f, prob), "f64")
        slip.append(0.05 - g["u"][0][-1])
        sxy.append(g["sigma"][1][1:-1].mean())
        print(velset, steps, "slip", slip[-1], "sigma_xy", sxy[-1])
    for seq in (slip, sxy):
        d = np.abs(np.diff(seq))
        assert d[1] < 0.7 * d[0], seq


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_tvd_limiter_active_on_a_shock_tube(storage):
    # a density and temperature jump along y (1-D Riemann problem in a
    # periodic box): the limiter clips at the two discontinuities
    from paper_1209_6548_amd import TVDLattice
    nx, ny = 3, 64
    prob = OF.TVDProblem(GH, (nx, ny), Kn=0.01, Pr=1.0, cfl=0.8, n_ref=ny)
    M = prob.M
    y = np.arange(M) // nx
    left = (y >= ny // 4) & (y < 3 * ny // 4)
    rho = np.where(left, 1.2, 0.9)
    T = np.where(left, 1.1, 0.95)
    u = np.zeros((2, M))
    lat = TVDLattice(nx, ny, storage=storage, cfl=0.8, n_ref=ny)
    lat.set_gas(0.01, 1.0)
    lat.init_equilibrium(rho, u, T)
    f = OF.equilibrium_state(prob, rho, u.T, T)
    lat.step(40)
    f = OF.run(f, prob, 40)
    orc = _fields(f, prob)
    H.assert_parity(lat.read_moments(), orc, storage)
    # the flow is one-dimensional: every row holds one value per field
    g = lat.read_moments()
    assert np.ptp(g["rho"].reshape(ny, nx), axis=1).max() == 0.0
    assert np.abs(orc["u"][1]).max() > 1e-3


def test_tvd_uniform_equilibrium_stays_uniform_under_force():
    # a uniform gas has no flux difference; the force only accelerates it
    from paper_1209_6548_amd import TVDLattice
    nx, ny = 40, 7
    prob = OF.TVDProblem(GH, (nx, ny), Kn=0.1, Pr=2 / 3, g=(0.05, 0.0, 0.0), cfl=0.5)
    lat = TVDLattice(nx, ny, storage="f64", cfl=0.5)
    lat.set_gas(0.1, 2 / 3)
    lat.set_body_force((0.05, 0.0))
    lat.init_equilibrium()
    lat.step(10)
    f = OF.run(OF.equilibrium_state(prob, np.ones(prob.M), np.zeros((prob.M, 2)), np.ones(prob.M)), prob, 10)
    g = lat.read_moments()
    for k in ("rho", "T"):
        assert np.ptp(g[k]) < 1e-15
    np.testing.assert_allclose(g["u"][0], 0.05 * 10 * prob.dt, rtol=1e-12)
    H.assert_parity(g, _fields(f, prob), "f64")


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_tvd_conserves_mass_momentum_energy(storage):
    # flux form telescopes on a periodic grid and the collision keeps the
    # collision invariants: the totals drift only by rounding
    lat, prob, f = _pair((96, 40), storage, g=(0.0, 0.0))
    def totals():
        m = lat.read_moments()
        rho, u, T = m["rho"], m["u"], m["T"]
        return np.array([rho.sum(), (rho * u[0]).sum(), (rho * u[1]).sum(),
                         (rho * (T * 2 + (u ** 2).sum(0))).sum()])
    t0 = totals()
    lat.step(50)
    t1 = totals()
    tol = {"f64": 1e-12, "f32": 2e-5}[storage] * prob.M
    np.testing.assert_allclose(t1, t0, atol=tol, rtol=0)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_tvd_restart_is_bit_identical(storage):
    lat, prob, _ = _pair((70, 9), storage)
    lat.step(5)
    h = lat.get_populations()
    lat.step(4)
    a = lat.get_populations()
    lat.set_populations(h)
    assert lat.steps_done == 0
    lat.step(4)
    np.testing.assert_array_equal(lat.get_populations(), a)


def _patch_step(pop, w, dims, cells, prob_full):
    """One oracle step of sampled cells of a big periodic grid: the update of
    cell (x, y) reads only (x +- 2, y) and (x, y +- 2), so the oracle steps
    the 5 x 5 periodic patch around it and keeps the center."""
    nx, ny = dims
    out = np.empty((GH.Q, len(cells)))
    sub = OF.TVDProblem(GH, (5, 5), Kn=prob_full.Kn, Pr=prob_full.Pr, varpi=prob_full.varpi,
                        g=prob_full.g, cfl=prob_full.cfl, n_ref=prob_full.n_ref)
    assert sub.dt == prob_full.dt
    for k, cell in enumerate(cells):
        y, x = divmod(int(cell), nx)
        ys = (y + np.arange(-2, 3)) % ny
        xs = (x + np.arange(-2, 3)) % nx
        idx = (ys[:, None] * nx + xs[None, :]).ravel()
        fp = w[:, None] * (1.0 + pop[:, idx])
        out[:, k] = OF.step(fp, sub)[:, 12] / w - 1.0
    return out


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_tvd_full_size_sampled_cells(storage):
    # the benchmark size (1024 x 1024): one step, sampled cells (including
    # every corner and row end) against the oracle stepped on their patches
    lat, prob, _ = _pair((1024, 1024), storage, seed=9)
    h0 = lat.get_populations()
    lat.step(1)
    h1 = lat.get_populations()
    nx, ny = prob.dims
    rng = np.random.default_rng(3)
    edge = [0, nx - 1, nx * (ny - 1), nx * ny - 1, nx * 511, nx * 511 + nx - 1, 63, 64, 65]
    cells = np.concatenate([edge, rng.integers(0, nx * ny, 200)])
    exp = _patch_step(h0, GH.w, prob.dims, cells, prob)
    got = h1[:, cells]
    tol = {"f64": 1e-13, "f32": 1e-6}[storage]
    np.testing.assert_allclose(got, exp, atol=tol, rtol=0)


def test_tvd_rejects_bad_arguments():
    from paper_1209_6548_amd import EsbgkError, TVDLattice
    with pytest.raises(EsbgkError):
        TVDLattice(8, 8, storage="f32", cfl=1.5)
    with pytest.raises(EsbgkError):
        TVDLattice(8, 8, storage="f32", cfl=0.0)
    with pytest.raises(EsbgkError):
        TVDLattice(8, 2, storage="f32", walls=True)     # a channel needs three rows
    lat = TVDLattice(8, 8, storage="f32")
    with pytest.raises(EsbgkError):
        lat.set_wall(0, 1.0)            # no walls on this lattice
    with pytest.raises(EsbgkError):
        lat.step(1)                     # no state yet
    with pytest.raises(EsbgkError):
        lat.set_gas(-1.0, 1.0)
    with pytest.raises(EsbgkError):
        lat.set_gas(0.1, 0.5)           # Pr < 2/3
    with pytest.raises(EsbgkError):
        lat.set_gas(1e-4, 1.0)          # forward Euler unstable: dt/tau >= 2
    with pytest.raises(EsbgkError):
        lat.set_body_force((np.nan, 0.0))
    lat.init_equilibrium()
    with pytest.raises(EsbgkError):
        lat.step(-1)
    lat.step(1)
    assert lat.steps_done == 1
    ch = TVDLattice(8, 8, storage="f32", walls=True)
    for bad in ((2, 1.0, (0, 0, 0)), (0, -1.0, (0, 0, 0)), (0, 1.0, (0.0, 0.1, 0.0)), (1, np.inf, (0, 0, 0))):
        with pytest.raises(EsbgkError):
            ch.set_wall(*bad)
