"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs, element by element.

Tolerances (both metrics in tests/helpers.py): scale-relative 1e-12 for FP64
storage and compute, 1e-6 for FP32 deviational storage with FP32 compute and
1e-3 for FP16 deviational storage, per moment field, plus signal-relative
gates. Grids are small but span several workgroups with a ragged tail;
walls, moving walls, thermal walls and the body force are all on.
"""

import numpy as np
import pytest

from oracle import lattice as OL
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _start(cfg, lat, prob, seed=11):
    rho, u, T, xi, amp = H.init_fields(cfg, prob.M, prob.D, prob.vs.Q, seed=seed)
    lat.init_equilibrium(rho, u, T, xi, amp)
    f = OL.equilibrium_state(prob, rho, u.T, T, xi, amp)
    return f


def _run_pair(cfg, storage, steps, scheme="trapezoid"):
    prob = H.oracle_problem(cfg, scheme)
    lat = H.gpu_lattice(cfg, storage, scheme)
    f = _start(cfg, lat, prob)
    h0 = lat.get_populations()
    np.testing.assert_allclose(h0, OL.to_deviation(f, prob),
                               atol={"f64": 1e-15, "f32": 1e-7, "f16": 1e-3}[storage], rtol=0)
    lat.step(steps)
    f = OL.run(f, prob, steps)
    return lat, prob, f


# Each slice (row in 2-D, z-layer in 3-D) is padded to a multiple of 64
# thread slots, so wavefronts never straddle slices; a wavefront pulls with
# scalar offsets when it and its 3-cell halo are inside the lattice, with
# per-lane wrapped offsets when some lane is within 3 cells of an in-slice
# edge, and slice by slice within 3 slices of the wall / periodic slice ends.
CASES = [
    ("D2Q37", (70, 9), False),      # 630 cells, idle slots in every row, periodic slice wrap
    ("D2Q37", (5, 40), True),       # thin channel: every wavefront wraps in x
    ("D2Q37", (72, 12), True),
    ("D2Q37", (200, 12), True),     # 4 wavefronts a row: interior ones take the scalar-offset pull
    ("D3Q39", (16, 12, 10), False),
    ("D3Q39", (5, 4, 11), True),
    ("D3Q39", (12, 10, 9), True),
    ("D3Q39", (134, 7, 8), True),   # wavefronts span rows; some are interior in x, y and z
]


@pytest.mark.parametrize("velset,dims,walls", CASES)
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_step_parity(velset, dims, walls, storage):
    cfg = H.small_cfg(velset, dims, walls)
    steps = 12
    lat, prob, f = _run_pair(cfg, storage, steps)
    gpu = lat.read_moments()
    orc = H.oracle_fields(f, prob)
    ea, er = H.assert_parity(gpu, orc, storage)
    print(f"{velset} {dims} walls={walls} {storage}: scale-rel {max(ea.values()):.2e} "
          f"signal-rel {max(er.values()):.2e}")
    if storage == "f64":
        h = lat.get_populations()
        ho = OL.to_deviation(f, prob)
        assert np.abs(h - ho).max() / np.abs(ho).max() < 1e-12


WALL_CASES = [c for c in CASES if c[2]]


@pytest.mark.parametrize("velset,dims,walls", WALL_CASES)
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_partial_accommodation_parity(velset, dims, walls, storage):
    """Maxwell's wall model (Sec. 3.2): a specular low wall and a partly
    accommodating high wall, moving and at different temperatures."""
    cfg = dict(H.small_cfg(velset, dims, walls), gamma=(0.0, 0.6))
    lat, prob, f = _run_pair(cfg, storage, 12)
    ea, er = H.assert_parity(lat.read_moments(), H.oracle_fields(f, prob), storage)
    print(f"{velset} {dims} gamma=(0, 0.6) {storage}: scale-rel {max(ea.values()):.2e} "
          f"signal-rel {max(er.values()):.2e}")
    if storage == "f64":
        h = lat.get_populations()
        ho = OL.to_deviation(f, prob)
        assert np.abs(h - ho).max() / np.abs(ho).max() < 1e-12


HEAT_CASES = [c for c in WALL_CASES if np.prod(c[1]) < 3000]


@pytest.mark.parametrize("velset,dims,walls", HEAT_CASES)
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_unsteady_heating_parity(velset, dims, walls, storage):
    """Sec. 4.2: wall temperatures T_w + A sin(theta t), rebuilt on the device
    before every step; 40 steps run through a captured 32-step graph and 8
    direct launches, then the read-out of level 40."""
    cfg = dict(H.small_cfg(velset, dims, walls), heating=((0.02, 3.0), (-0.015, 5.0)))
    steps = 40
    lat, prob, f = _run_pair(cfg, storage, steps)
    ea, er = H.assert_parity(lat.read_moments(), H.oracle_fields(f, prob, n=steps), storage)
    print(f"{velset} {dims} heated {storage}: scale-rel {max(ea.values()):.2e} signal-rel {max(er.values()):.2e}")


def test_unsteady_heating_restart_is_bit_identical():
    cfg = dict(H.small_cfg("D2Q37", (200, 12), True), heating=((0.02, 3.0), (0.01, 7.0)))
    lat = H.gpu_lattice(cfg, "f32")
    lat.init_equilibrium()
    lat.step(10)
    saved = lat.get_state()
    lat.step(45)
    a = lat.get_populations()
    lat.set_state(saved)
    assert lat.steps_done == 10
    lat.step(45)
    np.testing.assert_array_equal(lat.get_populations(), a)


@pytest.mark.parametrize("velset,dims,walls", [CASES[1], CASES[5]])
def test_euler_scheme_parity(velset, dims, walls):
    cfg = H.small_cfg(velset, dims, walls, Kn=0.2)
    lat, prob, f = _run_pair(cfg, "f64", 10, scheme="euler")
    H.assert_parity(lat.read_moments(), H.oracle_fields(f, prob), "f64")


@pytest.mark.parametrize("varpi,Pr", [(1.0, 1.0), (0.75, 0.8)])
def test_gas_parameters_parity(varpi, Pr):
    cfg = H.small_cfg("D2Q37", (16, 10), True, Pr=Pr, varpi=varpi)
    lat, prob, f = _run_pair(cfg, "f64", 8)
    H.assert_parity(lat.read_moments(), H.oracle_fields(f, prob), "f64")


def test_reductions_match_oracle():
    cfg = H.small_cfg("D2Q37", (20, 12), True)
    prob = H.oracle_problem(cfg)
    lat = H.gpu_lattice(cfg, "f64")
    f = _start(cfg, lat, prob)
    r0 = lat.reduce()
    o0 = OL.reductions(f, prob)
    lat.step(5)
    f = OL.run(f, prob, 5)
    r1 = lat.reduce()
    o1 = OL.reductions(f, prob, u_prev=o0["u"])
    for r, o in ((r0, o0), (r1, o1)):
        assert r["mass"] == pytest.approx(o["mass"], rel=1e-13)
        assert r["energy"] == pytest.approx(o["energy"], rel=1e-13)
        np.testing.assert_allclose(r["mom"][:2], o["mom"], atol=1e-13 * prob.M)
        assert r["mdot"] == pytest.approx(o["mdot"], rel=1e-11)
    assert r1["residual"] == pytest.approx(o1["residual"], rel=1e-10)
    assert r1["step"] == 5
    # the walls conserve mass
    assert r1["mass"] == pytest.approx(r0["mass"], rel=1e-14)


def test_fused_reduction_equals_explicit():
    cfg = H.small_cfg("D2Q37", (64, 16), True)
    prob = H.oracle_problem(cfg)
    a = H.gpu_lattice(cfg, "f64")
    b = H.gpu_lattice(cfg, "f64")
    _start(cfg, a, prob)
    _start(cfg, b, prob)
    a.set_reduce_interval(4)
    a.step(8)                 # fused reductions before steps 4 and 8
    b.step(3)
    rb0 = b.reduce()
    b.step(4)
    rb1 = b.reduce()
    b.step(1)
    ra = a.last_reduction()
    assert ra["step"] == 7 == rb1["step"]
    for k in ("mass", "energy", "mdot", "residual"):
        assert ra[k] == pytest.approx(rb1[k], rel=1e-14, abs=1e-300), k
    np.testing.assert_array_equal(a.get_populations(), b.get_populations())
    assert rb0["step"] == 3


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_graph_replay_equals_direct_launches(storage):
    cfg = H.small_cfg("D2Q37", (40, 24), True)
    prob = H.oracle_problem(cfg)
    a = H.gpu_lattice(cfg, storage)
    b = H.gpu_lattice(cfg, storage)
    _start(cfg, a, prob)
    _start(cfg, b, prob)
    b.set_graph_steps(0)                   # one launch per step
    a.set_graph_steps(8)
    for lat in (a, b):
        lat.set_reduce_interval(13)        # fused reductions inside and between graphs
        lat.step(3)                        # odd: graphs start from the other buffer too
        lat.step(57)
    np.testing.assert_array_equal(a.get_populations(), b.get_populations())
    ra, rb = a.last_reduction(), b.last_reduction()
    assert ra["step"] == rb["step"] == 51
    assert ra["energy"] == rb["energy"] and ra["residual"] == rb["residual"]


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_checkpoint_restart_is_bit_identical(storage):
    cfg = H.small_cfg("D3Q39", (6, 5, 9), True)
    prob = H.oracle_problem(cfg)
    a = H.gpu_lattice(cfg, storage)
    _start(cfg, a, prob)
    a.step(3)
    raw = a.get_state()
    a.step(4)
    ha = a.get_populations()
    b = H.gpu_lattice(cfg, storage)
    b.set_state(raw)
    assert b.steps_done == 3
    b.step(4)
    np.testing.assert_array_equal(b.get_populations(), ha)


def test_set_populations_roundtrip_and_rounding():
    cfg = H.small_cfg("D2Q37", (10, 8), False)
    rng = np.random.default_rng(5)
    h = 0.01 * rng.standard_normal((37, 80))
    for storage, dt in (("f64", np.float64), ("f32", np.float32), ("f16", np.float16)):
        lat = H.gpu_lattice(cfg, storage)
        lat.set_populations(h)
        np.testing.assert_array_equal(lat.get_populations(), h.astype(dt).astype(np.float64))


def test_couette_1x32_fp64_against_oracle():
    from paper_1209_6548_amd import lattice_info, workloads
    r = lattice_info("D2Q37")["r"]
    cfg = workloads.couette_1x32(r)
    prob = H.oracle_problem(cfg)
    lat = H.gpu_lattice(cfg, "f64")
    xi = workloads.noise(cfg["noise_seed"], 37, prob.M)
    lat.init_equilibrium(None, None, None, xi, cfg["noise_amp"])
    f = OL.equilibrium_state(prob, np.ones(prob.M), np.zeros((prob.M, 2)), np.ones(prob.M), xi, cfg["noise_amp"])
    steps = 1500
    lat.step(steps)
    f = OL.run(f, prob, steps)
    ea, er = H.assert_parity(lat.read_moments(), H.oracle_fields(f, prob), "f64")
    print("couette 1x32 fp64:", ea, er)


def test_full_size_poiseuille_sampled_fp32():
    """1024 x 1024 FP32 in the benchmark's launch configuration: after a few
    steps, one more step at 4096 sampled cells (walls, edges, interior) is
    compared with the oracle's step of the same cells from the GPU state."""
    from paper_1209_6548_amd import lattice_info, workloads
    r = lattice_info("D2Q37")["r"]
    cfg = workloads.poiseuille_thermal_1024(r, storage="f32")
    prob = H.oracle_problem(cfg)
    lat = H.gpu_lattice(cfg, "f32")
    rng = np.random.default_rng(9)
    xi = rng.standard_normal((37, prob.M))
    lat.init_equilibrium(None, None, None, xi, 1e-3)
    lat.step(3)
    h_prev = lat.get_populations()
    lat.step(1)
    h_next = lat.get_populations()
    nx, ny = prob.dims
    cells = np.unique(np.concatenate([
        rng.integers(0, prob.M, 3000),
        np.arange(nx) + 0 * nx, np.arange(nx) + (ny - 1) * nx,           # wall layers
        np.arange(0, prob.M, nx), np.arange(nx - 1, prob.M, nx)]))[:4096]
    f_prev = OL.from_deviation(h_prev, prob)
    f_ref = OL.step_cells(f_prev, prob, cells)
    got = OL.from_deviation(h_next[:, cells], prob)
    # one FP32 step: absolute population error a few ulp of the FP32 values
    err = np.abs(got - f_ref) / prob.vs.w[:, None]
    assert err.max() < 2e-6, err.max()


def test_batch_matches_oracle_per_problem():
    from paper_1209_6548_amd import Batch, make_problem
    cfgs = [H.small_cfg("D2Q37", (4, ny), True, Kn=kn, Pr=pr) for ny, kn, pr in
            ((16, 0.05, 2 / 3), (33, 0.2, 1.0), (7, 0.1, 0.8), (64, 0.02, 2 / 3), (12, 0.5, 1.0))]
    probs = [make_problem("D2Q37", c["dims"][0], c["dims"][1], 1, storage="f64", Kn=c["Kn"], Pr=c["Pr"],
                          varpi=c["varpi"], T_w=c["T_w"], u_w=c["u_w"], g=c["g"]) for c in cfgs]
    b = Batch(probs)
    b.set_layout(128, 2)           # several problems per workgroup
    rng = np.random.default_rng(4)
    cells = [c["dims"][0] * c["dims"][1] for c in cfgs]
    xi = rng.standard_normal(37 * sum(cells))
    b.init_equilibrium(xi, 1e-3)
    steps = 10
    b.step(steps)
    off = 0
    for i, c in enumerate(cfgs):
        prob = H.oracle_problem(c)
        x = xi[off:off + 37 * cells[i]].reshape(37, cells[i])
        off += 37 * cells[i]
        f = OL.equilibrium_state(prob, np.ones(prob.M), np.zeros((prob.M, 2)), np.ones(prob.M), x, 1e-3)
        f = OL.run(f, prob, steps)
        H.assert_parity(b.read_moments(i), H.oracle_fields(f, prob), "f64")


def test_batch_accommodation_matches_oracle():
    from paper_1209_6548_amd import Batch, make_problem
    gammas = ((0.0, 0.0), (0.5, 1.0), (1.0, 0.25))
    cfgs = [dict(H.small_cfg("D2Q37", (4, ny), True, Kn=kn), gamma=gam) for (ny, kn), gam in
            zip(((16, 0.05), (23, 0.2), (9, 0.1)), gammas)]
    probs = [make_problem("D2Q37", c["dims"][0], c["dims"][1], 1, storage="f64", Kn=c["Kn"], Pr=c["Pr"],
                          varpi=c["varpi"], T_w=c["T_w"], u_w=c["u_w"], g=c["g"], accommodation=c["gamma"])
             for c in cfgs]
    b = Batch(probs)
    b.set_layout(64, 2)
    b.init_equilibrium()
    steps = 15
    b.step(steps)
    for i, c in enumerate(cfgs):
        prob = H.oracle_problem(c)
        f = OL.equilibrium_state(prob, np.ones(prob.M), np.zeros((prob.M, 2)), np.ones(prob.M))
        f = OL.run(f, prob, steps)
        H.assert_parity(b.read_moments(i), H.oracle_fields(f, prob), "f64")


def test_batch_fp32_layouts_agree():
    from paper_1209_6548_amd import Batch, lattice_info, workloads, make_problem
    r = lattice_info("D2Q37")["r"]
    specs = workloads.channel_batch(r, n=40, seed=8, ny_range=(16, 96))
    probs = [make_problem("D2Q37", s["dims"][0], s["dims"][1], storage="f32", Kn=s["Kn"], Pr=s["Pr"],
                          T_w=s["T_w"], u_w=s["u_w"], g=s["g"]) for s in specs]
    outs = []
    for layout in ((1024, 4), (256, 40), (64, 7)):
        b = Batch(probs)
        b.set_layout(*layout)
        b.init_equilibrium()
        b.step(25)
        outs.append([b.get_populations(i) for i in (0, 17, 39)])
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            np.testing.assert_array_equal(x, y)


def test_invalid_arguments_raise():
    from paper_1209_6548_amd import EsbgkError
    cfg = H.small_cfg("D2Q37", (8, 8), True)
    lat = H.gpu_lattice(cfg, "f64")
    with pytest.raises(EsbgkError):
        lat.step(1)                         # no state yet
    with pytest.raises(EsbgkError):
        lat.set_gas(0.1, 0.5)               # Pr < 2/3 (b < -1/2)
    with pytest.raises(EsbgkError):
        lat.set_gas(-1.0, 1.0)
    with pytest.raises(EsbgkError):
        lat.set_wall(0, 1.0, (0.0, 0.1))    # normal wall velocity
    for gam in (-0.1, 1.5, float("nan")):
        with pytest.raises(EsbgkError):
            lat.set_accommodation(0, gam)
    with pytest.raises(EsbgkError):
        lat.set_accommodation(2, 0.5)
    with pytest.raises(EsbgkError):
        H.gpu_lattice(H.small_cfg("D2Q37", (8, 8), False), "f64").set_accommodation(0, 0.5)
    with pytest.raises(EsbgkError):
        lat.set_heating(0, 1.5, 1.0)        # |A| >= T_w
    with pytest.raises(EsbgkError):
        lat.set_heating(1, 0.01, float("inf"))
    lat2 = H.gpu_lattice(H.small_cfg("D2Q37", (8, 16), True, Kn=0.5), "f64", scheme="euler")
    with pytest.raises(EsbgkError) as ei:
        lat2.set_gas(0.001, 1.0)            # dt/tau >> 2 with forward Euler
    assert ei.value.code == -5


def test_nonfinite_state_is_reported():
    from paper_1209_6548_amd import EsbgkError
    cfg = H.small_cfg("D2Q37", (8, 8), False)
    lat = H.gpu_lattice(cfg, "f64")
    h = np.zeros((37, 64))
    h[3, 10] = np.nan
    lat.set_populations(h)
    with pytest.raises(EsbgkError) as ei:
        lat.reduce()
    assert ei.value.code == -4
    with pytest.raises(EsbgkError):
        lat.step(1)                         # sticky
