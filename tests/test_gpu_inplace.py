"""In-place step pairs (esbgk_set_inplace) against two-buffer steps, bit for
bit, through the C ABI: 2-D and 3-D lattices, periodic and walled (moving,
heated walls, unsteady heating), every storage, odd step counts (the first
step then uses two buffers), graph replays and direct launches, fused
reductions; pushes through the three pull modes (interior wavefronts, in-slice
wrap, slices next to the walls or the periodic seam). Lattices with partial
accommodation fall back to two buffers."""

import numpy as np
import pytest

from tests import helpers as H

pytestmark = pytest.mark.gpu

CASES = [("D2Q37", (200, 12), True), ("D2Q37", (70, 9), False), ("D2Q37", (1, 33), True),
         ("D3Q39", (192, 8, 10), True), ("D3Q39", (9, 7, 6), False)]


def _start(cfg, storage, seed=5):
    D = len(cfg["dims"])
    Q = 37 if D == 2 else 39
    cells = int(np.prod(cfg["dims"]))
    rho, u, T, xi, amp = H.init_fields(cfg, cells, D, Q, seed=seed)
    lat = H.gpu_lattice(cfg, storage)
    lat.init_equilibrium(rho, u, T, xi, amp)
    return lat


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("velset,dims,walls", CASES)
def test_pairs_equal_two_buffers(velset, dims, walls, storage):
    cfg = H.small_cfg(velset, dims, walls)
    a = _start(cfg, storage)
    b = _start(cfg, storage)
    a.set_inplace(True)
    b.set_inplace(False)
    a.set_graph_steps(4)       # replays of two pairs, then direct pairs and a last two-buffer step
    b.set_graph_steps(0)
    for lat in (a, b):
        lat.set_reduce_interval(5)
        lat.step(11)
        lat.step(2)
    np.testing.assert_array_equal(a.get_populations(), b.get_populations())
    ra, rb = a.last_reduction(), b.last_reduction()
    assert ra["step"] == rb["step"] == 9
    assert ra["energy"] == rb["energy"] and ra["residual"] == rb["residual"] and ra["mdot"] == rb["mdot"]
    ma, mb = a.read_moments(), b.read_moments()
    for k in ma:
        np.testing.assert_array_equal(ma[k], mb[k])


def test_pairs_with_unsteady_heating_and_restart():
    cfg = H.small_cfg("D2Q37", (80, 16), True)
    a = _start(cfg, "f32")
    b = _start(cfg, "f32")
    a.set_inplace(True)
    b.set_inplace(False)
    for lat in (a, b):
        lat.set_heating(1, 0.02, 5.0)
        lat.step(40)
    np.testing.assert_array_equal(a.get_populations(), b.get_populations())
    raw = a.get_state()
    a.step(33)
    c = _start(cfg, "f32")
    c.set_inplace(True)
    c.set_heating(1, 0.02, 5.0)
    c.set_state(raw)
    c.step(33)
    np.testing.assert_array_equal(a.get_populations(), c.get_populations())


def test_partial_accommodation_uses_two_buffers():
    cfg = dict(H.small_cfg("D2Q37", (70, 12), True), gamma=(0.6, 1.0))
    a = _start(cfg, "f64")
    b = _start(cfg, "f64")
    a.set_inplace(True)
    b.set_inplace(False)
    a.step(9)
    b.step(9)
    np.testing.assert_array_equal(a.get_populations(), b.get_populations())


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_pairs_at_full_size(storage):
    """The benchmark channel (1024 x 1024, walls, force), where pairs are the
    default: 6 steps in pairs equal 6 two-buffer steps over all cells (the
    two-buffer step is checked against the oracle at this size in
    test_gpu_fullsize.py)."""
    from paper_1209_6548_amd import lattice_info, workloads
    import bench
    cfg = workloads.poiseuille_thermal_1024(lattice_info("D2Q37")["r"])
    a = bench.make_lattice(cfg, storage)
    b = bench.make_lattice(cfg, storage)
    b.set_inplace(False)
    for lat in (a, b):
        lat.set_graph_steps(4)
        lat.step(6)
    np.testing.assert_array_equal(a.get_state(), b.get_state())


@pytest.mark.parametrize("storage,n,pairs", [("f32", 896, False), ("f32", 1024, True), ("f32", 1448, True),
                                             ("f32", 2048, False), ("f16", 1024, False), ("f16", 1448, True),
                                             ("f64", 1024, True)])
def test_default_mode_picks_pairs_by_size(storage, n, pairs):
    """Mode 2 uses pairs when the two buffers overflow the 256 MB
    memory-side cache and one buffer is at most 384 MB (the sizes where
    pairs were measured faster)."""
    from paper_1209_6548_amd import lattice_info, workloads
    import bench
    cfg = dict(workloads.poiseuille_thermal_1024(lattice_info("D2Q37")["r"]), dims=(n, n))
    lat = bench.make_lattice(cfg, storage)
    assert lat.inplace_active == pairs
    lat.set_inplace(1)
    assert lat.inplace_active
    lat.set_inplace(0)
    assert not lat.inplace_active
    lat.close()
