"""Degenerate inputs of the GPU paths, checked through the C ABI:

* a step count of zero leaves every handle's state and step counter as
  they were (single lattice, the paper's TVD scheme, a batch);
* a lattice of one cell (every pull wraps onto the cell itself, so a
  uniform gas only collides and accelerates) against the FP64 oracle, on
  D2Q37, D3Q39 and the paper's D2Q36.
"""

import numpy as np
import pytest

from oracle import lattice as OL
from oracle import offlattice as OF
from tests import helpers as H

pytestmark = pytest.mark.gpu


def test_zero_steps_change_nothing():
    from paper_1209_6548_amd import Batch, TVDLattice, make_problem
    cfg = H.small_cfg("D2Q37", (70, 9), True)
    lat = H.gpu_lattice(cfg, "f32", "trapezoid")
    rho, u, T, xi, amp = H.init_fields(cfg, 70 * 9, 2, 37)
    lat.init_equilibrium(rho, u, T, xi, amp)
    lat.step(3)
    h = lat.get_populations()
    lat.step(0)
    assert lat.steps_done == 3
    np.testing.assert_array_equal(lat.get_populations(), h)

    tvd = TVDLattice(20, 12, storage="f32", walls=True, velset="D2Q36GH")
    tvd.init_equilibrium(noise=np.random.default_rng(1).standard_normal((36, 240)), amplitude=0.01)
    tvd.step(2)
    h = tvd.get_populations()
    tvd.step(0)
    assert tvd.steps_done == 2
    np.testing.assert_array_equal(tvd.get_populations(), h)

    b = Batch([make_problem("D2Q37", 4, ny, storage="f32", Kn=0.1, Pr=2 / 3) for ny in (16, 23, 40)])
    b.init_equilibrium()
    b.step(2)
    h = [b.get_populations(i) for i in range(3)]
    b.step(0)
    for i in range(3):
        np.testing.assert_array_equal(b.get_populations(i), h[i])


@pytest.mark.parametrize("velset,dims", [("D2Q37", (1, 1)), ("D3Q39", (1, 1, 1))])
def test_one_cell_lattice_fp64(velset, dims):
    cfg = H.small_cfg(velset, dims, False)
    prob = H.oracle_problem(cfg, "trapezoid")
    lat = H.gpu_lattice(cfg, "f64", "trapezoid")
    Q = prob.vs.Q
    rho, u, T, xi, amp = H.init_fields(cfg, 1, prob.D, Q, seed=4)
    lat.init_equilibrium(rho, u, T, xi, amp)
    f = OL.equilibrium_state(prob, rho, u.T, T, xi, amp)
    lat.step(6)
    f = OL.run(f, prob, 6)
    H.assert_parity(lat.read_moments(), H.oracle_fields(f, prob), "f64")
    h, ho = lat.get_populations(), OL.to_deviation(f, prob)
    assert np.abs(h - ho).max() / np.abs(ho).max() < 1e-12


def test_one_cell_tvd_fp64():
    from paper_1209_6548_amd import TVDLattice
    gh = OF.ProductSet(6, 2, 4)
    prob = OF.TVDProblem(gh, (1, 1), Kn=0.05, Pr=2 / 3, g=(0.02, -0.01, 0.0), cfl=0.5, n_ref=16)
    lat = TVDLattice(1, 1, storage="f64", cfl=0.5, n_ref=16, velset="D2Q36GH")
    lat.set_gas(0.05, 2 / 3)
    lat.set_body_force((0.02, -0.01))
    rho, u, T, xi, amp = H.init_fields(None, 1, 2, gh.Q, seed=4)
    lat.init_equilibrium(rho, u, T, xi, amp)
    f = OF.equilibrium_state(prob, rho, u.T, T, xi, amp)
    lat.step(6)
    f = OF.run(f, prob, 6)
    h, ho = lat.get_populations(), f / gh.w[:, None] - 1.0
    assert np.abs(h - ho).max() / np.abs(ho).max() < 1e-12


def test_graph_release_waits_for_queued_replays():
    """esbgk_step returns as soon as its graph replays are queued. Changing the
    graph length, switching unsteady heating on and destroying the handle
    release the captured graphs; they first wait for the stream, so the
    queued replays finish. The state then equals direct launches bit for
    bit, and a fresh handle steps normally afterwards."""
    cfg = H.small_cfg("D2Q37", (200, 64), True)
    rho, u, T, xi, amp = H.init_fields(cfg, 200 * 64, 2, 37, seed=9)

    def fresh():
        lat = H.gpu_lattice(cfg, "f32")
        lat.init_equilibrium(rho, u, T, xi, amp)
        return lat

    ref = fresh()
    ref.set_graph_steps(0)
    ref.step(160)
    h_ref = ref.get_populations()
    ref.close()

    lat = fresh()
    lat.step(64)               # two replays of the 32-step graph, queued
    lat.set_graph_steps(16)    # releases both graphs
    lat.step(32)
    lat.set_graph_steps(32)
    lat.step(64)
    assert lat.steps_done == 160
    np.testing.assert_array_equal(lat.get_populations(), h_ref)

    lat.step(64)
    lat.set_heating(1, 0.01, 3.0)   # heating on: the graphs are captured again with the table rebuilds
    lat.set_heating(1, 0.0, 0.0)
    lat.step(32)
    lat.close()                      # replays still queued

    again = fresh()
    again.set_graph_steps(0)
    again.step(160)
    np.testing.assert_array_equal(again.get_populations(), h_ref)
