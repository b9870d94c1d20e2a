"""Parity at the benchmark sizes, in the launch configuration bench.py times:
one more GPU step at sampled cells is compared with the oracle's step of the
same cells from the GPU state (walls, periodic edges, interior, random), and
the batched-channel workload is compared problem by problem.

Tolerance for one step from identical stored inputs: half an ulp of the
storage type at the oracle's value (the final rounding) plus the FP32
arithmetic of the collision (FP32 and FP16 storage) or 1e-13 (FP64)."""

import numpy as np
import pytest

from oracle import lattice as OL
from tests import helpers as H

pytestmark = pytest.mark.gpu

DT = {"f64": np.float64, "f32": np.float32, "f16": np.float16}


def _sample_cells(prob, rng, n_random=3000):
    dims = prob.dims
    nx = dims[0]
    M = prob.M
    layer = int(np.prod(dims[:-1]))
    parts = [rng.integers(0, M, n_random),
             np.arange(min(layer, 512)),                              # first layer (wall or periodic edge)
             M - 1 - np.arange(min(layer, 512)),                      # last layer
             np.arange(0, M, nx)[rng.integers(0, M // nx, 300)],      # x = 0 column cells
             np.arange(nx - 1, M, nx)[rng.integers(0, M // nx, 300)]]
    return np.unique(np.concatenate(parts))


def _smooth_fields(prob, amp=2e-3):
    """rho, u, T with a few smooth modes, so every sampled cell is off rest."""
    shape = prob.dims[::-1]
    grids = np.meshgrid(*[2 * np.pi * (np.arange(n) + 0.5) / n for n in shape], indexing="ij")
    x = grids[-1].reshape(-1)
    y = grids[-2].reshape(-1)
    z = grids[0].reshape(-1) if prob.D == 3 else 0.0 * x
    rho = 1.0 + amp * np.cos(x + 2 * y)
    u = np.zeros((prob.D, prob.M))
    u[0] = amp * np.sin(y + z)
    u[1] = amp * np.cos(3 * x)
    T = 1.0 + amp * np.sin(2 * x - y + z)
    return rho, u, T


def _one_step_parity(cfg, storage, steps_before=3, seed=9, amp=1e-3):
    prob = H.oracle_problem(cfg)
    lat = H.gpu_lattice(cfg, storage)
    rng = np.random.default_rng(seed)
    if prob.M <= (1 << 21):
        xi = rng.standard_normal((prob.vs.Q, prob.M))
        lat.init_equilibrium(None, None, None, xi, amp)
        del xi
    else:
        lat.init_equilibrium(*_smooth_fields(prob))
    lat.step(steps_before)                      # graphs are not used for fewer steps than a graph holds
    raw_prev = lat.get_state()
    lat.step(1)
    raw_next = lat.get_state()
    cells = _sample_cells(prob, rng)
    prev = H.StoredPopulations(raw_prev, prob.vs.Q, prob.M, DT[storage], prob.vs.w)
    f_ref = OL.step_cells(prev, prob, cells)
    h_ref = f_ref / prob.vs.w[:, None] - 1.0
    nxt = H.StoredPopulations(raw_next, prob.vs.Q, prob.M, DT[storage], prob.vs.w)
    h_got = nxt.h[:, cells].astype(np.float64)
    err = np.abs(h_got - h_ref)
    if storage == "f64":
        bound = 1e-13 * np.maximum(1.0, np.abs(h_ref))
    else:
        bound = 0.5 * H.ulp(h_ref, DT[storage]) + 4e-7 * (1.0 + np.abs(h_ref))
    worst = float(np.max(err / bound))
    print(f"{cfg.get('name', cfg['dims'])} {storage}: {len(cells)} cells, max |dh| {err.max():.2e}, "
          f"worst err/bound {worst:.2f}")
    assert worst <= 1.0
    return lat


@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
def test_poiseuille_1024_one_step(storage):
    from paper_1209_6548_amd import lattice_info, workloads
    cfg = workloads.poiseuille_thermal_1024(lattice_info("D2Q37")["r"], storage=storage)
    _one_step_parity(cfg, storage)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_shear_wave_box_256_one_step(storage):
    from paper_1209_6548_amd import lattice_info, workloads
    cfg = dict(name="shear_wave_256^3", velset="D3Q39", dims=(256, 256, 256), walls=False, Kn=0.02, Pr=2 / 3,
               varpi=0.5, g=(0.0, 0.0, 0.0))
    _one_step_parity(cfg, storage, steps_before=2)


def test_channel_512x512x256_f16_one_step():
    from paper_1209_6548_amd import lattice_info, workloads
    cfg = workloads.channel_3d(lattice_info("D3Q39")["r"])
    _one_step_parity(cfg, "f16", steps_before=2)


def test_slices_past_the_32bit_window_fp32():
    """2048 x 2048 slices: seven slice blocks span more than 4 GiB, past the
    32-bit offsets of the scalar-offset pull, so every wavefront pulls slice by
    slice. One step at sampled cells (walls, edges, interior) against the oracle."""
    from paper_1209_6548_amd import lattice_info, workloads
    cfg = workloads.channel_3d(lattice_info("D3Q39")["r"], nx=2048, ny=2048, nz=8, storage="f32")
    slice_block = (39 * 2048 * 2048 + 256) * 4
    assert 7 * slice_block >= 1 << 32
    _one_step_parity(cfg, "f32", steps_before=2)


def test_couette_1x32_fp64_full_run():
    """The 1 x 32 Couette case for its full 20 000 steps, FP64, vs. the oracle."""
    from paper_1209_6548_amd import lattice_info, workloads
    cfg = workloads.couette_1x32(lattice_info("D2Q37")["r"])
    prob = H.oracle_problem(cfg)
    lat = H.gpu_lattice(cfg, "f64")
    xi = workloads.noise(cfg["noise_seed"], 37, prob.M)
    lat.init_equilibrium(None, None, None, xi, cfg["noise_amp"])
    f = OL.equilibrium_state(prob, np.ones(prob.M), np.zeros((prob.M, 2)), np.ones(prob.M), xi, cfg["noise_amp"])
    lat.step(cfg["steps"])
    f = OL.run(f, prob, cfg["steps"])
    ea, er = H.assert_parity(lat.read_moments(), H.oracle_fields(f, prob), "f64")
    print("couette 1x32, 20000 steps, fp64:", {k: f"{v:.1e}" for k, v in ea.items()})


def test_channel_batch_512_sampled_problems():
    """The 512-channel batch in one persistent launch (autotuned layout, FP32):
    after 40 steps, sampled problems match the oracle run of the same problem."""
    from paper_1209_6548_amd import Batch, lattice_info, make_problem, workloads
    specs = workloads.channel_batch(lattice_info("D2Q37")["r"])
    probs = [make_problem("D2Q37", s["dims"][0], s["dims"][1], storage="f32", Kn=s["Kn"], Pr=s["Pr"],
                          T_w=s["T_w"], u_w=s["u_w"], g=s["g"]) for s in specs]
    b = Batch(probs)
    b.autotune(5)
    b.init_equilibrium()
    steps = 40
    b.step(steps)
    rng = np.random.default_rng(1)
    pick = list(rng.choice(len(specs), 6, replace=False)) + [int(np.argmax([s["dims"][1] for s in specs]))]
    for i in pick:
        s = specs[i]
        prob = H.oracle_problem(s)
        f = OL.equilibrium_state(prob, np.ones(prob.M), np.zeros((prob.M, 2)), np.ones(prob.M))
        f = OL.run(f, prob, steps)
        ea, er = H.assert_parity(b.read_moments(i), H.oracle_fields(f, prob), "f32")
        print(f"batch problem {i} ({s['case']}, ny={s['dims'][1]}): scale-rel {max(ea.values()):.1e}")
