"""The batched persistent path against the FP64 oracle, through the C ABI:

* FP64 reductions per problem (mass, energy, momentum, mass flow rate,
  residual), fused into the persistent kernel every R steps and formed on
  demand, against oracle.lattice.reductions of each problem's own oracle run
  (FP64 storage), and of the GPU's own stored state (FP32 and FP16 storage,
  where the check isolates the reduction arithmetic from the storage
  rounding);
* the fused reductions of FP32 storage against the FP64 oracle's trajectory
  at a gate derived from FP32 arithmetic;
* moment parity of FP16-storage batches and of D3Q39 batches (3-D channels
  with walls across z);
* the captured-graph launch against direct launches (bit for bit), a change
  of the reduction interval between launches, and the autotuned layout's
  report;
* problems cut into pieces over several workgroups (one launch per step)
  against whole problems, bit for bit.
"""

import numpy as np
import pytest

from oracle import lattice as OL
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _cfgs_2d():
    return [H.small_cfg("D2Q37", (4, ny), True, Kn=kn, Pr=pr) for ny, kn, pr in
            ((16, 0.05, 2 / 3), (33, 0.2, 1.0), (7, 0.1, 0.8), (70, 0.02, 2 / 3), (12, 0.5, 1.0))]


def _cfgs_3d():
    return [H.small_cfg("D3Q39", dims, True, Kn=kn, Pr=pr) for dims, kn, pr in
            (((3, 4, 9), 0.1, 2 / 3), ((5, 2, 14), 0.05, 1.0), ((1, 1, 7), 0.2, 0.8), ((6, 5, 8), 0.3, 2 / 3))]


def _batch(cfgs, storage, layout=None):
    from paper_1209_6548_amd import Batch, make_problem
    D = len(cfgs[0]["dims"])
    probs = []
    for c in cfgs:
        d = tuple(c["dims"]) + (1,) * (3 - D)
        probs.append(make_problem(c["velset"], d[0], d[1], d[2], storage=storage, Kn=c["Kn"], Pr=c["Pr"],
                                  varpi=c["varpi"], T_w=c["T_w"], u_w=c["u_w"], g=c["g"]))
    b = Batch(probs)
    if layout:
        b.set_layout(*layout)
    return b


def _start(b, cfgs, seed=4, amp=1e-3):
    """Seeded noisy rest state in the batch and the matching oracle states."""
    Q = b.Q
    cells = [int(np.prod(c["dims"])) for c in cfgs]
    xi = np.random.default_rng(seed).standard_normal(Q * sum(cells))
    b.init_equilibrium(xi, amp)
    states, probs, off = [], [], 0
    for c, m in zip(cfgs, cells):
        prob = H.oracle_problem(c)
        x = xi[off:off + Q * m].reshape(Q, m)
        off += Q * m
        D = prob.D
        states.append(OL.equilibrium_state(prob, np.ones(m), np.zeros((m, D)), np.ones(m), x, amp))
        probs.append(prob)
    return states, probs


def _check_red(r, o, M, tol, res_tol):
    assert abs(r["mass"] - o["mass"]) <= tol * o["mass"], ("mass", r["mass"], o["mass"])
    assert abs(r["energy"] - o["energy"]) <= tol * o["energy"], ("energy", r["energy"], o["energy"])
    D = len(o["mom"])
    assert np.max(np.abs(r["mom"][:D] - o["mom"])) <= tol * M, ("mom", r["mom"], o["mom"])
    assert abs(r["mdot"] - o["mdot"]) <= tol, ("mdot", r["mdot"], o["mdot"])
    assert abs(r["residual"] - o["residual"]) <= res_tol * max(o["residual"], 1e-300), \
        ("residual", r["residual"], o["residual"])


@pytest.mark.parametrize("dim", [2, 3])
def test_batch_reductions_match_oracle_fp64(dim):
    """Fused reductions at levels 4 and 9 (R = 5), an explicit one at level
    12, against each problem's oracle run; FP64 storage."""
    cfgs = _cfgs_2d() if dim == 2 else _cfgs_3d()
    b = _batch(cfgs, "f64", layout=(128, 2))
    states, probs = _start(b, cfgs)
    b.set_reduce_interval(5)
    b.step(12)
    fused = b.last_reduction()
    explicit = b.reduce()
    for i, (f, prob) in enumerate(zip(states, probs)):
        f4 = OL.run(f, prob, 4)
        o4 = OL.reductions(f4, prob)
        f9 = OL.run(f4, prob, 5)
        o9 = OL.reductions(f9, prob, u_prev=o4["u"])
        f12 = OL.run(f9, prob, 3)
        o12 = OL.reductions(f12, prob, u_prev=o9["u"])
        assert fused[i]["step"] == 9 and explicit[i]["step"] == 12
        _check_red(fused[i], o9, prob.M, 1e-12, 1e-9)
        _check_red(explicit[i], o12, prob.M, 1e-12, 1e-9)
        H.assert_parity(b.read_moments(i), H.oracle_fields(f12, prob), "f64")


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("dim", [2, 3])
def test_batch_explicit_reduction_of_stored_state(storage, dim):
    """The explicit FP64 reduction of FP32 / FP16 storage equals the oracle's
    reductions of the GPU's own stored state: FP64 arithmetic on the same
    populations. The wall ghosts of its pull take rho_W from the wall partial
    sums that the step kernel formed in FP32 (sums of at most 26 terms
    w h, |w h| < 0.01 here: a few 1e-10 absolute), hence a gate of 1e-9
    relative instead of FP64 rounding; the residual's previous velocity is
    kept in FP32 (one rounding of u, 6e-8 relative, against a change of u of
    about 1e-3 relative over the four steps: 1e-4)."""
    cfgs = _cfgs_2d() if dim == 2 else _cfgs_3d()
    b = _batch(cfgs, storage)
    _, probs = _start(b, cfgs)
    b.step(7)
    first = b.reduce()
    prev = []
    for i, prob in enumerate(probs):
        f = OL.from_deviation(b.get_populations(i), prob)
        o = OL.reductions(f, prob)
        assert first[i]["residual"] == 0.0 and first[i]["step"] == 7
        _check_red(first[i], o, prob.M, 1e-9, 0.0)
        prev.append(o["u"].astype(np.float32).astype(np.float64))
    b.step(4)
    second = b.reduce()
    for i, prob in enumerate(probs):
        f = OL.from_deviation(b.get_populations(i), prob)
        o = OL.reductions(f, prob, u_prev=prev[i])
        _check_red(second[i], o, prob.M, 1e-9, 1e-4)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batch_fused_reductions_against_fp64_trajectory(storage):
    """Fused reductions of reduced-precision storage against the FP64 oracle
    run: the sums of the reconstructed FP32 state carry the storage rounding
    of the populations (|h| ~ 1e-3 here: FP32 ulp ~ 1e-10, FP16 ulp ~ 1e-6 per
    step) and FP32 arithmetic (~1e-7 relative); gates 1e-6 (FP32) and 1e-3
    (FP16) relative to the scales (mass, energy, M for momentum, 1 for the
    mass flow rate); the residual, a ratio of differences, 1e-3 and 0.1."""
    cfgs = _cfgs_2d()
    b = _batch(cfgs, storage)
    states, probs = _start(b, cfgs)
    b.set_reduce_interval(6)
    b.step(12)
    red = b.last_reduction()
    tol, res_tol = (1e-6, 1e-3) if storage == "f32" else (1e-3, 0.1)
    for i, (f, prob) in enumerate(zip(states, probs)):
        f5 = OL.run(f, prob, 5)
        o5 = OL.reductions(f5, prob)
        f11 = OL.run(f5, prob, 6)
        o11 = OL.reductions(f11, prob, u_prev=o5["u"])
        assert red[i]["step"] == 11
        _check_red(red[i], o11, prob.M, tol, res_tol)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_batch_d3q39_matches_oracle(storage):
    cfgs = _cfgs_3d()
    b = _batch(cfgs, storage, layout=(192, 3))
    states, probs = _start(b, cfgs, seed=6, amp=2e-2)
    b.step(9)
    for i, (f, prob) in enumerate(zip(states, probs)):
        f = OL.run(f, prob, 9)
        H.assert_parity(b.read_moments(i), H.oracle_fields(f, prob), storage)


def test_batch_fp16_matches_oracle():
    cfgs = _cfgs_2d()
    b = _batch(cfgs, "f16", layout=(256, 2))
    states, probs = _start(b, cfgs, seed=2, amp=2e-2)
    b.step(10)
    for i, (f, prob) in enumerate(zip(states, probs)):
        f = OL.run(f, prob, 10)
        H.assert_parity(b.read_moments(i), H.oracle_fields(f, prob), "f16")


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_batch_graph_equals_direct(storage):
    """Replayed graphs (the persistent kernel and the level update) give the
    same bits as direct launches, with step counts of both parities, a
    reduction interval changed between launches and reductions falling
    inside and between launches."""
    cfgs = _cfgs_2d()
    a = _batch(cfgs, storage)
    d = _batch(cfgs, storage)
    _start(a, cfgs)
    _start(d, cfgs)
    d.use_graphs(False)
    for b in (a, d):
        b.set_reduce_interval(4)
        b.step(3)
        b.step(6)
        b.step(3)
        b.set_reduce_interval(7)
        b.step(5)
        b.step(6)
        assert b.steps_done == 23
    for i in range(len(cfgs)):
        np.testing.assert_array_equal(a.get_populations(i), d.get_populations(i))
    ra, rd = a.last_reduction(), d.last_reduction()
    for x, y in zip(ra, rd):
        assert x["step"] == y["step"] == 20
        assert x["energy"] == y["energy"] and x["residual"] == y["residual"] and x["mdot"] == y["mdot"]


def test_batch_autotune_reports_layout():
    from paper_1209_6548_amd import lattice_info, workloads
    r = lattice_info("D2Q37")["r"]
    specs = workloads.channel_batch(r, n=48, seed=8, ny_range=(16, 128))
    cfgs = [dict(s, velset="D2Q37") for s in specs]
    b = _batch(cfgs, "f32")
    t, nb = b.autotune(steps_per_trial=5)
    info = b.layout_info()
    assert info["threads"] == t and info["bins"] == nb
    assert 1 <= info["max_pieces_per_workgroup"] <= 64
    assert info["max_cells_per_thread"] >= 1
    # the state must be set again after tuning; then it steps like a fresh batch
    b.init_equilibrium()
    b.step(4)
    ref = _batch(cfgs, "f32")
    ref.init_equilibrium()
    ref.step(4)
    for i in (0, 17, 47):
        np.testing.assert_array_equal(b.get_populations(i), ref.get_populations(i))


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("dim", [2, 3])
def test_batch_split_problems_equal_whole(storage, dim):
    """Problems cut into 64- and 128-cell pieces spread over the workgroups
    (each step its own launch, the per-problem sums added by a kernel after
    the step) give the same populations and reductions, bit for bit, as whole
    problems: through graphs and direct launches, with fused reductions and an
    explicit one."""
    cfgs = _cfgs_2d() if dim == 2 else _cfgs_3d()
    for piece, graphs in ((64, True), (128, False)):
        want = _batch(cfgs, storage, layout=(256, 4))
        b = _batch(cfgs, storage, layout=(256, 4))
        b.set_split(piece)
        pc, active = b.split
        assert pc == piece and active
        b.use_graphs(graphs)
        for x in (b, want):
            _start(x, cfgs)
            x.set_reduce_interval(4)
            x.step(5)
            x.step(6)
        for i in range(len(cfgs)):
            np.testing.assert_array_equal(b.get_populations(i), want.get_populations(i))
        for x, y in zip(b.last_reduction(), want.last_reduction()):
            assert x["step"] == y["step"] == 7
            assert x["mass"] == y["mass"] and x["energy"] == y["energy"] and x["mdot"] == y["mdot"]
            assert x["residual"] == y["residual"]
        for x, y in zip(b.reduce(), want.reduce()):
            assert x["step"] == y["step"] == 11
            assert x["mass"] == y["mass"] and x["energy"] == y["energy"] and x["residual"] == y["residual"]


def test_batch_split_rejects_bad_piece_and_whole_restores():
    from paper_1209_6548_amd import EsbgkError
    cfgs = _cfgs_2d()
    b = _batch(cfgs, "f32")
    for bad in (-64, 32, 100):
        with pytest.raises(EsbgkError):
            b.set_split(bad)
    b.set_split(4096)              # larger than every problem: nothing is cut
    assert b.split == (4096, False)
    assert b.layout()[1] == len(cfgs)   # the default bin count, capped at one bin per problem
    b.set_split(64)                # 11 pieces: the cap rises with them
    assert b.split == (64, True) and b.layout()[1] == 11
    b.set_split(0)
    assert b.split == (0, False) and b.layout()[1] == len(cfgs)
