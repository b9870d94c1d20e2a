"""esbgk_reduce_noalloc (no workspace scratch: a static device array) against
esbgk_reduce on identical handles, two calls in a row with the second on a
smaller lattice, through the C ABI."""

import numpy as np
import pytest

from tests import helpers as H

pytestmark = pytest.mark.gpu


def _pair(cfg, storage):
    lats = []
    D = len(cfg["dims"])
    Q = 37 if D == 2 else 39
    cells = int(np.prod(cfg["dims"]))
    rho, u, T, xi, amp = H.init_fields(cfg, cells, D, Q, seed=21)
    for _ in range(2):
        lat = H.gpu_lattice(cfg, storage)
        lat.init_equilibrium(rho, u, T, xi, amp)
        lat.step(3)
        lats.append(lat)
    return lats


def _same(r, s):
    for k in ("mass", "energy", "mdot"):
        assert r[k] == pytest.approx(s[k], rel=1e-13, abs=1e-300), k
    np.testing.assert_allclose(r["mom"], s["mom"], rtol=0, atol=1e-13 * abs(r["mass"]))
    assert r["residual"] == pytest.approx(s["residual"], rel=1e-10, abs=1e-300)
    assert r["step"] == s["step"]


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_reduce_noalloc_matches_reduce(storage):
    big = H.small_cfg("D3Q39", (160, 120, 40), True)     # 768 000 cells: 3000 blocks fold onto 1024 workgroups
    small = H.small_cfg("D2Q37", (70, 9), True)          # 630 cells: 3 blocks
    for cfg in (big, small):
        a, b = _pair(cfg, storage)
        for rep in range(2):                             # the second call has a previous u: residual > 0
            ra = a.reduce()
            rb = b.reduce_noalloc()
            _same(rb, ra)
            if rep == 1:
                assert rb["residual"] > 0.0
            a.step(2)
            b.step(2)
        np.testing.assert_array_equal(a.get_populations(), b.get_populations())
        assert b.last_reduction()["step"] == rb["step"]
        a.close()
        b.close()
