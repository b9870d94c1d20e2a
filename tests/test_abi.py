"""CPU checks of the C ABI library: it loads, exports every function that
include/esbgk.h declares, derives the same velocity sets as the oracle and
validates shapes on the host (no GPU work)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "esbgk.h")
LIB = os.path.join(ROOT, "paper_1209_6548_amd", "libesbgk.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libesbgk.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(esbgk_\w+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("esbgk_create", "esbgk_step", "esbgk_read_moments", "esbgk_set_gas", "esbgk_set_wall",
              "esbgk_set_body_force", "esbgk_batch_step", "esbgk_reduce"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("name", ["D2Q37", "D3Q39"])
def test_library_tables_equal_the_oracle(name):
    from oracle import quadrature
    from paper_1209_6548_amd import lattice_info
    info = lattice_info(name)
    vs = quadrature.velocity_set(name)
    assert info["Q"] == vs.Q and info["D"] == vs.D and info["N"] == vs.N
    np.testing.assert_array_equal(info["e"], vs.e)
    assert info["r"] == pytest.approx(vs.r, rel=1e-15)
    np.testing.assert_allclose(info["w"], vs.w, rtol=1e-14)


def test_workspace_bytes_validates_shapes():
    from paper_1209_6548_amd import binding as B
    lib = B.lib()
    ok = B.Shape(B.D2Q37, 64, 32, 1, 1, B.F32, B.TRAPEZOID, 0)
    n = lib.esbgk_workspace_bytes(ctypes.byref(ok))
    # two population buffers of 37 x 2048 floats at least
    assert n >= 2 * 37 * 64 * 32 * 4
    bad = [B.Shape(3, 8, 8, 1, 0, 0, 0, 0),            # unknown set
           B.Shape(B.D2Q37, 8, 8, 2, 0, 0, 0, 0),      # nz != 1 in 2-D
           B.Shape(B.D2Q37, 8, 5, 1, 1, 0, 0, 0),      # wall axis < 6
           B.Shape(B.D3Q39, 8, 8, 0, 0, 0, 0, 0),      # empty
           B.Shape(B.D2Q37, 8, 8, 1, 0, 3, 0, 0),      # storage
           B.Shape(B.D2Q37, 8, 8, 1, 0, 0, 2, 0),      # scheme
           B.Shape(B.D3Q39, 2048, 2048, 1024, 0, 0, 0, 0)]  # >= 2^31 cells
    for s in bad:
        assert lib.esbgk_workspace_bytes(ctypes.byref(s)) == 0


def test_create_rejects_missing_workspace():
    from paper_1209_6548_amd import binding as B
    lib = B.lib()
    s = B.Shape(B.D2Q37, 8, 8, 1, 0, B.F64, 0, 0)
    ctx = ctypes.c_void_p()
    assert lib.esbgk_create(ctypes.byref(s), None, 0, None, ctypes.byref(ctx)) == B.E_NOMEM
    assert not ctx.value


def test_fast_division_constants():
    # the kernels divide cell indices by nx and ny with (umulhi(n, m) + n) >> l
    from paper_1209_6548_amd import binding  # noqa: F401  (library loads)
    for d in [1, 2, 3, 4, 5, 7, 16, 32, 100, 255, 256, 257, 1000, 1024, 4097, 65537, 1 << 20, (1 << 31) - 1]:
        l = 0
        while (1 << l) < d:
            l += 1
        m = ((1 << 32) * ((1 << l) - d)) // d + 1
        rng = np.random.default_rng(d)
        ns = np.concatenate([rng.integers(0, 1 << 31, 2000), [0, d - 1, d, d + 1, (1 << 31) - 1]])
        for n in ns:
            n = int(n)
            q = (((n * m) >> 32) + n) >> l
            assert q == n // d, (d, n)


@pytest.mark.parametrize("name,n,D,N", [("D2Q16GH", 4, 2, 3), ("D2Q36GH", 6, 2, 4), ("D2Q64GH", 8, 2, 4),
                                        ("D3Q216GH", 6, 3, 4)])
def test_tvd_set_equals_the_oracle_product_set(name, n, D, N):
    from oracle import offlattice
    from paper_1209_6548_amd import binding as B
    from paper_1209_6548_amd import tvd_velocity_set
    c, w = tvd_velocity_set(name)
    vs = offlattice.ProductSet(n, D, N)
    # same order; both sides round the 50-digit (oracle) or long-double
    # (library) roots
    np.testing.assert_array_equal(c, vs.c)
    np.testing.assert_allclose(w, vs.w, rtol=5e-16, atol=0)
    # opposites are exact negatives on the library side too
    P = vs.Q // 2
    np.testing.assert_array_equal(c[P:], -c[:P])
    Q, NN = ctypes.c_int(), ctypes.c_int()
    assert B.lib().esbgk_tvd_set_info(B._GH_SET[name], ctypes.byref(Q), ctypes.byref(NN), None, None) == 0
    assert (Q.value, NN.value) == (vs.Q, N)


def test_tvd_set_info_rejects_other_sets():
    from paper_1209_6548_amd import binding as B
    for v in (0, B.D2Q37, B.D3Q39, 7):
        assert B.lib().esbgk_tvd_set_info(v, None, None, None, None) == B.E_INVALID


def test_tvd_workspace_bytes_validates_shapes():
    from paper_1209_6548_amd import binding as B
    lib = B.lib()
    ok = B.Shape(B.D2Q36GH, 64, 32, 1, 0, B.F32, B.EULER, 0)
    assert lib.esbgk_tvd_workspace_bytes(ctypes.byref(ok)) >= 2 * 36 * 64 * 32 * 4
    bad = [B.Shape(B.D2Q37, 8, 8, 1, 0, B.F32, B.EULER, 0),    # on-lattice set
           B.Shape(B.D2Q36GH, 8, 8, 2, 0, B.F32, B.EULER, 0),  # 3-D
           B.Shape(B.D2Q36GH, 8, 2, 1, 1, B.F32, B.EULER, 0),  # walls need ny >= 3
           B.Shape(B.D2Q36GH, 8, 8, 1, 2, B.F32, B.EULER, 0),  # walls flag
           B.Shape(B.D2Q36GH, 8, 8, 1, 0, B.F32, B.TRAPEZOID, 0),
           B.Shape(B.D2Q36GH, 0, 8, 1, 0, B.F32, B.EULER, 0),
           B.Shape(B.D2Q36GH, 8, 8, 1, 0, 3, B.EULER, 0)]
    for s in bad:
        assert lib.esbgk_tvd_workspace_bytes(ctypes.byref(s)) == 0
    # a channel (walls across y) needs two wall rows and one between
    ch = B.Shape(B.D2Q36GH, 8, 3, 1, 1, B.F64, B.EULER, 0)
    assert lib.esbgk_tvd_workspace_bytes(ctypes.byref(ch)) > 0
    # and the on-lattice entry points reject the off-lattice set
    assert lib.esbgk_workspace_bytes(ctypes.byref(ok)) == 0


def test_tvd_create_rejects_missing_workspace_and_bad_cfl():
    from paper_1209_6548_amd import binding as B
    lib = B.lib()
    s = B.Shape(B.D2Q36GH, 8, 8, 1, 0, B.F64, B.EULER, 0)
    t = ctypes.c_void_p()
    assert lib.esbgk_tvd_create(ctypes.byref(s), 0.5, None, 0, None, ctypes.byref(t)) == B.E_NOMEM
    assert not t.value
    assert lib.esbgk_tvd_create(ctypes.byref(s), 1.5, None, 0, None, ctypes.byref(t)) == B.E_INVALID
    assert b"cfl" in lib.esbgk_tvd_last_error(None)


def test_tvd_bound_check_on_host():
    """esbgk_tvd_bounded: axes * cfl <= 1 - dt/tau at rho = T = 1, with
    dt = cfl / (n_ref max|c|) and tau = Kn/Pr (no GPU needed)."""
    from paper_1209_6548_amd import binding as B
    cmax = float(np.max(np.abs(B.tvd_velocity_set("D2Q36GH")[0])))
    n_ref, Kn, Pr = 11, 0.05, 2 / 3
    w = lambda cfl: cfl / (n_ref * cmax) * Pr / Kn   # noqa: E731
    assert B.tvd_bounded("D2Q36GH", n_ref, 0.4, Kn, Pr, 2) == B.OK
    assert 2 * 0.4 <= 1 - w(0.4)
    assert B.tvd_bounded("D2Q36GH", n_ref, 0.5, Kn, Pr, 2) == B.E_UNSTABLE
    assert 2 * 0.5 > 1 - w(0.5)
    assert B.tvd_bounded("D2Q36GH", n_ref, 0.5, Kn, Pr, 1) == B.OK
    # the defaults of TVDLattice sum the Courant numbers of every axis to 0.9
    assert B.default_tvd_cfl(2) == 0.45 and B.default_tvd_cfl(3) == 0.3
    assert B.tvd_bounded("D2Q36GH", 1024, B.default_tvd_cfl(2), 0.05, 2 / 3, 2) == B.OK
    assert B.tvd_bounded("D3Q216GH", 128, B.default_tvd_cfl(3), 0.05, 2 / 3, 3) == B.OK
    # a collision weight of 0.15 leaves 0.85 for the advection: 0.9 is too much there
    assert B.tvd_bounded("D3Q216GH", 8, 0.3, 0.05, 2 / 3, 3) == B.E_UNSTABLE
    for bad in ((0, 0.3, 0.05, 2 / 3, 2), (11, 1.5, 0.05, 2 / 3, 2), (11, 0.3, 0.0, 2 / 3, 2),
                (11, 0.3, 0.05, 0.5, 2), (11, 0.3, 0.05, 2 / 3, 3)):
        assert B.tvd_bounded("D2Q36GH", *bad) == B.E_INVALID


def test_batch_rejects_unstable_euler_problem():
    """A batched Euler problem with dt/tau >= 2 at rho = T = 1 is rejected like
    esbgk_set_gas rejects it (workspace size 0); the trapezoidal rule takes
    it."""
    import ctypes

    from paper_1209_6548_amd import binding as B
    r = B.lattice_info("D2Q37")["r"]
    ny = 16
    dt = 1.0 / (ny * r)

    def prob(scheme, Kn, Pr):
        p = B.Problem()
        p.shape = B.Shape(B.D2Q37, 4, ny, 1, 1, B.F32, scheme, 0)
        p.Kn, p.Pr, p.varpi = Kn, Pr, 0.5
        p.T_w[0] = p.T_w[1] = 1.0
        return p

    L = B.lib()
    for scheme, Kn, Pr, ok in ((B.EULER, dt / 1.9, 1.0, True), (B.EULER, dt / 2.1, 1.0, False),
                               (B.EULER, dt / 2.1 * 0.9, 0.9, False), (B.TRAPEZOID, dt / 2.1, 1.0, True)):
        arr = (B.Problem * 1)(prob(scheme, Kn, Pr))
        assert (L.esbgk_batch_workspace_bytes(ctypes.cast(arr, ctypes.c_void_p), 1) > 0) == ok
