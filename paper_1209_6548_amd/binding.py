"""Thin Python binding of libesbgk.so (argument marshalling only).

Every step of the lattice ES-BGK path runs in the library's HIP kernels.
PyTorch only provides the device workspace (torch.empty, uint8) and the HIP
stream (torch.cuda.current_stream). Calls mirror the C ABI in
include/esbgk.h; a non-zero status raises EsbgkError with the library's
message.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesbgk.so")

OK, E_INVALID, E_NOMEM, E_HIP, E_NONFINITE, E_UNSTABLE, E_STATE = 0, -1, -2, -3, -4, -5, -6
D2Q37, D3Q39, D2Q36GH, D2Q16GH, D2Q64GH, D3Q216GH = 1, 2, 3, 4, 5, 6
F64, F32, F16 = 0, 1, 2
TRAPEZOID, EULER = 0, 1

_VELSET = {"D2Q37": D2Q37, "D3Q39": D3Q39}
_GH_SET = {"D2Q16GH": D2Q16GH, "D2Q36GH": D2Q36GH, "D2Q64GH": D2Q64GH, "D3Q216GH": D3Q216GH}
_STORAGE = {"f64": F64, "f32": F32, "f16": F16}
_SCHEME = {"trapezoid": TRAPEZOID, "euler": EULER}
_NAMES = {E_INVALID: "E_INVALID", E_NOMEM: "E_NOMEM", E_HIP: "E_HIP", E_NONFINITE: "E_NONFINITE",
          E_UNSTABLE: "E_UNSTABLE", E_STATE: "E_STATE"}


class EsbgkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Shape(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("velset", "nx", "ny", "nz", "walls", "storage", "scheme", "n_ref")]


class Problem(ctypes.Structure):
    _fields_ = [("shape", Shape), ("Kn", ctypes.c_double), ("Pr", ctypes.c_double), ("varpi", ctypes.c_double),
                ("T_w", ctypes.c_double * 2), ("u_w", (ctypes.c_double * 3) * 2), ("g", ctypes.c_double * 3),
                ("specular", ctypes.c_double * 2)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built.

    PyTorch is imported first: it carries its own HIP runtime with the same
    soname as the system one, so loading torch first makes libesbgk.so bind
    to that runtime instead of starting a second one in the process (two
    runtimes cannot share the device, the streams or the memory)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1209_6548_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D, SZ, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_int64
        DP = ctypes.POINTER(ctypes.c_double)
        sig = {
            "esbgk_lattice_info": (I, [I, P, P, P, P, P, P]),
            "esbgk_workspace_bytes": (SZ, [P]),
            "esbgk_create": (I, [P, P, SZ, P, P]),
            "esbgk_destroy": (I, [P]),
            "esbgk_set_gas": (I, [P, D, D, D]),
            "esbgk_set_wall": (I, [P, I, D, DP]),
            "esbgk_set_wall_accommodation": (I, [P, I, D]),
            "esbgk_set_wall_heating": (I, [P, I, D, D]),
            "esbgk_set_body_force": (I, [P, DP]),
            "esbgk_init_equilibrium": (I, [P, DP, DP, DP, DP, D]),
            "esbgk_set_populations": (I, [P, DP]),
            "esbgk_get_populations": (I, [P, DP]),
            "esbgk_state_bytes": (SZ, [P]),
            "esbgk_get_state": (I, [P, P, SZ]),
            "esbgk_set_state": (I, [P, P, SZ]),
            "esbgk_step": (I, [P, I64]),
            "esbgk_set_graph_steps": (I, [P, I]),
            "esbgk_set_inplace": (I, [P, I]),
            "esbgk_inplace_active": (I, [P]),
            "esbgk_read_moments": (I, [P, DP, P]),
            "esbgk_reduce": (I, [P, DP]),
            "esbgk_reduce_noalloc": (I, [P, DP]),
            "esbgk_set_reduce_interval": (I, [P, I64]),
            "esbgk_last_reduction": (I, [P, DP]),
            "esbgk_steps_done": (I64, [P]),
            "esbgk_last_error": (ctypes.c_char_p, [P]),
            "esbgk_batch_workspace_bytes": (SZ, [P, I]),
            "esbgk_batch_create": (I, [P, I, P, SZ, P, P]),
            "esbgk_batch_destroy": (I, [P]),
            "esbgk_batch_init_equilibrium": (I, [P, DP, D]),
            "esbgk_batch_step": (I, [P, I64]),
            "esbgk_batch_read_moments": (I, [P, I, DP, P]),
            "esbgk_batch_get_populations": (I, [P, I, DP]),
            "esbgk_batch_set_layout": (I, [P, I, I]),
            "esbgk_batch_layout": (I, [P, P, P]),
            "esbgk_batch_autotune": (I, [P, I]),
            "esbgk_batch_steps_done": (I64, [P]),
            "esbgk_batch_use_graphs": (I, [P, I]),
            "esbgk_batch_set_reduce_interval": (I, [P, I64]),
            "esbgk_batch_reduce": (I, [P, DP]),
            "esbgk_batch_last_reduction": (I, [P, DP]),
            "esbgk_batch_layout_info": (I, [P, P, P]),
            "esbgk_batch_set_split": (I, [P, I]),
            "esbgk_batch_split": (I, [P, P, P]),
            "esbgk_batch_last_error": (ctypes.c_char_p, [P]),
            "esbgk_tvd_info": (I, [DP, DP]),
            "esbgk_tvd_set_info": (I, [I, P, P, DP, DP]),
            "esbgk_tvd_workspace_bytes": (SZ, [P]),
            "esbgk_tvd_create": (I, [P, D, P, SZ, P, P]),
            "esbgk_tvd_destroy": (I, [P]),
            "esbgk_tvd_time_step": (D, [P]),
            "esbgk_tvd_bounded": (I, [I, I, D, D, D, I]),
            "esbgk_tvd_set_gas": (I, [P, D, D, D]),
            "esbgk_tvd_set_body_force": (I, [P, DP]),
            "esbgk_tvd_set_wall": (I, [P, I, D, DP]),
            "esbgk_tvd_init_equilibrium": (I, [P, DP, DP, DP, DP, D]),
            "esbgk_tvd_set_populations": (I, [P, DP]),
            "esbgk_tvd_get_populations": (I, [P, DP]),
            "esbgk_tvd_step": (I, [P, I64]),
            "esbgk_tvd_read_moments": (I, [P, DP, P]),
            "esbgk_tvd_steps_done": (I64, [P]),
            "esbgk_tvd_last_error": (ctypes.c_char_p, [P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def lattice_info(velset):
    """Velocity set (Sec. 2.2) as derived by the library: Q, D, N, r, e, w."""
    vid = _VELSET[velset] if isinstance(velset, str) else velset
    Q, D, N = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    r = ctypes.c_double()
    e = (ctypes.c_int * (39 * 3))()
    w = (ctypes.c_double * 39)()
    rc = lib().esbgk_lattice_info(vid, ctypes.byref(Q), ctypes.byref(D), ctypes.byref(N), ctypes.byref(r), e, w)
    if rc:
        raise EsbgkError(rc, "lattice_info")
    q, d = Q.value, D.value
    return dict(Q=q, D=d, N=N.value, r=r.value, e=np.array(e[:q * d], dtype=np.int64).reshape(q, d),
                w=np.array(w[:q]))


def _stream_ptr(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def split_fields(raw, D):
    """Name the rows of a moments array [F][cells]."""
    k = 0
    out = {"rho": raw[0]}
    k = 1
    out["u"] = raw[k:k + D]
    k += D
    out["T"] = raw[k]
    k += 1
    ns = D * (D + 1) // 2
    out["sigma"] = raw[k:k + ns]
    k += ns
    out["q"] = raw[k:k + D]
    return out


class Lattice:
    """One lattice on the GPU: a handle of the C ABI plus its workspace."""

    def __init__(self, velset="D2Q37", nx=64, ny=64, nz=1, walls=False, storage="f32", scheme="trapezoid",
                 n_ref=0, device="cuda:0"):
        import torch
        self.device = torch.device(device)
        self.velset = velset
        info = lattice_info(velset)
        self.Q, self.D, self.N, self.r = info["Q"], info["D"], info["N"], info["r"]
        self.dims = (nx, ny) if self.D == 2 else (nx, ny, nz)
        self.cells = nx * ny * nz
        self.storage = storage
        self.shape = Shape(_VELSET[velset], nx, ny, nz, int(bool(walls)), _STORAGE[storage], _SCHEME[scheme], n_ref)
        L = lib()
        nbytes = L.esbgk_workspace_bytes(ctypes.byref(self.shape))
        if nbytes == 0:
            raise EsbgkError(E_INVALID, "invalid shape")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._ctx = ctypes.c_void_p()
        rc = L.esbgk_create(ctypes.byref(self.shape), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                            _stream_ptr(self.device), ctypes.byref(self._ctx))
        if rc:
            msg = L.esbgk_last_error(None)
            raise EsbgkError(rc, f"create: {msg.decode() if msg else ''}")

    # -- plumbing --
    def _check(self, rc, what):
        if rc:
            msg = lib().esbgk_last_error(self._ctx)
            raise EsbgkError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().esbgk_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- parameters --
    def set_gas(self, Kn, Pr, varpi=0.5):
        self._check(lib().esbgk_set_gas(self._ctx, Kn, Pr, varpi), "set_gas")

    def set_wall(self, side, T, u=(0.0, 0.0, 0.0)):
        uu = np.zeros(3)
        uu[:len(u)] = u
        self._check(lib().esbgk_set_wall(self._ctx, int(side), float(T), _dp(uu)), "set_wall")

    def set_accommodation(self, side, gamma):
        """Maxwell's wall model: fraction gamma of wall `side` re-emitted
        diffusely, 1 - gamma reflected specularly (default 1)."""
        self._check(lib().esbgk_set_wall_accommodation(self._ctx, int(side), float(gamma)), "set_accommodation")

    def set_heating(self, side, amplitude, theta):
        """Unsteady heating of wall `side`: T_w + amplitude sin(theta t)."""
        self._check(lib().esbgk_set_wall_heating(self._ctx, int(side), float(amplitude), float(theta)),
                    "set_heating")

    def set_body_force(self, g):
        gg = np.zeros(3)
        gg[:len(g)] = g
        self._check(lib().esbgk_set_body_force(self._ctx, _dp(gg)), "set_body_force")

    # -- state --
    def init_equilibrium(self, rho=None, u=None, T=None, noise=None, amplitude=0.0):
        rho = _f64(rho, (self.cells,))
        u = _f64(u, (self.D, self.cells))
        T = _f64(T, (self.cells,))
        noise = _f64(noise, (self.Q, self.cells))
        self._check(lib().esbgk_init_equilibrium(self._ctx, _dp(rho), _dp(u), _dp(T), _dp(noise), float(amplitude)),
                    "init_equilibrium")

    def set_populations(self, h):
        h = _f64(h, (self.Q, self.cells))
        self._check(lib().esbgk_set_populations(self._ctx, _dp(h)), "set_populations")

    def get_populations(self):
        h = np.empty((self.Q, self.cells))
        self._check(lib().esbgk_get_populations(self._ctx, _dp(h)), "get_populations")
        return h

    def get_state(self):
        n = lib().esbgk_state_bytes(self._ctx)
        buf = (ctypes.c_char * n)()
        self._check(lib().esbgk_get_state(self._ctx, buf, n), "get_state")
        return bytes(buf)

    def set_state(self, raw):
        buf = ctypes.create_string_buffer(raw, len(raw))
        self._check(lib().esbgk_set_state(self._ctx, buf, len(raw)), "set_state")

    def step(self, n=1):
        self._check(lib().esbgk_step(self._ctx, int(n)), "step")

    def set_inplace(self, mode):
        """esbgk_set_inplace: True / 1 pairs of steps in one buffer, False / 0
        two buffers, 2 (default) pairs where they were measured faster."""
        self._check(lib().esbgk_set_inplace(self._ctx, int(mode)), "set_inplace")

    @property
    def inplace_active(self):
        """True when steps advance in in-place pairs (esbgk_inplace_active)."""
        return lib().esbgk_inplace_active(self._ctx) == 1

    def set_graph_steps(self, steps):
        self._check(lib().esbgk_set_graph_steps(self._ctx, int(steps)), "set_graph_steps")

    @property
    def steps_done(self):
        return lib().esbgk_steps_done(self._ctx)

    def read_moments_raw(self):
        F = 9 if self.D == 2 else 14
        out = np.empty((F, self.cells))
        f = ctypes.c_int()
        self._check(lib().esbgk_read_moments(self._ctx, _dp(out), ctypes.byref(f)), "read_moments")
        return out

    def read_moments(self):
        return split_fields(self.read_moments_raw(), self.D)

    def _red(self, out):
        return dict(mass=out[0], energy=out[1], mom=out[2:5].copy(), mdot=out[5], residual=out[6], step=int(out[7]))

    def reduce(self):
        out = np.empty(8)
        self._check(lib().esbgk_reduce(self._ctx, _dp(out)), "reduce")
        return self._red(out)

    def reduce_noalloc(self):
        """esbgk_reduce_noalloc: the same reductions with no workspace scratch."""
        out = np.empty(8)
        self._check(lib().esbgk_reduce_noalloc(self._ctx, _dp(out)), "reduce_noalloc")
        return self._red(out)

    def set_reduce_interval(self, R):
        self._check(lib().esbgk_set_reduce_interval(self._ctx, int(R)), "set_reduce_interval")

    def last_reduction(self):
        out = np.empty(8)
        self._check(lib().esbgk_last_reduction(self._ctx, _dp(out)), "last_reduction")
        return self._red(out)


def make_problem(velset, nx, ny, nz=1, storage="f32", scheme="trapezoid", n_ref=0, Kn=0.1, Pr=1.0, varpi=0.5,
                 T_w=(1.0, 1.0), u_w=((0, 0, 0), (0, 0, 0)), g=(0, 0, 0), accommodation=(1.0, 1.0)):
    p = Problem()
    p.shape = Shape(_VELSET[velset], nx, ny, nz, 1, _STORAGE[storage], _SCHEME[scheme], n_ref)
    p.Kn, p.Pr, p.varpi = Kn, Pr, varpi
    for s in range(2):
        p.T_w[s] = T_w[s]
        for i in range(3):
            p.u_w[s][i] = u_w[s][i] if i < len(u_w[s]) else 0.0
    for i in range(3):
        p.g[i] = g[i] if i < len(g) else 0.0
    for s in range(2):
        p.specular[s] = 1.0 - accommodation[s]
    return p


class Batch:
    """Many independent channels advanced by one persistent kernel."""

    def __init__(self, problems, device="cuda:0"):
        import torch
        self.device = torch.device(device)
        self.n = len(problems)
        arr = (Problem * self.n)(*problems)
        self._arr = arr
        vs = problems[0].shape.velset
        info = lattice_info(vs)
        self.Q, self.D = info["Q"], info["D"]
        self.cells = [p.shape.nx * p.shape.ny * p.shape.nz for p in problems]
        L = lib()
        nbytes = L.esbgk_batch_workspace_bytes(arr, self.n)
        if nbytes == 0:
            raise EsbgkError(E_INVALID, "invalid batch")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._b = ctypes.c_void_p()
        rc = L.esbgk_batch_create(arr, self.n, ctypes.c_void_p(self.ws.data_ptr()), nbytes, _stream_ptr(self.device),
                                  ctypes.byref(self._b))
        if rc:
            raise EsbgkError(rc, "batch_create")

    def _check(self, rc, what):
        if rc:
            msg = lib().esbgk_batch_last_error(self._b)
            raise EsbgkError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            lib().esbgk_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_equilibrium(self, noise=None, amplitude=0.0):
        noise = _f64(noise, (-1,))
        self._check(lib().esbgk_batch_init_equilibrium(self._b, _dp(noise), float(amplitude)), "batch_init")

    def autotune(self, steps_per_trial=20):
        self._check(lib().esbgk_batch_autotune(self._b, int(steps_per_trial)), "batch_autotune")
        return self.layout()

    def set_layout(self, threads, nbins):
        self._check(lib().esbgk_batch_set_layout(self._b, int(threads), int(nbins)), "batch_set_layout")

    def layout(self):
        t, n = ctypes.c_int(), ctypes.c_int()
        self._check(lib().esbgk_batch_layout(self._b, ctypes.byref(t), ctypes.byref(n)), "batch_layout")
        return t.value, n.value

    def step(self, n=1):
        self._check(lib().esbgk_batch_step(self._b, int(n)), "batch_step")

    @property
    def steps_done(self):
        return lib().esbgk_batch_steps_done(self._b)

    def use_graphs(self, on):
        self._check(lib().esbgk_batch_use_graphs(self._b, int(bool(on))), "batch_use_graphs")

    def layout_info(self):
        mp, mc = ctypes.c_int(), ctypes.c_int64()
        self._check(lib().esbgk_batch_layout_info(self._b, ctypes.byref(mp), ctypes.byref(mc)), "batch_layout_info")
        t, nb = self.layout()
        piece, active = self.split
        return dict(threads=t, bins=nb, max_pieces_per_workgroup=mp.value, max_cells_per_thread=mc.value,
                    piece_cells=piece, split=active)

    def set_split(self, piece_cells):
        """Cut problems larger than piece_cells (a multiple of 64; 0: whole
        problems) into pieces spread over the workgroups."""
        self._check(lib().esbgk_batch_set_split(self._b, int(piece_cells)), "batch_set_split")

    @property
    def split(self):
        """(piece_cells, whether some problem is cut)."""
        pc, act = ctypes.c_int(), ctypes.c_int()
        self._check(lib().esbgk_batch_split(self._b, ctypes.byref(pc), ctypes.byref(act)), "batch_split")
        return pc.value, bool(act.value)

    def set_reduce_interval(self, R):
        self._check(lib().esbgk_batch_set_reduce_interval(self._b, int(R)), "batch_set_reduce_interval")

    @staticmethod
    def _reds(out):
        return [dict(mass=o[0], energy=o[1], mom=o[2:5].copy(), mdot=o[5], residual=o[6], step=int(o[7]))
                for o in out.reshape(-1, 8)]

    def reduce(self):
        """FP64 reductions of every problem at the current level (list of dicts)."""
        out = np.empty(8 * self.n)
        self._check(lib().esbgk_batch_reduce(self._b, _dp(out)), "batch_reduce")
        return self._reds(out)

    def last_reduction(self):
        out = np.empty(8 * self.n)
        self._check(lib().esbgk_batch_last_reduction(self._b, _dp(out)), "batch_last_reduction")
        return self._reds(out)

    def read_moments(self, i):
        F = 9 if self.D == 2 else 14
        out = np.empty((F, self.cells[i]))
        f = ctypes.c_int()
        self._check(lib().esbgk_batch_read_moments(self._b, int(i), _dp(out), ctypes.byref(f)), "batch_moments")
        return split_fields(out, self.D)

    def get_populations(self, i):
        h = np.empty((self.Q, self.cells[i]))
        self._check(lib().esbgk_batch_get_populations(self._b, int(i), _dp(h)), "batch_populations")
        return h


def tvd_velocity_set(velset="D2Q36GH"):
    """Abscissae c[Q][D] and weights w[Q] of a Gauss-Hermite product set of
    the paper's own scheme (D2Q16GH, D2Q36GH: the paper's, D2Q64GH, and the
    paper's 3-D set D3Q216GH)."""
    Q, N = ctypes.c_int(), ctypes.c_int()
    vid = _GH_SET[velset]
    rc = lib().esbgk_tvd_set_info(vid, ctypes.byref(Q), ctypes.byref(N), None, None)
    if rc:
        raise EsbgkError(rc, "tvd_set_info")
    c = np.empty((Q.value, 3 if velset == "D3Q216GH" else 2))
    w = np.empty(Q.value)
    rc = lib().esbgk_tvd_set_info(vid, None, None, _dp(c), _dp(w))
    if rc:
        raise EsbgkError(rc, "tvd_set_info")
    return c, w


def default_tvd_cfl(D):
    """Default Courant number of the TVD scheme: 0.45 in 2-D, 0.3 in 3-D, so
    that the Courant numbers of a field varying along every axis sum to 0.9."""
    return 0.45 if D == 2 else 0.3


def tvd_bounded(velset, n_ref, cfl, Kn, Pr, axes):
    """esbgk_tvd_bounded: OK (0) when axes * cfl <= 1 - dt/tau at rho = T = 1
    (forward Euler on the collision and the unsplit flux sum stays a convex
    combination), E_UNSTABLE otherwise, E_INVALID for bad arguments."""
    return lib().esbgk_tvd_bounded(_GH_SET[velset], int(n_ref), float(cfl), float(Kn), float(Pr), int(axes))


class TVDLattice:
    """The paper's own scheme (forward Euler, TVD minmod fluxes) on a
    Gauss-Hermite product set (the paper's D2Q36GH by default; D2Q16GH and
    D2Q64GH for velocity-set studies; the paper's 3-D set D3Q216GH with
    nz): periodic in every axis but the last, which is periodic or
    (walls=True) bounded by diffuse walls on its first and last nodes."""

    def __init__(self, nx=64, ny=64, storage="f32", cfl=None, n_ref=0, walls=False, velset="D2Q36GH",
                 device="cuda:0", nz=1):
        import torch
        self.device = torch.device(device)
        self.D = 3 if velset == "D3Q216GH" else 2
        # default Courant number inside the bound of tvd_bounded for a field
        # that varies along every axis (sum of |nu| = 0.9)
        cfl = default_tvd_cfl(self.D) if cfl is None else cfl
        self.cfl = float(cfl)
        nwall = ny if self.D == 2 else nz
        self.n_ref = n_ref if n_ref > 0 else (nwall - 1 if walls else nx)
        self.dims = (nx, ny) if self.D == 2 else (nx, ny, nz)
        self.cells = nx * ny * nz
        self.storage = storage
        self.walls = bool(walls)
        self.velset = velset
        Q, N = ctypes.c_int(), ctypes.c_int()
        if lib().esbgk_tvd_set_info(_GH_SET[velset], ctypes.byref(Q), ctypes.byref(N), None, None):
            raise EsbgkError(E_INVALID, f"unknown set {velset}")
        self.Q, self.N = Q.value, N.value
        self.shape = Shape(_GH_SET[velset], nx, ny, nz, int(self.walls), _STORAGE[storage], EULER, n_ref)
        L = lib()
        nbytes = L.esbgk_tvd_workspace_bytes(ctypes.byref(self.shape))
        if nbytes == 0:
            raise EsbgkError(E_INVALID, "invalid shape")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._t = ctypes.c_void_p()
        rc = L.esbgk_tvd_create(ctypes.byref(self.shape), float(cfl), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                _stream_ptr(self.device), ctypes.byref(self._t))
        if rc:
            msg = L.esbgk_tvd_last_error(None)
            raise EsbgkError(rc, f"tvd_create: {msg.decode() if msg else ''}")
        self.c, self.w = tvd_velocity_set(velset)

    def _check(self, rc, what):
        if rc:
            msg = lib().esbgk_tvd_last_error(self._t)
            raise EsbgkError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "_t", None) and self._t.value:
            lib().esbgk_tvd_destroy(self._t)
            self._t = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dt(self):
        return lib().esbgk_tvd_time_step(self._t)

    @property
    def steps_done(self):
        return lib().esbgk_tvd_steps_done(self._t)

    def set_gas(self, Kn, Pr, varpi=0.5):
        self._check(lib().esbgk_tvd_set_gas(self._t, Kn, Pr, varpi), "tvd_set_gas")
        axes = sum(1 for n in self.dims if n > 1)
        if axes and tvd_bounded(self.velset, self.n_ref, self.cfl, Kn, Pr, axes) == E_UNSTABLE:
            import warnings
            warnings.warn(f"TVD step not bounded for a field varying along {axes} axes: {axes} * cfl = "
                          f"{axes * self.cfl:.3g} > 1 - dt/tau", RuntimeWarning, stacklevel=2)

    def set_body_force(self, g):
        gg = np.zeros(3)
        gg[:len(g)] = g
        self._check(lib().esbgk_tvd_set_body_force(self._t, _dp(gg)), "tvd_set_body_force")

    def set_wall(self, side, T, u=(0.0, 0.0, 0.0)):
        uu = np.zeros(3)
        uu[:len(u)] = u
        self._check(lib().esbgk_tvd_set_wall(self._t, int(side), float(T), _dp(uu)), "tvd_set_wall")

    def init_equilibrium(self, rho=None, u=None, T=None, noise=None, amplitude=0.0):
        rho = _f64(rho, (self.cells,))
        u = _f64(u, (self.D, self.cells))
        T = _f64(T, (self.cells,))
        noise = _f64(noise, (self.Q, self.cells))
        self._check(lib().esbgk_tvd_init_equilibrium(self._t, _dp(rho), _dp(u), _dp(T), _dp(noise),
                                                     float(amplitude)), "tvd_init_equilibrium")

    def set_populations(self, h):
        h = _f64(h, (self.Q, self.cells))
        self._check(lib().esbgk_tvd_set_populations(self._t, _dp(h)), "tvd_set_populations")

    def get_populations(self):
        h = np.empty((self.Q, self.cells))
        self._check(lib().esbgk_tvd_get_populations(self._t, _dp(h)), "tvd_get_populations")
        return h

    def step(self, n=1):
        self._check(lib().esbgk_tvd_step(self._t, int(n)), "tvd_step")

    def read_moments(self):
        out = np.empty((9 if self.D == 2 else 14, self.cells))
        f = ctypes.c_int()
        self._check(lib().esbgk_tvd_read_moments(self._t, _dp(out), ctypes.byref(f)), "tvd_read_moments")
        return split_fields(out, self.D)
