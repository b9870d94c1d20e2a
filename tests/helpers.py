"""Shared test utilities: build the oracle problem and the GPU lattice from one
workload description, lay out the oracle's fields like the library's, and the
error metrics used for parity.

Two metrics per moment field X (rho, u, T, sigma, q):

* scale-relative: max |X_gpu - X_oracle| divided by the field's reference
  scale in the paper's nondimensionalisation (rho0, sqrt(R T0), T0, p0,
  p0 sqrt(R T0)), all equal to one, i.e. the absolute error in the paper's
  units. Gated at 1e-12 (FP64), 1e-6 (FP32 storage), 1e-3 (FP16 storage).
* signal-relative: max |X_gpu - X_oracle| / max |X_oracle - X_rest| with
  X_rest = 1 for rho and T and 0 otherwise: the error relative to the size of
  the signal the field carries. Its floor is the storage rounding of the
  populations (ulp of |h| ~ 0.1-0.3 per step) over the signal, so its gates
  are looser: 1e-10, 1e-4, 3e-2. A field whose signal is tiny or absent (a
  density change of 1e-8 in a weakly forced FP32 channel, the density of a
  uniformly accelerated gas) sits at the rounding floor that the other
  fields' larger deviations leave in it; its error is divided by a floor
  instead: 1e-5 for FP64 and FP32, 1e-2 for FP16. The absolute error such a
  field may carry is then 1e-15, 1e-9 and 3e-4: a thousand times below the
  scale gate for FP64 and FP32, a third of it for FP16, whose populations
  round at 1e-4 to 1e-3.
"""

import numpy as np

from oracle import lattice as OL
from oracle import quadrature

REST = {"rho": 1.0, "u": 0.0, "T": 1.0, "sigma": 0.0, "q": 0.0}


def oracle_velocity_set(name):
    return quadrature.velocity_set(name)


def oracle_problem(cfg, scheme="trapezoid"):
    vs = oracle_velocity_set(cfg["velset"])
    kw = dict(Kn=cfg["Kn"], Pr=cfg["Pr"], varpi=cfg.get("varpi", 0.5), walls=cfg.get("walls", False),
              g=tuple(cfg.get("g", (0, 0, 0))), scheme=scheme, n_ref=cfg.get("n_ref", 0))
    if kw["walls"]:
        gam = cfg.get("gamma", (1.0, 1.0))
        heat = cfg.get("heating", ((0.0, 0.0), (0.0, 0.0)))
        kw["wall_lo"] = OL.Wall(cfg["T_w"][0], tuple(cfg["u_w"][0]), gam[0], *heat[0])
        kw["wall_hi"] = OL.Wall(cfg["T_w"][1], tuple(cfg["u_w"][1]), gam[1], *heat[1])
    return OL.Problem(vs, tuple(cfg["dims"]), **kw)


def gpu_lattice(cfg, storage=None, scheme="trapezoid"):
    from paper_1209_6548_amd import Lattice
    dims = tuple(cfg["dims"]) + (1,) * (3 - len(cfg["dims"]))
    lat = Lattice(cfg["velset"], dims[0], dims[1], dims[2], walls=cfg.get("walls", False),
                  storage=storage or cfg.get("storage", "f32"), scheme=scheme, n_ref=cfg.get("n_ref", 0))
    lat.set_gas(cfg["Kn"], cfg["Pr"], cfg.get("varpi", 0.5))
    if cfg.get("walls", False):
        lat.set_wall(0, cfg["T_w"][0], cfg["u_w"][0])
        lat.set_wall(1, cfg["T_w"][1], cfg["u_w"][1])
        if "gamma" in cfg:
            lat.set_accommodation(0, cfg["gamma"][0])
            lat.set_accommodation(1, cfg["gamma"][1])
        if "heating" in cfg:
            lat.set_heating(0, *cfg["heating"][0])
            lat.set_heating(1, *cfg["heating"][1])
    lat.set_body_force(cfg.get("g", (0, 0, 0)))
    return lat


def oracle_fields(f, prob, cells=None, n=0):
    """The oracle's eq. mac fields of stored level n in the library's layout."""
    rho, u, T, sigma, q = OL.macroscopic(f, prob, cells, n=n)
    D = prob.D
    sig = np.array([sigma[:, i, j] for i in range(D) for j in range(i, D)])
    return {"rho": rho, "u": u.T.copy(), "T": T, "sigma": sig, "q": q.T.copy()}


TOL_SCALE = {"f64": 1e-12, "f32": 1e-6, "f16": 1e-3}
TOL_SIGNAL = {"f64": 1e-10, "f32": 1e-4, "f16": 3e-2}
SIGNAL_FLOOR = {"f64": 1e-5, "f32": 1e-5, "f16": 1e-2}


def field_abs_errors(gpu, orc):
    return {k: float(np.max(np.abs(np.asarray(gpu[k]) - np.asarray(orc[k])))) for k in REST}


def assert_parity(gpu, orc, storage, scale_tol=None, signal_tol=None):
    """Both metrics within their gates; returns them for reporting."""
    ea = field_abs_errors(gpu, orc)
    er = field_errors(gpu, orc, SIGNAL_FLOOR[storage])
    st = TOL_SCALE[storage] if scale_tol is None else scale_tol
    sg = TOL_SIGNAL[storage] if signal_tol is None else signal_tol
    assert max(ea.values()) < st, ("scale-relative", ea)
    assert max(er.values()) < sg, ("signal-relative", er)
    return ea, er


def field_errors(gpu, orc, floor=0.0):
    out = {}
    for k, rest in REST.items():
        den = max(float(np.max(np.abs(np.asarray(orc[k]) - rest))), floor)
        num = np.max(np.abs(np.asarray(gpu[k]) - np.asarray(orc[k])))
        out[k] = num / den if den > 0 else num
    return out


def init_fields(cfg, cells, D, Q, seed=11, amp=0.02, du=0.03, dT=0.03):
    """Seeded non-uniform start (rho, u, T fields and population noise)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.03 * rng.uniform(-1, 1, cells)
    u = du * rng.uniform(-1, 1, (D, cells))
    T = 1.0 + dT * rng.uniform(-1, 1, cells)
    xi = rng.standard_normal((Q, cells))
    return rho, u, T, xi, amp


def small_cfg(velset, dims, walls, force=True, Kn=0.05, Pr=2 / 3, varpi=0.5):
    D = 2 if velset == "D2Q37" else 3
    cfg = dict(velset=velset, dims=dims, walls=walls, Kn=Kn, Pr=Pr, varpi=varpi,
               g=(0.02, -0.01, 0.005)[:D] + (0.0,) * (3 - D) if force else (0.0, 0.0, 0.0))
    if walls:
        if D == 2:
            cfg["u_w"] = ((-0.04, 0.0, 0.0), (0.05, 0.0, 0.0))
        else:
            cfg["u_w"] = ((-0.04, 0.02, 0.0), (0.05, -0.01, 0.0))
        cfg["T_w"] = (0.98, 1.04)
    return cfg


class StoredPopulations:
    """Read-only (Q, M) view of the physical populations f = w (1 + h) over a
    raw stored state (h in its storage dtype), converting only the entries an
    index asks for. Lets the oracle step sampled cells of grids whose FP64
    populations would not fit in host memory."""

    def __init__(self, raw, Q, M, dtype, w):
        self.h = np.frombuffer(raw, dtype=dtype, count=Q * M).reshape(Q, M)
        self.w = np.asarray(w, dtype=np.float64)
        self.shape = (Q, M)

    def __getitem__(self, key):
        a, b = key
        vals = np.asarray(self.h[a, b], dtype=np.float64)
        return self.w[a] * (1.0 + vals)


def ulp(x, dtype):
    """Spacing of dtype at |x| (elementwise), as float64."""
    return np.spacing(np.abs(np.asarray(x, dtype=np.float64)).astype(dtype)).astype(np.float64)
