"""Write the FP64 oracle fixtures of the configuration-length parity tests.

    python -m tests.golden.make_fixtures [name ...]     # default: all

Calls only oracle/ (the FP64 CPU solver) and the seeded input generators of
paper_1209_6548_amd/workloads.py (inputs, no arithmetic of the method). Each
fixture is tests/golden/<name>.npz: the oracle's eq. mac fields (rho, u, T,
sigma, q in the library's layout) at checkpoint levels, its FP64 reductions
(mass, energy, mass flow rate) there, and the residual
||u^n - u^(n-R)||_2 / ||u^n||_2 every R = 1000 steps. The instances are
reduced forms of the benchmark workloads, run for their own length:

* column_1024_pr{067,1}: the 1024 x 1024 force-driven Poiseuille channel
  with thermal walls (T = 1.0 / 1.05, g_x = 1e-5 lattice units, Kn = 0.05,
  D2Q37), which is uniform along x, as its 1 x 1024 column; 50 000 steps from
  rest, for Pr = 2/3 and Pr = 1.
* box_32: the decaying thermal shear wave of the 256^3 box (D3Q39, Kn =
  0.02, Pr = 2/3, u_x = 1e-3 sin(2 pi z/L), T = 1 + 1e-3 cos(2 pi y/L), 1e-5
  population noise) on 32^3 cells, the same k L and Kn, for 250 steps: the
  same time in units of L/sqrt(R T0) as 2000 steps of the 256^3 box (about
  five e-folds of the shear wave). The same 2000 steps on 32^3 would be eight
  times longer and leave no signal above the noise.
* channel_col_256: the 512 x 512 x 256 channel (D3Q39, walls across z at
  T = 1.0 / 1.02, g_x = 5e-5 lattice units, Kn = 0.2, Pr = 2/3), uniform in
  x and y, as its 1 x 1 x 256 column, run from rest until the residual falls
  below 1e-10 (steady state).
* batch3: one channel of each case of the 512-channel mix (Couette,
  force-driven Poiseuille, Fourier; the narrowest of each), 20 000 steps.

The walls and the moments follow oracle/lattice.py (readings of the paper's
Sec. 3.2 and eq. mac); trapezoidal scheme throughout.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import lattice as OL  # noqa: E402
from oracle import quadrature  # noqa: E402
from paper_1209_6548_amd import workloads  # noqa: E402

R_RES = 1000


def fields(f, prob):
    rho, u, T, sigma, q = OL.macroscopic(f, prob)
    D = prob.D
    sig = np.array([sigma[:, i, j] for i in range(D) for j in range(i, D)])
    return {"rho": rho, "u": u.T.copy(), "T": T, "sigma": sig, "q": q.T.copy()}


def problem(vs, cfg):
    kw = dict(Kn=cfg["Kn"], Pr=cfg["Pr"], varpi=cfg.get("varpi", 0.5), walls=cfg["walls"], g=tuple(cfg["g"]))
    if cfg["walls"]:
        kw["wall_lo"] = OL.Wall(cfg["T_w"][0], tuple(cfg["u_w"][0]))
        kw["wall_hi"] = OL.Wall(cfg["T_w"][1], tuple(cfg["u_w"][1]))
    if "n_ref" in cfg:
        kw["n_ref"] = cfg["n_ref"]
    return OL.Problem(vs, tuple(cfg["dims"]), **kw)


def run(name, vs, cfg, f, checkpoints, until_residual=None, max_steps=None, log=print):
    """Step the oracle, recording fields and reductions at the checkpoints and
    the residual every R_RES steps; with until_residual, stop at the first
    residual below it (a checkpoint is taken there)."""
    prob = problem(vs, cfg)
    out = {"config": json.dumps({k: v for k, v in cfg.items() if k not in ("rho", "u", "T")}),
           "residual_steps": [], "residual": []}
    level, u_prev = 0, None
    cps = sorted(checkpoints)
    end = max_steps if until_residual else cps[-1]
    t0 = time.time()
    done = []
    while level < end:
        nxt = min([c for c in cps if c > level] + [(level // R_RES + 1) * R_RES, end])
        f = OL.run(f, prob, nxt - level, n0=level)
        level = nxt
        stop = False
        if level % R_RES == 0:
            red = OL.reductions(f, prob, u_prev=u_prev)
            if u_prev is not None:
                out["residual_steps"].append(level)
                out["residual"].append(red["residual"])
                stop = until_residual is not None and red["residual"] < until_residual
            u_prev = red["u"]
        if level in cps or stop or level == end:
            red = OL.reductions(f, prob)
            fl = fields(f, prob)
            for k, v in fl.items():
                out[f"{k}@{level}"] = v
            out[f"mass@{level}"] = red["mass"]
            out[f"energy@{level}"] = red["energy"]
            out[f"mdot@{level}"] = red["mdot"]
            done.append(level)
            log(f"[{name}] level {level}: mass {red['mass']:.15g} mdot {red['mdot']:.6e} "
                f"({time.time() - t0:.0f} s)")
        if stop:
            break
    out["checkpoints"] = np.array(done)
    out["residual_steps"] = np.array(out["residual_steps"])
    out["residual"] = np.array(out["residual"])
    np.savez_compressed(os.path.join(HERE, f"{name}.npz"), **out)
    return out


def rest_state(vs, cfg):
    prob = problem(vs, cfg)
    M = prob.M
    return OL.equilibrium_state(prob, np.ones(M), np.zeros((M, prob.D)), np.ones(M))


def column_1024(Pr):
    vs = quadrature.d2q37()
    cfg = workloads.poiseuille_thermal_1024(vs.r, Pr=Pr)
    cfg = dict(cfg, dims=(1, 1024))       # uniform along x: its column
    name = "column_1024_pr067" if Pr < 0.9 else "column_1024_pr1"
    return run(name, vs, cfg, rest_state(vs, cfg), [5000, 20000, 50000])


def box_32():
    vs = quadrature.d3q39()
    cfg = workloads.shear_wave_box(vs.r, n=32)
    prob = problem(vs, cfg)
    xi = workloads.noise(cfg["noise_seed"], vs.Q, prob.M)
    f = OL.equilibrium_state(prob, cfg["rho"], cfg["u"].T, cfg["T"], xi, cfg["noise_amp"])
    return run("box_32", vs, dict(cfg, steps=250), f, [50, 250])


def channel_col_256():
    vs = quadrature.d3q39()
    cfg = workloads.channel_3d(vs.r, nx=1, ny=1, nz=256)
    return run("channel_col_256", vs, cfg, rest_state(vs, cfg), [2000], until_residual=1e-10, max_steps=60000)


def batch3():
    vs = quadrature.d2q37()
    specs = workloads.channel_batch(vs.r)
    picked = []
    for case in ("couette", "poiseuille", "fourier"):
        idx = min((i for i, s in enumerate(specs) if s["case"] == case), key=lambda i: specs[i]["dims"][1])
        picked.append(idx)
    outs = {}
    for idx in picked:
        cfg = dict(specs[idx], index=idx)
        outs[idx] = run(f"batch3_{idx}", vs, cfg, rest_state(vs, cfg), [2000, 20000])
    return outs


JOBS = {"column_1024_pr067": lambda: column_1024(2 / 3), "column_1024_pr1": lambda: column_1024(1.0),
        "box_32": box_32, "channel_col_256": channel_col_256, "batch3": batch3}


if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    for n in names:
        JOBS[n]()
