"""Seeded synthetic workloads (inputs only; no arithmetic of the method).

The paper's benchmarks are 1-D channel flows (Couette, Fourier, force-driven
Poiseuille) and an unsteady heating problem whose comparison data (DSMC,
LVDSMC, R13, numerical ES-BGK) is not available. These recipes stand in for
them with the same geometry class, at the sizes the library is measured on.
Both the HIP path and the CPU oracle receive the same fields and noise
arrays from here.

Units. Wall speeds and body forces quoted "in lattice units" (cells per step
and cells per step^2) are converted to the paper's nondimensional units with
the velocity scale r of the velocity set (c = r e) and the number of cells
N_L across the reference length:  u = r u_lat,  g = r^2 N_L g_lat.
"""

import numpy as np


def noise(seed, Q, cells):
    """Standard normal xi[Q][cells] (PCG64). The initial populations are
    f_alpha = f_eq,alpha (1 + amplitude xi_alpha)."""
    return np.random.default_rng(seed).standard_normal((Q, cells))


def u_nd(r, u_lat):
    return r * u_lat


def g_nd(r, n_ref, g_lat):
    return r * r * n_ref * g_lat


def couette_1x32(r):
    """Planar Couette: 1 x 32 cells between diffuse walls moving at +-0.05
    (lattice units), T_w = 1, Kn = 0.1, Pr = 2/3, rest start plus 1e-4 noise,
    FP64; 20 000 steps."""
    uw = u_nd(r, 0.05)
    return dict(name="couette_1x32", velset="D2Q37", dims=(1, 32), walls=True, Kn=0.1, Pr=2 / 3, varpi=0.5,
                T_w=(1.0, 1.0), u_w=((-uw, 0, 0), (uw, 0, 0)), g=(0.0, 0.0, 0.0), noise_seed=0,
                noise_amp=1e-4, steps=20000, storage="f64")


def poiseuille_thermal_1024(r, Pr=2 / 3, storage="f32", n=1024):
    """Force-driven Poiseuille with thermal walls: n x n cells (periodic x,
    diffuse walls in y at T = 1.0 and 1.05, at rest), g_x = 1e-5 (lattice
    units), Kn = 0.05; rest start; 50 000 steps."""
    return dict(name=f"poiseuille_thermal_{n}x{n}", velset="D2Q37", dims=(n, n), walls=True, Kn=0.05, Pr=Pr,
                varpi=0.5, T_w=(1.0, 1.05), u_w=((0, 0, 0), (0, 0, 0)), g=(g_nd(r, n, 1e-5), 0.0, 0.0),
                noise_seed=None, noise_amp=0.0, steps=50000, storage=storage)


def shear_wave_box(r, n=256, storage="f32", seed=2):
    """Decaying thermal shear wave in a periodic box of n^3 cells:
    u_x = 1e-3 sin(2 pi z / L), T = 1 + 1e-3 cos(2 pi y / L), rho = 1, plus
    1e-5 noise; Kn = 0.02, Pr = 2/3 (amplitudes nondimensional)."""
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ux = 1e-3 * np.sin(2 * np.pi * (z.reshape(-1) + 0.5) / n)
    T = 1.0 + 1e-3 * np.cos(2 * np.pi * (y.reshape(-1) + 0.5) / n)
    u = np.zeros((3, n ** 3))
    u[0] = ux
    return dict(name=f"shear_wave_{n}^3", velset="D3Q39", dims=(n, n, n), walls=False, Kn=0.02, Pr=2 / 3,
                varpi=0.5, g=(0.0, 0.0, 0.0), rho=np.ones(n ** 3), u=u, T=T, noise_seed=seed, noise_amp=1e-5,
                steps=2000, storage=storage)


def channel_3d(r, nx=512, ny=512, nz=256, storage="f16"):
    """3-D channel: nx x ny x nz cells, diffuse walls in z at T = 1.0 / 1.02,
    g_x = 5e-5 (lattice units), Kn = 0.2, Pr = 2/3; rest start; 100 000
    steps."""
    return dict(name=f"channel_{nx}x{ny}x{nz}", velset="D3Q39", dims=(nx, ny, nz), walls=True, Kn=0.2, Pr=2 / 3,
                varpi=0.5, T_w=(1.0, 1.02), u_w=((0, 0, 0), (0, 0, 0)), g=(g_nd(r, nz, 5e-5), 0.0, 0.0),
                noise_seed=None, noise_amp=0.0, steps=100000, storage=storage)


def channel_batch(r, n=512, seed=3, nx=4, ny_range=(16, 512), storage="f32"):
    """512 independent 2-D channels: ny uniform in [16, 512], nx = 4 periodic,
    Kn log-uniform in [0.01, 0.5], Pr in {2/3, 0.8, 1}; cases Couette
    (u_w = +-0.05 lattice units), force-driven Poiseuille (g log-uniform in
    [1e-6, 1e-4] lattice units) and Fourier (wall temperatures 1 -+ dT/2,
    dT uniform in [0.01, 0.1]); 20 000 steps."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        ny = int(rng.integers(ny_range[0], ny_range[1] + 1))
        Kn = float(np.exp(rng.uniform(np.log(0.01), np.log(0.5))))
        Pr = float(rng.choice([2 / 3, 0.8, 1.0]))
        case = int(rng.integers(0, 3))
        T_w, u_w, g = (1.0, 1.0), ((0, 0, 0), (0, 0, 0)), (0.0, 0.0, 0.0)
        if case == 0:
            uw = u_nd(r, 0.05)
            u_w = ((-uw, 0, 0), (uw, 0, 0))
        elif case == 1:
            g = (g_nd(r, ny, float(np.exp(rng.uniform(np.log(1e-6), np.log(1e-4))))), 0.0, 0.0)
        else:
            dT = float(rng.uniform(0.01, 0.1))
            T_w = (1.0 - dT / 2, 1.0 + dT / 2)
        out.append(dict(name=f"channel{i}", velset="D2Q37", dims=(nx, ny), walls=True, Kn=Kn, Pr=Pr, varpi=0.5,
                        T_w=T_w, u_w=u_w, g=g, case=("couette", "poiseuille", "fourier")[case], storage=storage))
    return out
