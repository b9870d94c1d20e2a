"""The paper's own space-time scheme (Sec. 3.1) on the paper's velocity set
(test infrastructure only).

Velocity set (Sec. 2.2): the tensor product of the n-point 1-D Gauss-Hermite
rule of eq. weight, c_alpha = (xi_i, xi_j), w_alpha = w_i w_j. With n = 6
each axis is exact to degree 11 (the paper's choice for N = 4). The abscissae
are off the lattice, so streaming is a finite-difference flux update.

Scheme (Sec. 3.1): forward Euler in time; the advection term is a TVD
finite-volume flux difference along each axis with the minmod limiter,

  f^{n+1} = f^n - nu_x [F_{i+1/2} - F_{i-1/2}] - nu_y [F_{j+1/2} - F_{j-1/2}]
            + (dt/tau)(f^ES - f^n) + dt F,

nu = c dt / dx, and for c > 0

  F_{i+1/2} = f_i + (1 - nu)/2 (f_{i+1} - f_i) Psi(Theta_i),
  Theta_i = (f_i - f_{i-1}) / (f_{i+1} - f_i),  Psi = max(0, min(1, Theta)).

The paper prints only c > 0; for c < 0 the upwind side is i + 1 (the same
formula mirrored):

  F_{i+1/2} = f_{i+1} - (1 - |nu|)/2 (f_{i+1} - f_i) Psi(Theta'_{i+1}),
  Theta'_{i+1} = (f_{i+2} - f_{i+1}) / (f_{i+1} - f_i).

Where the denominator of Theta vanishes the limited term (f_{i+1} - f_i) Psi
is zero whatever Psi is; it is taken as zero. Every right-hand-side term is
evaluated at level n. The collision and force terms are those of the
on-lattice oracle with the Euler weights (omega = dt/tau, phi = 1), built
from the moments of f^n.

Boundaries: periodic in every axis, or (walls=True) diffuse walls across
the last axis after Sec. 3.2 (the first version of the boundary conditions
of Sofonea et al. that the paper adopts). The first and last nodes of that
axis lie on the walls and are updated like every node; the two ghost nodes
beyond each wall that the stencil reaches hold copies of the wall node.
After the update, the wall node's populations that move into the gas
(c.n > 0, n the inward normal) are replaced by rho_W S(T_W, u_W), with
rho_W = sum_{c.n<0} |c.n| f / sum_{c.n>0} |c.n| S over the populations of
the first node off the wall (the superscripts 0 and 1 of the paper's
formula are node rows along the normal, as j in f^{n,j}): the wall emits
the normal particle flux that reaches it from that node. The scheme does
not conserve mass exactly: where the flow near the wall is not uniform
the emitted flux differs from what crosses the wall face, by a small
amount per step. Walls are fully diffuse (the paper implements only
gamma = 1) at a fixed temperature.

Time step: dt = CFL dx / max|c|, CFL in (0, 1] (the TVD update is stable for
|nu| <= 1); dx = 1/N_L, N_L = nx for periodic boxes and the wall distance
ny - 1 in nodes for channels.
"""

from dataclasses import dataclass, field
from itertools import product

import numpy as np

from . import lattice, model, quadrature


class ProductSet:
    """Tensor-product Gauss-Hermite set (no rest velocity for even n).

    Order: the representatives (first component positive), sorted by |c|^2
    and then by descending tuple of root indices, followed by their opposites
    in the same order, so that alpha + P holds -c_alpha (P = Q/2)."""

    def __init__(self, n=6, D=2, N=4):
        if n % 2:
            raise ValueError("an even rule has no zero root: every velocity has an opposite")
        xi, w1 = quadrature.hermite_rule_1d(n)
        half = n // 2                               # xi[half:] are the positive roots
        # the rule is symmetric; take the positive half and mirror it so that
        # opposite velocities are exact negatives of each other
        xi = np.concatenate([-xi[half:][::-1], xi[half:]])
        w1 = np.concatenate([w1[half:][::-1], w1[half:]])
        reps = []
        for idx in product(range(n), repeat=D):
            if idx[0] >= half:                      # first component positive
                reps.append(idx)
        # |c|^2 summed over the sorted squares, so that permuted tuples tie
        # exactly and the root-index rule (not rounding) orders them
        reps.sort(key=lambda t: (sum(sorted(xi[k] ** 2 for k in t)), tuple(-k for k in t)))
        opp = [tuple(n - 1 - k for k in t) for t in reps]   # xi[n-1-k] = -xi[k]
        order = reps + opp
        self.name = f"D{D}Q{n ** D}GH"
        self.idx = np.array(order, dtype=np.int64)          # root index per axis
        self.c = xi[self.idx]
        self.w = np.prod(w1[self.idx], axis=1)
        self.Q, self.D = self.c.shape
        self.P = self.Q // 2
        self.N = N
        self.degree = 2 * n - 1                              # per axis
        self.roots = xi
        self.e = None
        self.opposite = np.concatenate([np.arange(self.P, self.Q), np.arange(0, self.P)])


@dataclass
class TVDProblem:
    """A lattice for the paper's scheme. dims = (nx, ny); walls=True puts
    diffuse walls on the first and last node rows of the last axis."""
    vs: object
    dims: tuple
    Kn: float
    Pr: float
    varpi: float = 0.5
    g: tuple = (0.0, 0.0, 0.0)
    cfl: float = 0.5
    n_ref: int = 0
    walls: bool = False
    wall_lo: lattice.Wall = field(default_factory=lattice.Wall)
    wall_hi: lattice.Wall = field(default_factory=lattice.Wall)

    def __post_init__(self):
        self.D = self.vs.D
        self.N = self.vs.N
        if len(self.dims) != self.D:
            raise ValueError("dims must have one extent per dimension")
        if not 0.0 < self.cfl <= 1.0:
            raise ValueError("the TVD update needs 0 < CFL <= 1")
        if self.walls:
            if self.dims[-1] < 3:
                raise ValueError("a channel needs two wall nodes and at least one node between them")
            for w in (self.wall_lo, self.wall_hi):
                if w.gamma != 1.0 or w.heat_amp != 0.0:
                    raise ValueError("the scheme's walls are fully diffuse at a fixed temperature")
        if self.n_ref == 0:
            self.n_ref = self.dims[-1] - 1 if self.walls else self.dims[0]
        self.dx = 1.0 / self.n_ref
        self.dt = self.cfl * self.dx / np.abs(self.vs.c).max()
        self.hs = 0.0                      # forward Euler: no change of variable
        self.scheme = "euler"
        self.b = model.b_from_prandtl(self.Pr)
        self.gvec = np.asarray(self.g[: self.D], dtype=np.float64)
        self.M = int(np.prod(self.dims))

    def grid(self, f):
        """View a (Q, M) state as (Q, *reversed dims): axis -1 is x."""
        return f.reshape((self.vs.Q,) + tuple(self.dims[::-1]))


def _psi(theta):
    """The minmod limiter of Sec. 3.1."""
    return np.maximum(0.0, np.minimum(1.0, theta))


def _limited(num, den):
    """den * Psi(num / den), zero where den vanishes."""
    out = np.zeros_like(den)
    nz = den != 0.0
    out[nz] = den[nz] * _psi(num[nz] / den[nz])
    return out


def face_flux(f, nu, axis):
    """Upwind TVD flux F_{i+1/2} at the face between cell i and i + 1 along
    the grid axis `axis` for one velocity (f an array over cells, periodic
    within the array); nu = c dt / dx of that velocity along the axis."""
    fm1 = np.roll(f, 1, axis)        # f_{i-1}
    fp1 = np.roll(f, -1, axis)       # f_{i+1}
    fp2 = np.roll(f, -2, axis)       # f_{i+2}
    d = fp1 - f                      # f_{i+1} - f_i
    if nu > 0:
        return f + 0.5 * (1.0 - nu) * _limited(f - fm1, d)
    return fp1 - 0.5 * (1.0 - abs(nu)) * _limited(fp2 - fp1, d)


def flux_difference(f, nu, axis, walls):
    """nu [F_{i+1/2} - F_{i-1/2}] along one grid axis for one velocity. The
    axis is extended by two nodes on each side: periodic images, or (walls)
    ghost nodes that copy the wall node. The fluxes are taken on the
    extended array, whose own wrap-around never reaches a kept value."""
    n = f.shape[axis]
    pad = [(0, 0)] * f.ndim
    pad[axis] = (2, 2)
    ext = np.pad(f, pad, mode="edge" if walls else "wrap")
    Fr = face_flux(ext, nu, axis)                # F at the right face of every extended node
    keep = np.arange(2, n + 2)
    right = np.take(Fr, keep, axis=axis)         # F_{i+1/2}
    left = np.take(Fr, keep - 1, axis=axis)      # F_{i-1/2} = F_{(i-1)+1/2}
    return nu * (right - left)


def advection(f, prob):
    """The flux-difference term nu_x [F_{i+1/2} - F_{i-1/2}] + nu_y [...] of
    every velocity at every cell, shape (Q, M)."""
    g = prob.grid(f)
    out = np.zeros_like(g)
    for a in range(prob.vs.Q):
        for d in range(prob.D):
            nu = prob.vs.c[a, d] * prob.dt / prob.dx
            if nu == 0.0:
                continue
            axis = prob.D - 1 - d    # grid axis of coordinate d (x is last)
            walls = prob.walls and d == prob.D - 1
            out[a] += flux_difference(g[a], nu, axis, walls)
    return out.reshape(f.shape)


def wall_state(prob, side):
    """S_alpha(T_W, u_W) (eq. feq0 at order N, rho = 1) of wall `side` and
    c.n with n its inward normal."""
    w = prob.wall_lo if side == 0 else prob.wall_hi
    u = np.asarray(w.u[: prob.D], dtype=np.float64)
    S = model.truncated_maxwellian(np.ones(1), u[None, :], np.full(1, w.T), prob.vs.c, prob.vs.w, prob.N)[:, 0]
    cn = prob.vs.c[:, -1] * (1.0 if side == 0 else -1.0)
    return S, cn


def wall_emission(f, prob):
    """Sec. 3.2: the wall nodes' populations with c.n > 0 become rho_W S,
    rho_W from the flux toward the wall at the first node off it."""
    g = prob.grid(f).copy()
    n = prob.dims[-1]
    for side, (jw, ji) in enumerate(((0, 1), (n - 1, n - 2))):
        S, cn = wall_state(prob, side)
        inc, out = cn < 0, cn > 0
        wall = g[:, jw]
        inner = g[:, ji]
        rho_w = np.tensordot(np.abs(cn[inc]), inner[inc], axes=1) / np.dot(np.abs(cn[out]), S[out])
        wall[out] = S[out].reshape((-1,) + (1,) * (wall.ndim - 1)) * rho_w[None]
    return g.reshape(f.shape)


def step(f, prob):
    """One step of the paper's scheme: every term at level n, then the wall
    emission of Sec. 3.2 (walls=True)."""
    f1 = lattice.collide(f, prob) - advection(f, prob)
    return wall_emission(f1, prob) if prob.walls else f1


def run(f, prob, nsteps):
    for _ in range(nsteps):
        f = step(f, prob)
    return f


def macroscopic(f, prob):
    """rho, u, T, sigma, q of the stored level (the physical f itself)."""
    return model.macroscopic(f, prob.vs.c)


def equilibrium_state(prob, rho, u, T, noise=None, amplitude=0.0):
    """f_alpha = rho S_alpha(T, u) (eq. feq0 at order N) (1 + amplitude xi)."""
    f = model.truncated_maxwellian(np.asarray(rho, float), np.asarray(u, float), np.asarray(T, float),
                                   prob.vs.c, prob.vs.w, prob.N)
    if noise is not None:
        f = f * (1.0 + amplitude * noise)
    return f
