"""Space-time scheme of the oracle: exact on-lattice streaming, the diffuse
wall, collision with the ES-BGK equilibrium and the body force (test
infrastructure only).

Layout. A state is an array f of shape (Q, M): the post-collision populations
f_alpha (absolute values, eq. lbgk's f_alpha = w_alpha f(c_alpha)/omega) of
M cells, flattened with x fastest, then y, then z.

Readings of the paper taken here (the paper's own scheme is an off-lattice
finite-difference one, Sec. 3.1; it notes that first-order upwind differencing
is the standard stream-collision scheme, which is what an on-lattice set with
integer e_alpha permits exactly):

* Space: one time step moves population alpha by e_alpha cells, so
  dt = dx / r with dx = 1/N_L (N_L cells across the reference length L that
  defines Kn, Sec. 2.2).
* Time: the relaxation and force terms of eq. lbgk are integrated along the
  characteristic either with forward Euler (the paper's Sec. 3.1 update at
  Courant number one) or with the trapezoidal rule, made explicit by the usual
  change of variable fbar = f + (dt/2tau)(f - f_ES) - (dt/2) F. Both give
      fbar*_alpha = fbar_alpha - omega (fbar_alpha - f_ES,alpha) + phi dt F_alpha
  with (omega, phi) = (dt/tau, 1) for Euler and (2x/(2+x), 1 - omega/2),
  x = dt/tau, for the trapezoidal rule, where f_ES and F are built from the
  moments of the physical f recovered from fbar (``physical_state``).
* Walls (Sec. 3.2): flat walls lie half a cell outside the first and last
  layer along the wall axis (the last spatial axis). With full accommodation
  (the paper's choice), every population that streams across a wall in one
  step is re-emitted as rho_W S(T_W, u_W): the ghost cells beyond the wall
  carry rho_W E_alpha, E = S(T_W, u_W) of eq. feq0 truncated at the bulk
  order N, with rho_W per wall-parallel column fixed by the flux balance of
  Sec. 3.2 where |xi . n| becomes the number of layers |e_n| that velocity
  crosses in one step.
* Maxwell's model (Sec. 3.2): a fraction gamma of the particles that hit a
  wall is re-emitted diffusely and 1 - gamma is reflected specularly. On the
  lattice a population alpha pulled from beyond the low wall (source layer
  t - e_n < 0) is gamma rho_W E_alpha + (1 - gamma) f_alpha'(column, layer
  e_n - 1 - t), alpha' the velocity with e_n negated: the particle that left
  that layer towards the wall, mirrored in the plane half a cell below layer
  0; likewise at the high wall with the plane half a cell above layer
  n - 1. rho_W keeps its definition, so the diffuse part returns the
  fraction gamma of the flux that crossed and the specular part the rest.
* Unsteady boundary heating (Sec. 4.2): a wall temperature
  T_W(t) = T + A sin(theta t), t in units of L / sqrt(R T0). The step that
  advances the stored level n to n + 1 streams during [n dt, (n + 1) dt] and
  re-emits at the midpoint, T_W((n + 1/2) dt); the moments of level n are
  those of the pull of that step.
"""

from dataclasses import dataclass, field

import numpy as np

from . import model


@dataclass
class Wall:
    T: float = 1.0
    u: tuple = (0.0, 0.0, 0.0)
    gamma: float = 1.0      # accommodation: fraction re-emitted diffusely (Sec. 3.2)
    heat_amp: float = 0.0   # unsteady heating T + heat_amp sin(heat_freq t) (Sec. 4.2)
    heat_freq: float = 0.0

    def temperature(self, t):
        return self.T + self.heat_amp * np.sin(self.heat_freq * t)


@dataclass
class Problem:
    """One lattice problem. dims = (nx, ny) or (nx, ny, nz), x fastest.
    walls=True puts diffuse walls across the last axis; every other axis (and
    every axis when walls=False) is periodic. n_ref is N_L; by default the
    extent of the wall axis (channels) or of x (periodic boxes)."""
    vs: object
    dims: tuple
    Kn: float
    Pr: float
    varpi: float = 0.5
    walls: bool = False
    wall_lo: Wall = field(default_factory=Wall)
    wall_hi: Wall = field(default_factory=Wall)
    g: tuple = (0.0, 0.0, 0.0)
    scheme: str = "trapezoid"
    n_ref: int = 0

    def __post_init__(self):
        vs = self.vs
        self.D = vs.D
        self.N = vs.N
        if len(self.dims) != self.D:
            raise ValueError("dims must have one extent per dimension")
        if self.n_ref == 0:
            self.n_ref = self.dims[-1] if self.walls else self.dims[0]
        self.dx = 1.0 / self.n_ref
        self.dt = self.dx / vs.r
        if self.scheme == "trapezoid":
            self.hs = 0.5 * self.dt
        elif self.scheme == "euler":
            self.hs = 0.0
        else:
            raise ValueError("scheme is 'trapezoid' or 'euler'")
        self.b = model.b_from_prandtl(self.Pr)
        self.gvec = np.asarray(self.g[: self.D], dtype=np.float64)
        self.M = int(np.prod(self.dims))
        # cell coordinates, x fastest
        grids = np.meshgrid(*[np.arange(n) for n in self.dims[::-1]], indexing="ij")
        self.coords = np.stack([gr.reshape(-1) for gr in grids[::-1]], axis=1)
        if self.walls:
            self.E_lo = self._wall_populations(self.wall_lo)
            self.E_hi = self._wall_populations(self.wall_hi)
            e = vs.e
            flipped = e.copy()
            flipped[:, -1] = -flipped[:, -1]
            lookup = {tuple(v): k for k, v in enumerate(e)}
            self.mirror = np.array([lookup[tuple(v)] for v in flipped])

    def _wall_populations(self, wall, T=None):
        u = np.asarray(wall.u[: self.D], dtype=np.float64)
        if u[-1] != 0.0:
            raise ValueError("wall velocity must be tangential")
        if not 0.0 <= wall.gamma <= 1.0:
            raise ValueError("accommodation must lie in [0, 1]")
        E = model.truncated_maxwellian(np.ones(1), u[None, :], np.array([wall.T if T is None else T]),
                                       self.vs.c, self.vs.w, self.N)
        return E[:, 0]

    def wall_emission(self, n):
        """S(T_W, u_W) of both walls for the step from level n to n + 1 (wall
        temperatures at the midpoint (n + 1/2) dt of its streaming)."""
        t = (n + 0.5) * self.dt
        out = []
        for wall, static in ((self.wall_lo, self.E_lo), (self.wall_hi, self.E_hi)):
            if wall.heat_amp == 0.0:
                out.append(static)
            else:
                out.append(self._wall_populations(wall, wall.temperature(t)))
        return out

    # ---- indexing -------------------------------------------------------
    def flat(self, p):
        """Flat index of integer coordinates p (..., D)."""
        idx = np.zeros(p.shape[:-1], dtype=np.int64)
        stride = 1
        for a, n in enumerate(self.dims):
            idx = idx + p[..., a] * stride
            stride *= n
        return idx

    def column(self, p):
        """Index of the wall-parallel column of coordinates p (the coordinates
        along every axis but the last)."""
        idx = np.zeros(p.shape[:-1], dtype=np.int64)
        stride = 1
        for a, n in enumerate(self.dims[:-1]):
            idx = idx + p[..., a] * stride
            stride *= n
        return idx

    @property
    def ncols(self):
        return int(np.prod(self.dims[:-1]))


def sources(prob, cells):
    """Pull sources of the given target cells: for each (alpha, cell) the flat
    index of x - e_alpha with periodic wrap, or -1 / -2 when that point lies
    beyond the low / high wall; plus the column of the (wrapped) source."""
    e = prob.vs.e
    p = prob.coords[cells]                                   # (K, D)
    s = p[None, :, :] - e[:, None, :]                        # (Q, K, D)
    n = np.array(prob.dims)
    last = prob.D - 1
    s_wrapped = s.copy()
    for a in range(prob.D):
        if prob.walls and a == last:
            continue
        s_wrapped[..., a] = np.mod(s[..., a], n[a])
    idx = np.full(s.shape[:2], -3, dtype=np.int64)
    col = prob.column(s_wrapped)
    if prob.walls:
        lo = s[..., last] < 0
        hi = s[..., last] >= n[last]
        inside = ~(lo | hi)
        clipped = s_wrapped.copy()
        clipped[..., last] = np.clip(clipped[..., last], 0, n[last] - 1)
        idx = np.where(inside, prob.flat(clipped), idx)
        idx = np.where(lo, -1, idx)
        idx = np.where(hi, -2, idx)
    else:
        idx = prob.flat(s_wrapped)
    return idx, col


def wall_density(f, prob, side, E=None):
    """rho_W per wall-parallel column (Sec. 3.2): the populations that cross
    the wall in the coming step, counted once per layer crossed, divided by the
    matching flux of S(T_W, u_W) (E; by default the static wall's) re-emitted
    into the gas."""
    e_n = prob.vs.e[:, -1]
    nW = prob.dims[-1]
    cols = np.arange(prob.ncols)
    numer = np.zeros(prob.ncols)
    if side == "lo":
        E = prob.E_lo if E is None else E
        outgoing = np.nonzero(e_n < 0)[0]
        for a in outgoing:
            for k in range(min(-e_n[a], nW)):
                numer += f[a, cols + k * prob.ncols]
        denom = sum(min(e_n[a], nW) * E[a] for a in np.nonzero(e_n > 0)[0])
    else:
        E = prob.E_hi if E is None else E
        outgoing = np.nonzero(e_n > 0)[0]
        for a in outgoing:
            for k in range(min(e_n[a], nW)):
                numer += f[a, cols + (nW - 1 - k) * prob.ncols]
        denom = sum(min(-e_n[a], nW) * E[a] for a in np.nonzero(e_n < 0)[0])
    return numer / denom


def gather(f, prob, cells=None, n=0):
    """Streaming: the pre-collision populations fbar_alpha(x) = f_alpha(x -
    e_alpha) of the target cells, with wall ghosts where the source lies beyond
    a wall; f is stored level n (its wall emission is the one of the step from
    n to n + 1). Returns shape (Q, K)."""
    if cells is None:
        cells = np.arange(prob.M)
    idx, col = sources(prob, cells)
    Q = prob.vs.Q
    out = np.empty(idx.shape)
    rows = np.arange(Q)[:, None]
    inside = idx >= 0
    out[inside] = f[np.broadcast_to(rows, idx.shape)[inside], idx[inside]]
    if prob.walls:
        E_lo, E_hi = prob.wall_emission(n)
        rw_lo = wall_density(f, prob, "lo", E_lo)
        rw_hi = wall_density(f, prob, "hi", E_hi)
        lo = idx == -1
        hi = idx == -2
        Elo = np.broadcast_to(E_lo[:, None], idx.shape)
        Ehi = np.broadcast_to(E_hi[:, None], idx.shape)
        out[lo] = prob.wall_lo.gamma * rw_lo[col[lo]] * Elo[lo]
        out[hi] = prob.wall_hi.gamma * rw_hi[col[hi]] * Ehi[hi]
        # specular part: alpha' = mirror(alpha) from the mirrored layer
        nW = prob.dims[-1]
        t = prob.coords[cells][:, -1][None, :]                      # target layer (1, K)
        e_n = prob.vs.e[:, -1][:, None]                            # (Q, 1)
        mir = np.broadcast_to(prob.mirror[:, None], idx.shape)
        for mask, layer, gam in ((lo, e_n - 1 - t, prob.wall_lo.gamma),
                                 (hi, 2 * nW - 1 - (t - e_n), prob.wall_hi.gamma)):
            if gam == 1.0 or not mask.any():
                continue
            src = col + np.broadcast_to(layer, idx.shape) * prob.ncols
            out[mask] += (1.0 - gam) * f[mir[mask], src[mask]]
    return out


@dataclass
class PhysicalState:
    rho: np.ndarray
    u: np.ndarray
    T: np.ndarray
    sigma: np.ndarray
    lam: np.ndarray
    tau: np.ndarray
    omega: np.ndarray
    phi: np.ndarray
    xh: np.ndarray
    a_es: list
    a_f: list
    M2: np.ndarray
    M3: np.ndarray
    f_es: np.ndarray


def _sym3(a, v):
    """a_ij v_k + a_ik v_j + a_jk v_i for a symmetric a (M,D,D), v (M,D)."""
    return (np.einsum("mij,mk->mijk", a, v) + np.einsum("mik,mj->mijk", a, v)
            + np.einsum("mjk,mi->mijk", a, v))


def physical_state(fbar, prob):
    """Moments of the physical distribution f at the current time level,
    recovered from the raw moments of fbar (eq. mac, Sec. 2.2).

    Inverting fbar = f + xh (f - f_ES) - hs F moment by moment, with
    hs = dt/2, xh = dt/(2 tau) for the trapezoidal rule and hs = xh = 0 for
    Euler (where fbar = f):
      * rho: sum F = 0 and the collision conserves mass, so rho = sum fbar;
      * rho u = j + hs rho g (sum F c = rho g; collision conserves momentum);
      * D rho T = tr Mbar2 + 2 hs rho g.u - rho u^2 (energy is conserved by
        the collision, sum F c^2 = 2 rho g.u);
      * the traceless second moment relaxes at rate 1/(Pr tau) because
        f_ES carries b sigma: sigma = traceless(Mbar2 + hs rho (g u + u g)
        - rho u u) / (1 + xh/Pr);
      * the third moment: M3 = [Mbar3 + xh sum f_ES ccc + hs sum F ccc]/(1+xh),
        where only the n <= 3 force terms have a third moment on a set exact
        to degree >= N + 3.
    """
    vs, D, N = prob.vs, prob.D, prob.N
    c, w = vs.c, vs.w
    g = prob.gvec
    rho, j, M2bar, M3bar = model.raw_moments(fbar, c, 3)
    d = np.eye(D)[None]
    u = (j + prob.hs * rho[:, None] * g[None, :]) / rho[:, None]
    uu = np.einsum("mi,mj->mij", u, u)
    trM2bar = np.trace(M2bar, axis1=1, axis2=2)
    gu = u @ g
    T = (trM2bar + 2.0 * prob.hs * rho * gu - rho * np.sum(u * u, axis=1)) / (D * rho)
    tau = model.relaxation_time(prob.Kn, prob.Pr, prob.varpi, rho, T)
    x = prob.dt / tau
    xh = prob.hs / tau
    guug = np.einsum("i,mj->mij", g, u) + np.einsum("mi,j->mij", u, g)
    S = M2bar + prob.hs * rho[:, None, None] * guug - rho[:, None, None] * uu
    trS = np.trace(S, axis1=1, axis2=2)
    sigma = (S - (trS / D)[:, None, None] * d) / (1.0 + xh / prob.Pr)[:, None, None]
    lam = model.es_tensor(T, sigma, rho, prob.b)
    a_es = model.es_coefficients(rho, u, lam, N)
    M2 = rho[:, None, None] * (uu + T[:, None, None] * d) + sigma
    a_f = [rho, rho[:, None] * u, M2 - rho[:, None, None] * d]
    f_es = model.hermite_projection(a_es, c, w)
    M3_es = model.raw_moments(f_es, c, 3)[3]
    if np.any(g != 0.0):
        F3 = model.force_term(g, a_f[:3], c, w, 3)
        M3_F = model.raw_moments(F3, c, 3)[3]
    else:
        M3_F = 0.0
    M3 = (M3bar + xh[:, None, None, None] * M3_es + prob.hs * M3_F) / (1.0 + xh)[:, None, None, None]
    if N >= 4:
        rho_u = rho[:, None] * u
        a3 = M3 - (np.einsum("mi,jk->mijk", rho_u, d[0]) + np.einsum("mj,ik->mijk", rho_u, d[0])
                   + np.einsum("mk,ij->mijk", rho_u, d[0]))
        a_f.append(a3)
    omega = x / (1.0 + xh)
    phi = 1.0 - omega * (prob.hs / prob.dt)
    return PhysicalState(rho, u, T, sigma, lam, tau, omega, phi, xh, a_es, a_f, M2, M3, f_es)


def equilibrium_and_force(st, prob):
    """f_ES^N (eq. approxfeq) and F (Sec. 2.2) at the quadrature nodes."""
    vs = prob.vs
    f_es = st.f_es
    if np.any(prob.gvec != 0.0):
        F = model.force_term(prob.gvec, st.a_f, vs.c, vs.w, prob.N)
    else:
        F = np.zeros_like(f_es)
    return f_es, F


def collide(fbar, prob):
    """fbar* = fbar - omega (fbar - f_ES) + phi dt F (discrete eq. lbgk)."""
    st = physical_state(fbar, prob)
    f_es, F = equilibrium_and_force(st, prob)
    return fbar - st.omega[None, :] * (fbar - f_es) + st.phi[None, :] * prob.dt * F


def step(f, prob, n=0):
    """One time step from stored level n: stream (with walls) then collide,
    for every cell."""
    return collide(gather(f, prob, n=n), prob)


def step_cells(f, prob, cells, n=0):
    """One time step evaluated only at the given target cells (for sampled
    comparisons on large grids); returns (Q, K)."""
    return collide(gather(f, prob, cells, n=n), prob)


def run(f, prob, nsteps, n0=0):
    """nsteps steps from stored level n0."""
    for k in range(nsteps):
        f = step(f, prob, n0 + k)
    return f


def physical_distribution(fbar, prob):
    """Recover f = (fbar + xh f_ES + hs F)/(1 + xh) and its physical state."""
    st = physical_state(fbar, prob)
    f_es, F = equilibrium_and_force(st, prob)
    f = (fbar + st.xh[None, :] * f_es + prob.hs * F) / (1.0 + st.xh)[None, :]
    return f, st


def macroscopic(f_state, prob, cells=None, n=0):
    """rho, u, T, sigma, q (eq. mac) of the distribution at stored level n:
    stream, recover the physical f, take its moments."""
    fbar = gather(f_state, prob, cells, n=n)
    f, _ = physical_distribution(fbar, prob)
    return model.macroscopic(f, prob.vs.c)


def equilibrium_state(prob, rho, u, T, noise=None, amplitude=0.0):
    """Initial stored populations f_alpha = rho S_alpha(T, u) (eq. feq0 at the
    bulk order N) times (1 + amplitude * noise_alpha) per cell."""
    f = model.truncated_maxwellian(np.asarray(rho, float), np.asarray(u, float),
                                   np.asarray(T, float), prob.vs.c, prob.vs.w, prob.N)
    if noise is not None:
        f = f * (1.0 + amplitude * noise)
    return f


def from_deviation(h, prob):
    """Storage format of the library: h_alpha = f_alpha / w_alpha - 1."""
    return prob.vs.w[:, None] * (1.0 + h)


def to_deviation(f, prob):
    return f / prob.vs.w[:, None] - 1.0


def reductions(f_state, prob, u_prev=None, n=0):
    """Global FP64 sums of the current level: mass sum rho, energy
    sum 1/2 sum_alpha f c^2, momentum sum rho u, the mass flow rate through a
    plane normal to x averaged over the nx planes, dx^(D-1)/nx sum rho u_x,
    and the relative change ||u - u_prev||_2 / ||u||_2 (0 when no previous
    field is given)."""
    fbar = gather(f_state, prob, n=n)
    f, st = physical_distribution(fbar, prob)
    c = prob.vs.c
    mass = st.rho.sum()
    energy = 0.5 * np.sum(f * np.sum(c * c, axis=1)[:, None])
    mom = (st.rho[:, None] * st.u).sum(axis=0)
    mdot = prob.dx ** (prob.D - 1) / prob.dims[0] * np.sum(st.rho * st.u[:, 0])
    if u_prev is None:
        resid = 0.0
    else:
        resid = np.sqrt(np.sum((st.u - u_prev) ** 2)) / np.sqrt(np.sum(st.u ** 2))
    return dict(mass=mass, energy=energy, mom=mom, mdot=mdot, residual=resid, u=st.u)
