"""Seeded synthetic initial data for the MEG7 hot path.

This module only builds initial states.  It holds none of the scheme's
arithmetic: it is shared by the CPU oracle tests and the GPU path so both
see the same bits.  Every state is returned as a float64 numpy array
Q[4][ny][nx] = (rho, rho u, rho v, E), x fastest, with
E = p/(gamma-1) + rho (u^2+v^2)/2 (the ideal-gas law of Sec. 1), and a
``Problem`` record holding the domain, boundary types and fluid constants.

Families
  vortex     isentropic vortex of the order-of-accuracy example (strength 5,
             Gaussian profile, free stream rho=u=v=p=1), periodic.
  riemann    four-quadrant Riemann problem in the layout of the paper's 2D
             Riemann example (split at (0.8, 0.8)), states drawn from a seed,
             transmissive boundaries.
  shear      periodic double shear layer, tanh profile +/-0.5, Mach 0.3,
             seeded sinusoidal perturbation on modes 1-8, Re = 1e4, Pr = 0.72.
  taylor_green  inviscid 2D Taylor-Green vortex (the z = 0 plane of the
             paper's Taylor-Green initial state), periodic on [0, 2 pi)^2.
  double_mach   the paper's double Mach reflection (walls, inflow, moving
             top boundary), 1024 x 256.
  viscous_shock_tube  the paper's viscous shock tube (no-slip walls), Re =
             1000, 1280 x 640.
"""
from dataclasses import dataclass, field
import math

import numpy as np

BC_PERIODIC = 0
BC_TRANSMISSIVE = 1
BC_REFLECT = 2      # slip wall: mirror, normal velocity negated
BC_NOSLIP = 3       # adiabatic no-slip wall: mirror, both velocity components negated
BC_INFLOW = 4       # fixed state in the ghost layers
GAMMA = 1.4


@dataclass
class Problem:
    family: str
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    bc_x: int
    bc_y: int
    gamma: float
    mu: float
    Pr: float
    cfl: float
    seed: int = 0
    Q: np.ndarray = field(default=None, repr=False)
    # optional per-side boundaries (left, right, bottom, top), each
    # (kind, state, kind1, state1, split0, split_speed): kind on the part of the
    # side whose tangential cell-centre coordinate is below split0 + split_speed t,
    # kind1 beyond; states are primitive (rho, u, v, p) for BC_INFLOW
    sides: list = None
    riemann: int = 0        # 1: the shock-stable HLLC
    t_final: float = None

    @property
    def dx(self):
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self):
        return (self.y1 - self.y0) / self.ny

    def geometry(self):
        return (self.x0, self.x1, self.y0, self.y1, self.bc_x, self.bc_y)


def cell_centres(nx, ny, x0, x1, y0, y1):
    x = x0 + (np.arange(nx) + 0.5) * (x1 - x0) / nx
    y = y0 + (np.arange(ny) + 0.5) * (y1 - y0) / ny
    return np.meshgrid(x, y, indexing="xy")


def prim_to_state(rho, u, v, p, gamma=GAMMA):
    """Stack primitive fields into the conservative SoA layout."""
    Q = np.empty((4,) + rho.shape, np.float64)
    Q[0] = rho
    Q[1] = rho * u
    Q[2] = rho * v
    Q[3] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return Q


# ---------------------------------------------------------------- vortex ---
def vortex_fields(X, Y, xc, yc, eps=5.0, gamma=GAMMA, period=None):
    """Isentropic vortex (order-of-accuracy example of Sec. 3) centred at
    (xc, yc); with ``period`` = (Lx, Ly) the nearest periodic image is used."""
    dx = X - xc
    dy = Y - yc
    if period is not None:
        Lx, Ly = period
        dx = dx - Lx * np.round(dx / Lx)
        dy = dy - Ly * np.round(dy / Ly)
    r2 = dx * dx + dy * dy
    T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    g = eps / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    u = 1.0 - g * dy
    v = 1.0 + g * dx
    return rho, u, v, p


def vortex(n, L=10.0, t=0.0, cfl=0.5, eps=5.0, ny=None, x0=0.0):
    """Vortex on [x0, x0+L]^2, centre at the box centre advected by (1,1) for
    time t (exact solution of the Euler equations)."""
    ny = n if ny is None else ny
    X, Y = cell_centres(n, ny, x0, x0 + L, x0, x0 + L)
    c = x0 + 0.5 * L
    rho, u, v, p = vortex_fields(X, Y, c + t, c + t, eps=eps, period=(L, L))
    P = Problem("vortex", n, ny, x0, x0 + L, x0, x0 + L, BC_PERIODIC, BC_PERIODIC,
                GAMMA, 0.0, 0.72, cfl)
    P.Q = prim_to_state(rho, u, v, p)
    return P


# --------------------------------------------------------------- riemann ---
def riemann_states(seed):
    """Quadrant states in the order NE, NW, SW, SE; each quadrant draws
    rho~U[0.1,1.5], u~U[-0.8,0.8], v~U[-0.8,0.8], p~U[0.03,1.5] in that order
    from numpy.random.default_rng(seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        u = rng.uniform(-0.8, 0.8)
        v = rng.uniform(-0.8, 0.8)
        p = rng.uniform(0.03, 1.5)
        out.append((rho, u, v, p))
    return out


def paper_riemann_states():
    """The configuration printed for the paper's 2D Riemann example."""
    s = 4.0 / math.sqrt(11.0)
    return [(1.5, 0.0, 0.0, 1.5), (33.0 / 62.0, s, 0.0, 0.3),
            (77.0 / 558.0, s, s, 9.0 / 310.0), (33.0 / 62.0, 0.0, s, 0.3)]


def riemann(n, seed=0, cfl=0.2, ny=None, states=None, split=(0.8, 0.8)):
    ny = n if ny is None else ny
    X, Y = cell_centres(n, ny, 0.0, 1.0, 0.0, 1.0)
    st = riemann_states(seed) if states is None else states
    xs, ys = split
    quad = np.where(X > xs, np.where(Y > ys, 0, 3), np.where(Y > ys, 1, 2))
    arr = np.array(st, np.float64)          # [4 quadrants][rho,u,v,p]
    rho, u, v, p = (arr[quad, k] for k in range(4))
    P = Problem("riemann", n, ny, 0.0, 1.0, 0.0, 1.0, BC_TRANSMISSIVE, BC_TRANSMISSIVE,
                GAMMA, 0.0, 0.72, cfl, seed)
    P.Q = prim_to_state(rho, u, v, p)
    return P


# ----------------------------------------------------------------- shear ---
def shear(n, seed=0, cfl=0.2, ny=None, delta=0.02, mach=0.3, Re=1.0e4, Pr=0.72,
          amp=1.0e-2, modes=8):
    ny = n if ny is None else ny
    X, Y = cell_centres(n, ny, 0.0, 1.0, 0.0, 1.0)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, modes)
    a = a / a.sum()
    phi = rng.uniform(0.0, 2.0 * math.pi, modes)
    u = np.where(Y < 0.5, 0.5 * np.tanh((Y - 0.25) / delta),
                 0.5 * np.tanh((0.75 - Y) / delta))
    env = np.exp(-((Y - 0.25) / 0.05) ** 2) + np.exp(-((Y - 0.75) / 0.05) ** 2)
    v = np.zeros_like(X)
    for k in range(modes):
        v += a[k] * np.sin(2.0 * math.pi * (k + 1) * X + phi[k])
    v = amp * v * env
    rho = np.ones_like(X)
    c = 0.5 / mach
    p = rho * c * c / GAMMA
    mu = 1.0 * 1.0 * 1.0 / Re          # rho * delta U * L / Re
    P = Problem("shear", n, ny, 0.0, 1.0, 0.0, 1.0, BC_PERIODIC, BC_PERIODIC,
                GAMMA, mu, Pr, cfl, seed)
    P.Q = prim_to_state(rho, u, v, p)
    return P


# ------------------------------------------------------------ taylor-green ---
def taylor_green(n, cfl=0.5, ny=None, p0=100.0):
    """Inviscid Taylor-Green vortex in 2D: the z = 0 plane of the initial state
    of the paper's Taylor-Green comparison (rho = 1, u = sin x cos y,
    v = -cos x sin y, p = p0 + (3 (cos 2x + cos 2y) - 2)/16) on [0, 2 pi)^2,
    periodic.  Mach number about 0.085 at p0 = 100."""
    ny = n if ny is None else ny
    L = 2.0 * math.pi
    X, Y = cell_centres(n, ny, 0.0, L, 0.0, L)
    rho = np.ones_like(X)
    u = np.sin(X) * np.cos(Y)
    v = -np.cos(X) * np.sin(Y)
    p = p0 + (3.0 * (np.cos(2.0 * X) + np.cos(2.0 * Y)) - 2.0) / 16.0
    P = Problem("taylor_green", n, ny, 0.0, L, 0.0, L, BC_PERIODIC, BC_PERIODIC,
                GAMMA, 0.0, 0.72, cfl)
    P.Q = prim_to_state(rho, u, v, p)
    return P


# -------------------------------------------------- wall-bounded problems ---
def single_side(kind, state=None):
    return (kind, state, kind, state, math.inf, 0.0)


def double_mach(nx=1024, ny=None, cfl=0.2):
    """Double Mach reflection (Woodward and Colella) as the paper sets it up:
    [0, 4] x [0, 1], a Mach-10 shock at 60 degrees to the wall through
    (1/6, 0); post-shock (8, 8.25 cos 30, -8.25 sin 30, 116.5), pre-shock
    (1.4, 0, 0, 1).  Boundaries: post-shock inflow on the left, transmissive
    on the right, on the bottom the post-shock state for x < 1/6 and a
    reflecting wall beyond, on the top the exact shock motion (post-shock
    state left of 1/6 + (1 + 20 t)/sqrt 3, pre-shock right of it).  The
    shock-stable HLLC, t = 0.2."""
    ny = nx // 4 if ny is None else ny
    X, Y = cell_centres(nx, ny, 0.0, 4.0, 0.0, 1.0)
    post = (8.0, 8.25 * math.cos(math.pi / 6.0), -8.25 * math.sin(math.pi / 6.0), 116.5)
    pre = (1.4, 0.0, 0.0, 1.0)
    behind = X < 1.0 / 6.0 + Y / math.tan(math.pi / 3.0)
    rho, u, v, p = (np.where(behind, a, b) for a, b in zip(post, pre))
    P = Problem("double_mach", nx, ny, 0.0, 4.0, 0.0, 1.0, BC_TRANSMISSIVE, BC_TRANSMISSIVE,
                GAMMA, 0.0, 0.72, cfl)
    P.Q = prim_to_state(rho, u, v, p)
    s3 = math.sqrt(3.0)
    P.sides = [single_side(BC_INFLOW, post), single_side(BC_TRANSMISSIVE),
               (BC_INFLOW, post, BC_REFLECT, None, 1.0 / 6.0, 0.0),
               (BC_INFLOW, post, BC_INFLOW, pre, 1.0 / 6.0 + 1.0 / s3, 20.0 / s3)]
    P.riemann = 1
    P.t_final = 0.2
    return P


def viscous_shock_tube(nx=1280, ny=None, cfl=0.2, Re=1000.0, Pr=0.73):
    """Viscous shock tube (Daru and Tenaud) as the paper sets it up:
    [0, 1] x [0, 0.5], (120, 0, 0, 120/gamma) for x < 0.5 and
    (1.2, 0, 0, 1.2/gamma) beyond, mu = 1/Re with Re = 1000; adiabatic no-slip
    walls left, right and bottom, a symmetry plane (reflecting) on top;
    t = 1."""
    ny = nx // 2 if ny is None else ny
    X, Y = cell_centres(nx, ny, 0.0, 1.0, 0.0, 0.5)
    left = X < 0.5
    rho = np.where(left, 120.0, 1.2)
    p = rho / GAMMA
    z = np.zeros_like(X)
    P = Problem("viscous_shock_tube", nx, ny, 0.0, 1.0, 0.0, 0.5, BC_TRANSMISSIVE,
                BC_TRANSMISSIVE, GAMMA, 1.0 / Re, Pr, cfl)
    P.Q = prim_to_state(rho, z, z, p)
    P.sides = [single_side(BC_NOSLIP), single_side(BC_NOSLIP), single_side(BC_NOSLIP),
               single_side(BC_REFLECT)]
    P.t_final = 1.0
    return P


# ------------------------------------------------------------------ misc ---
def free_stream(n, rho=1.0, u=0.3, v=-0.2, p=0.7, bc=BC_PERIODIC, mu=0.0, ny=None):
    ny = n if ny is None else ny
    shape = (ny, n)
    P = Problem("free", n, ny, 0.0, 1.0, 0.0, 1.0, bc, bc, GAMMA, mu, 0.72, 0.2)
    P.Q = prim_to_state(np.full(shape, rho), np.full(shape, u), np.full(shape, v),
                        np.full(shape, p))
    return P


def make(family, n, seed=0, **kw):
    if family == "vortex":
        return vortex(n, **kw)
    if family == "riemann":
        return riemann(n, seed=seed, **kw)
    if family == "shear":
        return shear(n, seed=seed, **kw)
    if family == "taylor_green":
        return taylor_green(n, **kw)
    if family == "double_mach":
        return double_mach(n, **kw)
    if family == "viscous_shock_tube":
        return viscous_shock_tube(n, **kw)
    raise ValueError(family)


# Four-quadrant draws (seeds) of the batched workload whose corner expansion
# drives the density to zero within 40 steps: the method has no positivity
# limiter and produces NaN there, in the CPU oracle as on the GPU.  The batch
# replaces each by seed + 100000; tests/test_inputs.py re-derives the set.
BATCH_VACUUM_SEEDS = frozenset({10092, 10205})


def batch_spec(nprob=512, seed=0, nmin=64, nmax=768):
    """Sizes and families of the batched workload: side n ~ U{nmin..nmax}
    (square grids), family uniform over {vortex, riemann, shear}, per-problem
    seed 10000 + index (a Riemann seed in BATCH_VACUUM_SEEDS takes
    seed + 100000 instead)."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(nmin, nmax + 1, nprob)
    fams = rng.integers(0, 3, nprob)
    names = ("vortex", "riemann", "shear")
    out = []
    for k, (f, s) in enumerate(zip(fams, sides)):
        sd = 10000 + k
        if names[f] == "riemann" and sd in BATCH_VACUUM_SEEDS:
            sd += 100000
        out.append((names[f], int(s), sd))
    return out


def mlp_init_params(seed, nf=28, nh=32):
    """Initial parameters of the learned detector (28 -> 32 -> 32 -> 1):
    He-uniform weights in the order W1 [32][28], W2 [32][32], w3 [32], all
    float32, and zero biases [65]; drawn from numpy.random.default_rng(seed)."""
    rng = np.random.default_rng(seed)
    w = np.concatenate([rng.uniform(-1, 1, nh * nf) * np.sqrt(6.0 / nf),
                        rng.uniform(-1, 1, nh * nh) * np.sqrt(6.0 / nh),
                        rng.uniform(-1, 1, nh) * np.sqrt(6.0 / nh)]).astype(np.float32)
    return w, np.zeros(nh + nh + 1, np.float32)


def balanced_batches(labels, batch, nbatches, seed):
    """Index arrays for balanced minibatches: half of each batch drawn from the
    cells labelled 1 and half from the cells labelled 0 (with replacement),
    from numpy.random.default_rng(seed); returns int32 [nbatches][batch]."""
    rng = np.random.default_rng(seed)
    pos = np.flatnonzero(labels)
    neg = np.flatnonzero(labels == 0)
    out = np.empty((nbatches, batch), np.int32)
    h = batch // 2
    for k in range(nbatches):
        a = pos[rng.integers(0, len(pos), h)] if len(pos) else neg[rng.integers(0, len(neg), h)]
        b = neg[rng.integers(0, len(neg), batch - h)] if len(neg) else pos[rng.integers(0, len(pos), batch - h)]
        out[k] = rng.permutation(np.concatenate([a, b]))
    return out


def hard_batches(labels, near, batch, nbatches, seed, frac_near=0.25):
    """Index arrays for minibatches with hard negatives: half of each batch
    from the cells labelled 1, `frac_near` of it from the cells labelled 0 that
    lie near a labelled cell (mask `near`), the rest from the other cells
    labelled 0 (each with replacement), from numpy.random.default_rng(seed);
    returns int32 [nbatches][batch]."""
    rng = np.random.default_rng(seed)
    labels = np.asarray(labels)
    pos = np.flatnonzero(labels)
    hard = np.flatnonzero((labels == 0) & near)
    easy = np.flatnonzero((labels == 0) & ~near)
    pools = [p for p in (pos, hard, easy)]
    h = batch // 2
    k = int(batch * frac_near)
    sizes = (h, k, batch - h - k)
    out = np.empty((nbatches, batch), np.int32)
    for b in range(nbatches):
        parts = []
        for pool, size in zip(pools, sizes):
            src = pool if len(pool) else np.flatnonzero(labels == 0)
            parts.append(src[rng.integers(0, len(src), size)])
        out[b] = rng.permutation(np.concatenate(parts))
    return out


# -------------------------------------------------------------------- 3D ---
@dataclass
class Problem3:
    """A 3D Euler problem: Q[5][nz][ny][nx] = (rho, rho u, rho v, rho w, E),
    x fastest, E = p/(gamma-1) + rho (u^2+v^2+w^2)/2."""
    family: str
    nx: int
    ny: int
    nz: int
    lo: tuple
    hi: tuple
    bc: tuple
    gamma: float
    cfl: float
    seed: int = 0
    Q: np.ndarray = field(default=None, repr=False)
    t_final: float = None

    def geometry(self):
        return (self.lo[0], self.hi[0], self.lo[1], self.hi[1], self.lo[2], self.hi[2])


def cell_centres3(n, lo, hi):
    ax = [lo[d] + (np.arange(n[d]) + 0.5) * (hi[d] - lo[d]) / n[d] for d in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


def prim_to_state3(rho, u, v, w, p, gamma=GAMMA):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, rho * w, E]), dtype=np.float64)


def taylor_green3d(n, cfl=0.2, p0=100.0):
    """The paper's inviscid Taylor-Green vortex on [0, 2 pi)^3, periodic:
    rho = 1, u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
    p = p0 + ((cos 2z + 2)(cos 2x + cos 2y) - 2)/16; run to t = 10."""
    L = 2.0 * math.pi
    X, Y, Z = cell_centres3((n, n, n), (0.0, 0.0, 0.0), (L, L, L))
    rho = np.ones_like(X)
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(X)
    p = p0 + ((np.cos(2.0 * Z) + 2.0) * (np.cos(2.0 * X) + np.cos(2.0 * Y)) - 2.0) / 16.0
    P = Problem3("taylor_green3d", n, n, n, (0.0, 0.0, 0.0), (L, L, L),
                 (BC_PERIODIC,) * 3, GAMMA, cfl)
    P.Q = prim_to_state3(rho, u, v, w, p)
    P.t_final = 10.0
    return P


def advected_wave3d(n, amp=0.2):
    """rho = 1 + amp sin(x + y + z), u = v = w = 1, p = 1 on [0, 2 pi)^3,
    periodic: an exact solution translating along (1, 1, 1), so
    dQ/dt = -(d/dx + d/dy + d/dz) Q exactly."""
    L = 2.0 * math.pi
    X, Y, Z = cell_centres3((n, n, n), (0.0, 0.0, 0.0), (L, L, L))
    rho = 1.0 + amp * np.sin(X + Y + Z)
    one = np.ones_like(X)
    P = Problem3("advected_wave3d", n, n, n, (0.0, 0.0, 0.0), (L, L, L),
                 (BC_PERIODIC,) * 3, GAMMA, 0.5)
    P.Q = prim_to_state3(rho, one, one, one, one)
    return P


def riemann3d(n, seed=0, ny=None, nz=None, cfl=0.2, split=(0.6, 0.55, 0.5)):
    """Eight-octant Riemann problem on [0,1]^3, transmissive: octant states
    (bit 0: x > split x, bit 1: y > split y, bit 2: z > split z) draw
    rho~U[0.1,1.5], u, v, w~U[-0.8,0.8], p~U[0.03,1.5] in that order from
    numpy.random.default_rng(seed), octant after octant."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    X, Y, Z = cell_centres3((n, ny, nz), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    rng = np.random.default_rng(seed)
    st = np.array([[rng.uniform(0.1, 1.5), rng.uniform(-0.8, 0.8), rng.uniform(-0.8, 0.8),
                    rng.uniform(-0.8, 0.8), rng.uniform(0.03, 1.5)] for _ in range(8)])
    octant = ((X > split[0]).astype(int) + 2 * (Y > split[1]).astype(int)
              + 4 * (Z > split[2]).astype(int))
    rho, u, v, w, p = (st[octant, k] for k in range(5))
    P = Problem3("riemann3d", n, ny, nz, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                 (BC_TRANSMISSIVE,) * 3, GAMMA, cfl, seed)
    P.Q = prim_to_state3(rho, u, v, w, p)
    return P
