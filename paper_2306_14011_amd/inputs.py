"""Seeded synthetic inputs shared by the GPU path, the oracle tests and the bench.

This module only builds initial states and workload descriptions from a seed.
It holds none of the finite-volume arithmetic (no reconstruction, flux,
residual, time step or reduction): both the HIP path and the CPU oracle take
its arrays as plain inputs.

Arrays are interior-only, float64, shape ``(nvar, nz, ny, nx)`` with
``nvar = ndim + 2`` conserved variables ``(rho, rho*u, rho*v[, rho*w], E)``,
the conserved vector of the governing equations (Sec. "The CFD Code Base",
Eq. QF). For 2D, ``nz == 1``.

The paper times a 2D supersonic inlet on a 3328x1024 curvilinear grid
(Sec. "A Test Case"); that grid and its solution are not available, so the
flows below (isentropic vortex, Gaussian density bumps, rotated Sod tube,
a batch of uneven vortex grids) stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4


@dataclass
class GridSpec:
    """Uniform Cartesian grid: ``n`` cells per axis on the box ``[lo, hi]``.

    ``bc[d] = (lo_kind, hi_kind)`` with 0 = periodic, 1 = transmissive.
    """

    ndim: int
    n: tuple
    lo: tuple
    hi: tuple
    bc: tuple
    gamma: float = GAMMA
    cfl: float = 0.5
    limiter: bool = True   # False: unlimited MUSCL (Psi = 1)
    kappa: float = -1.0    # MUSCL kappa of the unlimited scheme: -1, 0, 1/3, 1/2 or 1
    bc_state: tuple = None  # (3, 2, nvar) conserved ghost state of inflow faces (kind 3)
    mu: float = 0.0         # dynamic viscosity: 0 for the Euler equations, > 0 adds the viscous flux
    prandtl: float = 0.72   # Prandtl number of the heat flux
    nodes: object = None    # 2D curvilinear grid: node coordinates, shape (2, ny + 1, nx + 1); None: the box

    @property
    def nvar(self) -> int:
        return self.ndim + 2

    @property
    def dx(self) -> tuple:
        return tuple((self.hi[d] - self.lo[d]) / self.n[d] for d in range(3))

    @property
    def shape(self) -> tuple:
        nx, ny, nz = self.n
        return (self.nvar, nz, ny, nx)

    @property
    def ncells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def centres(self):
        """Cell-centre coordinates, each of shape (nz, ny, nx)."""
        xs = [self.lo[d] + (np.arange(self.n[d]) + 0.5) * self.dx[d] for d in range(3)]
        z, y, x = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
        return x, y, z


def grid2d(nx, ny, lo=(0.0, 0.0), hi=(10.0, 10.0), bc=((0, 0), (0, 0)), cfl=0.5, gamma=GAMMA):
    return GridSpec(2, (int(nx), int(ny), 1), (lo[0], lo[1], 0.0), (hi[0], hi[1], 1.0),
                    (tuple(bc[0]), tuple(bc[1]), (0, 0)), gamma, cfl)


def grid3d(nx, ny, nz, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
           bc=((1, 1), (0, 0), (0, 0)), cfl=0.5, gamma=GAMMA):
    return GridSpec(3, (int(nx), int(ny), int(nz)), tuple(lo), tuple(hi),
                    tuple(tuple(b) for b in bc), gamma, cfl)


def primitive_to_conserved(g: GridSpec, rho, vel, p):
    """Pack density, velocity components and pressure into ``(nvar, nz, ny, nx)``.

    Total energy of a calorically perfect gas, E = p/(gamma-1) + rho|u|^2/2.
    """
    U = np.empty(g.shape, dtype=np.float64)
    U[0] = rho
    ke = np.zeros_like(rho)
    for d in range(g.ndim):
        U[1 + d] = rho * vel[d]
        ke = ke + vel[d] * vel[d]
    U[g.ndim + 1] = p / (g.gamma - 1.0) + 0.5 * rho * ke
    return U


# ---------------------------------------------------------------------------
# Isentropic vortex (Shu / Yee form) on a freestream of Mach 0.5.

def freestream_velocity(gamma=GAMMA, mach=0.5):
    """Diagonal freestream with |V| = mach * sqrt(gamma) (rho = p = 1)."""
    s = mach * math.sqrt(gamma) / math.sqrt(2.0)
    return (s, s)


def vortex_centre(seed: int, jitter=0.5, base=(5.0, 5.0)):
    rng = np.random.default_rng(seed)
    off = rng.uniform(-jitter, jitter, size=2)
    return (base[0] + off[0], base[1] + off[1])


def vortex_state(g: GridSpec, centre, beta=5.0, t=0.0, mach=0.5, points=None):
    """Isentropic vortex point values at the cell centres at time ``t`` (or
    at ``points`` = (x, y), arrays of shape (ny, nx), e.g. the node centroids
    of a curvilinear grid).

    At ``t > 0`` the vortex has been carried by the freestream, so this is also
    the exact solution of the Euler equations on the periodic box.
    """
    gam = g.gamma
    if points is None:
        x, y, _ = g.centres()
        x, y = x[0], y[0]
    else:
        x, y = points
    ux, uy = freestream_velocity(gam, mach)
    Lx = g.hi[0] - g.lo[0]
    Ly = g.hi[1] - g.lo[1]
    xc = g.lo[0] + np.mod(centre[0] + ux * t - g.lo[0], Lx)
    yc = g.lo[1] + np.mod(centre[1] + uy * t - g.lo[1], Ly)
    dxv = x - xc
    dyv = y - yc
    dxv = dxv - Lx * np.round(dxv / Lx)      # minimum-image distance
    dyv = dyv - Ly * np.round(dyv / Ly)
    r2 = dxv * dxv + dyv * dyv
    f = np.exp(0.5 * (1.0 - r2))
    u = ux - beta / (2.0 * math.pi) * f * dyv
    v = uy + beta / (2.0 * math.pi) * f * dxv
    T = 1.0 - (gam - 1.0) * beta * beta / (8.0 * gam * math.pi ** 2) * f * f
    rho = T ** (1.0 / (gam - 1.0))
    p = rho * T
    return primitive_to_conserved(g, rho[None], (u[None], v[None]), p[None])


def gaussian_bumps(g: GridSpec, U, seed: int, count=32, sigma=0.25, amp=1e-2):
    """Add ``count`` seeded Gaussian density bumps (amplitude amp*rho_inf).

    Velocity and pressure are kept, so E is rebuilt from the new density.
    """
    rng = np.random.default_rng(seed + 7919)
    x, y, _ = g.centres()
    x, y = x[0], y[0]
    Lx = g.hi[0] - g.lo[0]
    Ly = g.hi[1] - g.lo[1]
    rho = U[0, 0].copy()
    u = U[1, 0] / rho
    v = U[2, 0] / rho
    p = (g.gamma - 1.0) * (U[3, 0] - 0.5 * rho * (u * u + v * v))
    cx = rng.uniform(g.lo[0], g.hi[0], size=count)
    cy = rng.uniform(g.lo[1], g.hi[1], size=count)
    for k in range(count):
        ddx = x - cx[k]
        ddy = y - cy[k]
        ddx = ddx - Lx * np.round(ddx / Lx)
        ddy = ddy - Ly * np.round(ddy / Ly)
        rho = rho + amp * np.exp(-(ddx * ddx + ddy * ddy) / (2.0 * sigma * sigma))
    return primitive_to_conserved(g, rho[None], (u[None], v[None]), p[None])


# ---------------------------------------------------------------------------
# Sod tube, optionally tilted.

SOD_LEFT = (1.0, 0.0, 1.0)      # rho, u, p
SOD_RIGHT = (0.125, 0.0, 0.1)


def sod_state(g: GridSpec, normal, origin):
    """Sod states on either side of the plane (x - origin).normal = 0."""
    x, y, z = g.centres()
    s = (x - origin[0]) * normal[0] + (y - origin[1]) * normal[1]
    if g.ndim == 3:
        s = s + (z - origin[2]) * normal[2]
    left = s < 0.0
    rho = np.where(left, SOD_LEFT[0], SOD_RIGHT[0])
    p = np.where(left, SOD_LEFT[2], SOD_RIGHT[2])
    zero = np.zeros_like(rho)
    return primitive_to_conserved(g, rho, tuple(zero for _ in range(g.ndim)), p)


def sod_rotated_normal(seed: int):
    """Seeded tilt: theta ~ U(0, pi/6) from the x axis, phi ~ U(0, 2 pi)."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, math.pi / 6.0)
    ph = rng.uniform(0.0, 2.0 * math.pi)
    return (math.cos(th), math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph))


def sod_axis_state(g: GridSpec, axis: int, x0=0.5):
    """Untilted Sod tube along ``axis`` with the jump at lo + x0*(hi-lo)."""
    normal = [0.0, 0.0, 0.0]
    normal[axis] = 1.0
    origin = [0.0, 0.0, 0.0]
    origin[axis] = g.lo[axis] + x0 * (g.hi[axis] - g.lo[axis])
    return sod_state(g, normal, origin)


# ---------------------------------------------------------------------------
# Workload recipes (sizes of the measured configurations).

def vortex_case(n=64, seed=0, beta=5.0):
    """Isentropic vortex, strength beta, Mach 0.5 diagonal, periodic [0,10]^2."""
    g = grid2d(n, n)
    return g, vortex_state(g, vortex_centre(seed), beta)


def vortex_bumps_case(n=2048, seed=0, beta=5.0):
    """Vortex plus 32 seeded Gaussian density bumps, periodic [0,10]^2."""
    g, U = vortex_case(n, seed, beta)
    return g, gaussian_bumps(g, U, seed)


def tiled_case(g, U, k):
    """k x k copies of the periodic 2D state U of grid g on a box k times as
    long in x and y: the same cell size and flow, k^2 times the cells."""
    if g.ndim != 2 or any(tuple(b) != (0, 0) for b in g.bc[:2]):
        raise ValueError("tiled_case needs a periodic 2D grid")
    hi = (g.lo[0] + k * (g.hi[0] - g.lo[0]), g.lo[1] + k * (g.hi[1] - g.lo[1]))
    gk = grid2d(g.n[0] * k, g.n[1] * k, lo=(g.lo[0], g.lo[1]), hi=hi, bc=g.bc[:2], cfl=g.cfl, gamma=g.gamma)
    return gk, np.ascontiguousarray(np.tile(U, (1, 1, k, k)))


def sod3d_case(n=256, seed=0):
    """Rotated Sod tube on [0,1]^3, transmissive x faces, periodic y/z."""
    g = grid3d(n, n, n)
    return g, sod_state(g, sod_rotated_normal(seed), (0.5, 0.5, 0.5))


@dataclass
class BatchSpec:
    grids: list = field(default_factory=list)   # GridSpec per member
    states: list = field(default_factory=list)  # interior states


def batch_case(count=96, seed=0, smin=128, smax=1024, make_states=True):
    """``count`` uneven periodic 2D vortex grids, sides drawn from smin..smax."""
    rng = np.random.default_rng(seed)
    out = BatchSpec()
    for _ in range(count):
        nx = int(rng.integers(smin, smax + 1))
        ny = int(rng.integers(smin, smax + 1))
        beta = float(rng.uniform(1.0, 5.0))
        c = rng.uniform(-2.5, 2.5, size=2)
        g = grid2d(nx, ny)
        out.grids.append(g)
        if make_states:
            out.states.append(vortex_state(g, (5.0 + c[0], 5.0 + c[1]), beta))
        else:
            out.states.append((5.0 + c[0], 5.0 + c[1], beta))
    return out


def adjoint_window(n=512, width=64):
    """Centred ``width``^2 cell window [n/2 - width/2, n/2 + width/2)^2."""
    a = n // 2 - width // 2
    return (a, a + width)


def random_directions(shape, count, seed, scales):
    """Seeded N(0,1) directions, scaled per variable and normalised to max-norm 1."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = rng.standard_normal(shape)
        for v in range(shape[0]):
            d[v] *= scales[v]
        d /= np.max(np.abs(d))
        out.append(d)
    return out


def smooth_source(g: GridSpec, seed: int, amp: float = 0.05):
    """Seeded smooth source field (nvar, nz, ny, nx): per variable, amp times a
    sum of three sine modes of random integer wavenumbers and phases over the
    cell centres of the box (periodic in every direction of the box)."""
    rng = np.random.default_rng(seed + 7919)
    nx, ny, nz = (int(v) for v in g.n)
    axes = []
    for d, m in enumerate((nx, ny, nz)):
        c = (np.arange(m) + 0.5) / m
        axes.append(c)
    X = axes[0][None, None, :]
    Y = axes[1][None, :, None]
    Z = axes[2][:, None, None]
    out = np.zeros((g.nvar, nz, ny, nx))
    for v in range(g.nvar):
        for _ in range(3):
            kx, ky = rng.integers(1, 4, 2)
            kz = rng.integers(1, 4) if g.ndim == 3 else 0
            ph = rng.uniform(0.0, 2.0 * math.pi)
            out[v] += np.sin(2.0 * math.pi * (kx * X + ky * Y + kz * Z) + ph)
    return amp * out


# ---------------------------------------------------------------------------
# Random draws of the autotuner's network (passed to both the GPU kernels and
# the oracle): initial parameters and the row order of every epoch.

MLP_LAYERS = ((14, 64), (64, 64), (64, 64), (64, 1))


def mlp_init(seed: int, n_in: int = 14):
    """Flat float64 parameters W1, b1, ..., W4, b4 (W[out][in]) of the network
    with n_in inputs; every layer uniform in +-sqrt(6 / (fan_in + fan_out))
    (Glorot & Bengio 2010)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((n_in, 64),) + MLP_LAYERS[1:]:
        b = math.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-b, b, size=(fo, fi)).ravel())
        parts.append(rng.uniform(-b, b, size=fo))
    return np.concatenate(parts)


def epoch_orders(n: int, epochs: int, seed: int):
    """One random permutation of range(n) per epoch, shape (epochs, n), int32."""
    rng = np.random.default_rng(seed + 104729)
    return np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)


def wavy_nodes(nx, ny, lo=(0.0, 0.0), hi=(10.0, 10.0), amp=0.05, rot=0.0):
    """Node coordinates (2, ny + 1, nx + 1) of a smoothly distorted grid of the
    box: x = xi + amp Lx sin(2 pi (eta - lo_y) / Ly), y = eta + amp Ly sin(2 pi
    (xi - lo_x) / Lx), then rotated by `rot` radians about the origin. The
    distortion is periodic, so the grid wraps like the box (periodic axes
    stay periodic in index space)."""
    Lx, Ly = hi[0] - lo[0], hi[1] - lo[1]
    xi = lo[0] + Lx * np.arange(nx + 1) / nx
    eta = lo[1] + Ly * np.arange(ny + 1) / ny
    E, X = np.meshgrid(eta, xi, indexing="ij")
    x = X + amp * Lx * np.sin(2 * np.pi * (E - lo[1]) / Ly)
    y = E + amp * Ly * np.sin(2 * np.pi * (X - lo[0]) / Lx)
    c, s = math.cos(rot), math.sin(rot)
    return np.stack([c * x - s * y, s * x + c * y])


def node_centroids(nodes):
    """Mean of each quadrilateral cell's four nodes: arrays (ny, nx) of x and y."""
    x, y = nodes
    cx = 0.25 * (x[:-1, :-1] + x[:-1, 1:] + x[1:, :-1] + x[1:, 1:])
    cy = 0.25 * (y[:-1, :-1] + y[:-1, 1:] + y[1:, :-1] + y[1:, 1:])
    return cx, cy
