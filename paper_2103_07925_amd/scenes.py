"""Seeded synthetic scene generators.

This module builds the inputs that both the HIP library and the CPU oracle
consume: particle positions on the initial lattice, particle kinds, material
indices, rigid-body membership and the per-scene parameters.  It holds none of
the method's arithmetic (no kernel, no density, no mass, no time step): every
derived quantity is computed separately by each consumer.

Lattice convention (Sec. "Initial particle spacing"): particles sit on a
regular grid of spacing dx at (m + 1/2) dx.  Walls are q = floor(r_c/dx) = 3
layers that continue the lattice outward, so the first wall layer sits dx/2
outside the fluid (Sec. "Boundary and coupling conditions").

Every random draw comes from numpy's PCG64 generator seeded by the caller.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FLUID, WALL, RIGID = 0, 1, 2


@dataclass
class Material:
    """One phase: reference density, reference pressure p0, kinematic
    viscosity, heat capacity, conductivity, body force per unit mass,
    transition temperature, partner phase after a transition (-1: none) and,
    for wall phases, whether the wall temperature is prescribed."""
    rho0: float
    p0: float = 0.0
    nu: float = 0.0
    cp: float = 1.0
    kappa: float = 0.0
    b: tuple = (0.0, 0.0, 0.0)
    T_t: float = 0.0
    switch_to: int = -1
    dirichlet: int = 0


@dataclass
class BodyInit:
    u: tuple = (0.0, 0.0, 0.0)
    w: tuple = (0.0, 0.0, 0.0)
    q: tuple = (1.0, 0.0, 0.0, 0.0)
    fixed: int = 0


@dataclass
class Scene:
    """Plain container of one scene's inputs (host, FP64, original-id order)."""
    name: str
    dim: int
    dx: float
    lo: np.ndarray
    hi: np.ndarray
    cell_edge: float
    x: np.ndarray            # (n, 3)
    u: np.ndarray            # (n, 3)
    T: np.ndarray            # (n,)
    kind: np.ndarray         # (n,) int32
    phase: np.ndarray        # (n,) int32
    body: np.ndarray         # (n,) int32, -1 unless rigid
    moving: np.ndarray       # (n,) int32, 1 for walls following the wall motion
    materials: list
    bodies: list
    dt: float = 0.0          # 0: derive from the stability bounds at t = 0
    max_bodies: int = 0      # capacity for bodies created by solidification
    k_c: float = -1.0        # < 0: default stiffness
    d_c: float = -1.0        # < 0: default damping
    thermal: int = 0
    contact: int = 1
    phase_switch: int = 0
    wall_A: float = 0.0      # moving-wall displacement A (cos(Omega t) - 1) along wall_dir
    wall_Omega: float = 0.0
    wall_dir: tuple = (1.0, 0.0, 0.0)
    heat_src: int = 0
    src_Q: float = 0.0
    src_sigma: float = 1.0
    src_s0: tuple = (0.0, 0.0)
    src_v: tuple = (0.0, 0.0)
    src_ztop: float = 0.0
    src_depth: float = 0.0
    p_b: float = 0.0         # background pressure of the transport-velocity formulation; 0: off
    periodic: tuple = (0, 0, 0)  # periodic axes (y, z only); extent a whole number of cells
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def counts(self) -> dict:
        return {
            "n": self.n,
            "fluid": int(np.sum(self.kind == FLUID)),
            "wall": int(np.sum(self.kind == WALL)),
            "rigid": int(np.sum(self.kind == RIGID)),
            "bodies": len(self.bodies),
        }


# ----------------------------------------------------------------------------
# lattice helpers
# ----------------------------------------------------------------------------

def lattice_sites(dim: int, lo_idx, hi_idx, dx: float) -> np.ndarray:
    """Sites (m + 1/2) dx for integer m in [lo_idx[a], hi_idx[a]) per axis,
    x-fastest order, returned as (n, 3) with z = 0 in 2D."""
    axes = [np.arange(lo_idx[a], hi_idx[a], dtype=np.int64) for a in range(dim)]
    if dim == 2:
        gy, gx = np.meshgrid(axes[1], axes[0], indexing="ij")
        idx = np.stack([gx.ravel(), gy.ravel(), np.zeros(gx.size, np.int64)], axis=1)
    else:
        gz, gy, gx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        idx = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    x = (idx.astype(np.float64) + 0.5) * dx
    if dim == 2:
        x[:, 2] = 0.0
    return x


def box_and_walls(dim: int, nsites, dx: float, layers: int = 3):
    """Interior sites of a box [0, n_a dx] and a closed shell of `layers`
    wall layers around it (edges and corners included)."""
    nsites = list(nsites)
    inner = lattice_sites(dim, [0] * dim, nsites, dx)
    outer = lattice_sites(dim, [-layers] * dim, [n + layers for n in nsites], dx)
    ext = np.array(nsites[:dim], dtype=np.float64) * dx
    inside = np.all((outer[:, :dim] > 0.0) & (outer[:, :dim] < ext), axis=1)
    walls = outer[~inside]
    lo = np.zeros(3)
    hi = np.zeros(3)
    lo[:dim] = -layers * dx
    hi[:dim] = ext + layers * dx
    return inner, walls, lo, hi


def in_ball(x: np.ndarray, centre, radius: float, dim: int) -> np.ndarray:
    c = np.asarray(centre, dtype=np.float64)
    d = x[:, :dim] - c[None, :dim]
    return np.sum(d * d, axis=1) <= radius * radius


def ball_sites(nsites, dx: float, dim: int, centre, radius: float) -> np.ndarray:
    """Indices of the sites of the lattice `lattice_sites(dim, 0, nsites, dx)`
    that are inside the ball (the same test as `in_ball`), found from the
    ball's bounding box of lattice indices rather than by testing every site."""
    c = np.asarray(centre, dtype=np.float64)
    rng_ = []
    for a in range(dim):
        m0 = max(0, int(math.floor((c[a] - radius) / dx - 0.5)) - 1)
        m1 = min(int(nsites[a]), int(math.ceil((c[a] + radius) / dx - 0.5)) + 2)
        rng_.append(np.arange(m0, max(m0, m1), dtype=np.int64))
    if dim == 2:
        gy, gx = np.meshgrid(rng_[1], rng_[0], indexing="ij")
        idx = (gx + int(nsites[0]) * gy).ravel()
        pts = np.stack([(gx.ravel() + 0.5) * dx, (gy.ravel() + 0.5) * dx, np.zeros(gx.size)], axis=1)
    else:
        gz, gy, gx = np.meshgrid(rng_[2], rng_[1], rng_[0], indexing="ij")
        idx = (gx + int(nsites[0]) * (gy + int(nsites[1]) * gz)).ravel()
        pts = np.stack([(gx.ravel() + 0.5) * dx, (gy.ravel() + 0.5) * dx, (gz.ravel() + 0.5) * dx], axis=1)
    return idx[in_ball(pts, c, radius, dim)]


def _assemble(name, dim, dx, lo, hi, groups, materials, bodies, **kw) -> Scene:
    """groups: list of (positions, kind, phase, body, moving, T) tuples."""
    xs, kinds, phases, bids, movs, Ts = [], [], [], [], [], []
    for (pos, kind, phase, body, moving, T) in groups:
        m = pos.shape[0]
        xs.append(pos)
        kinds.append(np.full(m, kind, np.int32))
        phases.append(np.broadcast_to(np.asarray(phase, np.int32), (m,)).copy())
        bids.append(np.broadcast_to(np.asarray(body, np.int32), (m,)).copy())
        movs.append(np.broadcast_to(np.asarray(moving, np.int32), (m,)).copy())
        Ts.append(np.broadcast_to(np.asarray(T, np.float64), (m,)).copy())
    x = np.concatenate(xs).astype(np.float64)
    n = x.shape[0]
    cell_edge = kw.pop("cell_edge", 3.0 * dx)
    return Scene(name=name, dim=dim, dx=dx, lo=lo.astype(np.float64), hi=hi.astype(np.float64),
                 cell_edge=cell_edge, x=x, u=np.zeros((n, 3)), T=np.concatenate(Ts),
                 kind=np.concatenate(kinds), phase=np.concatenate(phases),
                 body=np.concatenate(bids), moving=np.concatenate(movs),
                 materials=materials, bodies=bodies, **kw)


def jitter(x: np.ndarray, mask: np.ndarray, dx: float, rng, dim: int, amp: float = 0.01):
    """Uniform jitter U(-amp dx, +amp dx) per axis of the masked rows."""
    j = rng.uniform(-amp * dx, amp * dx, size=(int(mask.sum()), dim))
    x = x.copy()
    x[np.where(mask)[0][:, None], np.arange(dim)[None, :]] += j
    return x


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

def speed_of_sound_10x(g: float, height: float) -> float:
    """Artificial speed of sound chosen as 10 x the free-fall speed over the
    fluid height, sqrt(2 g H) (the scene parameter, not part of the method)."""
    return 10.0 * math.sqrt(2.0 * g * height)


def config_c1(seed: int = 0, jitter_amp: float = 0.01, with_disc: bool = True,
              n_side: int = 32, dx: float = 0.025) -> Scene:
    """2D box, 32 x 32 fluid sites, dx = 0.025, 3 wall layers, one rigid disc
    of radius 0.1 (4 dx) centred on the lattice vertex (0.4, 0.6), density
    1250 (the density ratio of the falling-disc example), g = 9.81, rho0 = 1000,
    nu = 1e-3, c = 10 sqrt(2 g H)."""
    dim = 2
    rng = np.random.default_rng(seed)
    inner, walls, lo, hi = box_and_walls(dim, (n_side, n_side), dx)
    H = n_side * dx
    g = 9.81
    c = speed_of_sound_10x(g, H)
    mats = [
        Material(rho0=1000.0, p0=1000.0 * c * c, nu=1e-3, b=(0.0, -g, 0.0)),   # fluid
        Material(rho0=1000.0),                                                  # wall
        Material(rho0=1250.0, b=(0.0, -g, 0.0)),                                # disc
    ]
    groups = []
    bodies = []
    if with_disc:
        disc = in_ball(inner, (0.4, 0.6, 0.0), 0.1, dim)
        fluid = inner[~disc]
        groups.append((inner[disc], RIGID, 2, 0, 0, 0.0))
        bodies.append(BodyInit())
    else:
        fluid = inner
    groups.insert(0, (fluid, FLUID, 0, -1, 0, 0.0))
    groups.append((walls, WALL, 1, -1, 0, 0.0))
    sc = _assemble("c1", dim, dx, lo, hi, groups, mats, bodies, max_bodies=len(bodies))
    if jitter_amp > 0:
        sc.x = jitter(sc.x, sc.kind == FLUID, dx, rng, dim, jitter_amp)
    sc.meta.update(seed=seed, c=c, steps=1000)
    return sc


def config_c2(seed: int = 0, n_side: int = 100, dx: float = 0.01, n_per_axis: int = 4,
              spacing_sites: int = 25, r_range=(4.0, 8.0), rho_range=(1.2, 3.0)) -> Scene:
    """3D closed box filled with fluid, n_side^3 interior sites, 3 wall layers,
    n_per_axis^3 rigid spheres on a regular grid of site-centred centres
    (12.5 dx + spacing_sites dx k), radii U(r_range) dx, densities
    U(rho_range) x 1000, all at rest, g on every phase, c = 10 sqrt(2 g H)."""
    dim = 3
    rng = np.random.default_rng(seed)
    inner, walls, lo, hi = box_and_walls(dim, (n_side,) * 3, dx)
    H = n_side * dx
    g = 9.81
    c = speed_of_sound_10x(g, H)
    gvec = (0.0, 0.0, -g)
    mats = [Material(rho0=1000.0, p0=1000.0 * c * c, nu=1e-3, b=gvec), Material(rho0=1000.0)]
    kind_of = np.full(inner.shape[0], FLUID, np.int32)
    phase_of = np.zeros(inner.shape[0], np.int32)
    body_of = np.full(inner.shape[0], -1, np.int32)
    bodies = []
    first = (spacing_sites // 2)
    k = 0
    for iz in range(n_per_axis):
        for iy in range(n_per_axis):
            for ix in range(n_per_axis):
                cidx = np.array([first + spacing_sites * ix, first + spacing_sites * iy,
                                 first + spacing_sites * iz], dtype=np.float64)
                centre = (cidx + 0.5) * dx
                R = rng.uniform(*r_range) * dx
                rho_s = rng.uniform(*rho_range) * 1000.0
                mats.append(Material(rho0=rho_s, b=gvec))
                sel = in_ball(inner, centre, R, dim) & (kind_of == FLUID)
                kind_of[sel] = RIGID
                phase_of[sel] = len(mats) - 1
                body_of[sel] = k
                bodies.append(BodyInit())
                k += 1
    groups = [
        (inner[kind_of == FLUID], FLUID, 0, -1, 0, 0.0),
        (inner[kind_of == RIGID], RIGID, phase_of[kind_of == RIGID], body_of[kind_of == RIGID], 0, 0.0),
        (walls, WALL, 1, -1, 0, 0.0),
    ]
    sc = _assemble("c2", dim, dx, lo, hi, groups, mats, bodies, max_bodies=len(bodies))
    sc.x = jitter(sc.x, sc.kind == FLUID, dx, rng, dim)
    sc.meta.update(seed=seed, c=c, steps=500)
    return sc


def lognormal_radii(rng, n: int, median: float, sigma: float) -> np.ndarray:
    return median * np.exp(sigma * rng.standard_normal(n))


def config_c3(seed: int = 0, nsites=(200, 200, 100), dx: float = 0.1, n_grains: int = 2000,
              median_r: float = 4.3, sigma_r: float = 0.3, dim: int = 3,
              rho_gas: float = 1e-3, p0: float = 100.0) -> Scene:
    """Two-phase liquid/gas box with a temperature field and heat conduction:
    rigid grains (solid metal, rho = 1, cp = 1, kappa = 10) with log-normal
    radii placed by random sequential addition (largest first, gap dx, at
    most 200 tries per grain on average) in the lower 75 % of the box,
    the rest gas (cp = 0.01, kappa = 0.1, density ratio 1000, viscosity ratio
    100 against the liquid metal phase).  Transition temperature 50; grains
    start at 25, gas at 50; a Gaussian surface heat source moves along x.
    Liquid metal (phase 1) below T_t solidifies into solid (phase 0); solid
    above T_t melts into liquid.  Walls keep a prescribed temperature 50."""
    rng = np.random.default_rng(seed)
    inner, walls, lo, hi = box_and_walls(dim, nsites[:dim], dx)
    g = 1.0
    gvec = (0.0, -g, 0.0) if dim == 2 else (0.0, 0.0, -g)
    mats = [
        Material(rho0=1.0, cp=1.0, kappa=10.0, b=gvec, T_t=50.0, switch_to=1),            # 0 solid metal
        Material(rho0=1.0, p0=p0, nu=1.0, cp=1.0, kappa=10.0, b=gvec, T_t=50.0, switch_to=0),  # 1 liquid metal
        Material(rho0=rho_gas, p0=p0, nu=10.0, cp=0.01, kappa=0.1, b=gvec),                # 2 gas
        Material(rho0=1.0, kappa=0.1, dirichlet=1),                                       # 3 wall
    ]
    ext = np.array(nsites[:dim], dtype=np.float64) * dx
    kind_of = np.full(inner.shape[0], FLUID, np.int32)
    phase_of = np.full(inner.shape[0], 2, np.int32)
    body_of = np.full(inner.shape[0], -1, np.int32)
    # largest first: random sequential addition then packs closer to the
    # intended solid fraction before it jams
    radii = np.sort(lognormal_radii(rng, n_grains, median_r * dx, sigma_r))[::-1]
    centres = []
    bodies = []
    upper = 0.75 * ext[dim - 1]
    tries = 0
    placed = np.zeros((n_grains, dim))
    placed_r = np.zeros(n_grains)
    for R in radii:
        while True:
            tries += 1
            if tries > 200 * n_grains:
                break
            cpos = np.zeros(3)
            for a in range(dim):
                top = upper if a == dim - 1 else ext[a]
                cpos[a] = rng.uniform(R + 2 * dx, top - R - 2 * dx) if top - R - 2 * dx > R + 2 * dx else 0.5 * top
            k = len(centres)
            d2 = np.sum((placed[:k] - cpos[:dim]) ** 2, axis=1)
            if not np.any(d2 < (placed_r[:k] + R + dx) ** 2):
                placed[k] = cpos[:dim]
                placed_r[k] = R
                centres.append((cpos, R))
                break
    for k, (cpos, R) in enumerate(centres):
        idx = ball_sites(nsites, dx, dim, cpos, R)
        sel = idx[kind_of[idx] == FLUID]
        if sel.size == 0:
            continue
        kind_of[sel] = RIGID
        phase_of[sel] = 0
        body_of[sel] = len(bodies)
        bodies.append(BodyInit())
    T_in = np.where(kind_of == RIGID, 25.0, 50.0)
    groups = [
        (inner[kind_of == FLUID], FLUID, phase_of[kind_of == FLUID], -1, 0, T_in[kind_of == FLUID]),
        (inner[kind_of == RIGID], RIGID, 0, body_of[kind_of == RIGID], 0, T_in[kind_of == RIGID]),
        (walls, WALL, 3, -1, 0, 50.0),
    ]
    ztop = float(ext[dim - 1])
    sc = _assemble("c3", dim, dx, lo, hi, groups, mats, bodies,
                   max_bodies=len(bodies) + max(64, len(bodies)),
                   thermal=1, phase_switch=1, heat_src=1,
                   src_Q=2.0e3 * dx ** (dim - 1), src_sigma=10.0 * dx,
                   src_s0=(0.1 * ext[0], 0.5 * ext[1] if dim == 3 else 0.0),
                   src_v=(0.5 * ext[0], 0.0), src_ztop=ztop, src_depth=3.0 * dx)
    sc.x = jitter(sc.x, sc.kind == FLUID, dx, rng, dim)
    sc.meta.update(seed=seed, steps=500)
    return sc


def config_c4(seed: int = 0, nsites=(400, 200, 100), dx: float = 0.1, n_frag: int = 500,
              r_range=(3.5, 10.5), dim: int = 3, c_factor: float = 10.0) -> Scene:
    """Container with fluid and irregular rigid fragments (unions of 2-6
    overlapping spheres) driven by a moving wall plate normal to x with a
    central square opening (50 % x 50 %), displacement A (cos(pi t / T_p) - 1)
    with A = 0.725 L_x / 2; velocity amplitude 0.1 c; contact on."""
    rng = np.random.default_rng(seed)
    inner, walls, lo, hi = box_and_walls(dim, nsites[:dim], dx)
    ext = np.array(nsites[:dim], dtype=np.float64) * dx
    Tp = 1.0
    A = 0.725 * ext[0] / 2.0
    u_wall = A * math.pi / Tp
    c = c_factor * u_wall
    rho0 = 1.0
    mats = [Material(rho0=rho0, p0=rho0 * c * c, nu=0.01 * u_wall * dx, b=(0.0, 0.0, 0.0)),
            Material(rho0=rho0), Material(rho0=rho0)]
    kind_of = np.full(inner.shape[0], FLUID, np.int32)
    phase_of = np.zeros(inner.shape[0], np.int32)
    body_of = np.full(inner.shape[0], -1, np.int32)
    # plate: 3 layers of moving wall sites at mid-x, with a central opening
    xm = 0.5 * ext[0]
    px = inner[:, 0]
    plate = np.abs(px - xm) < 1.5 * dx
    if dim == 3:
        opening = (np.abs(inner[:, 1] - 0.5 * ext[1]) < 0.25 * ext[1]) & (np.abs(inner[:, 2] - 0.5 * ext[2]) < 0.25 * ext[2])
    else:
        opening = np.abs(inner[:, 1] - 0.5 * ext[1]) < 0.25 * ext[1]
    plate &= ~opening
    kind_of[plate] = WALL
    phase_of[plate] = 1
    bodies = []
    for k in range(n_frag):
        nsph = int(rng.integers(2, 7))
        base = np.array([rng.uniform(0.05, 0.95) * ext[a] for a in range(dim)] + [0.0] * (3 - dim))
        parts = []
        r0 = rng.uniform(*r_range) * dx
        for s in range(nsph):
            R = r0 if s == 0 else rng.uniform(*r_range) * dx
            off = rng.uniform(-r0, r0, size=3)
            if dim == 2:
                off[2] = 0.0
            cc = base + (off if s > 0 else 0.0)
            parts.append(ball_sites(nsites, dx, dim, cc, R))
        sel = np.unique(np.concatenate(parts))
        sel = sel[kind_of[sel] == FLUID]
        # stay clear of the plate and the walls
        sel = sel[np.abs(px[sel] - xm) > 4.0 * dx]
        if sel.size < 4:
            continue
        kind_of[sel] = RIGID
        phase_of[sel] = 2
        body_of[sel] = len(bodies)
        bodies.append(BodyInit())
    groups = [
        (inner[kind_of == FLUID], FLUID, 0, -1, 0, 0.0),
        (inner[kind_of == RIGID], RIGID, 2, body_of[kind_of == RIGID], 0, 0.0),
        (walls, WALL, 1, -1, 0, 0.0),
        (inner[(kind_of == WALL)], WALL, 1, -1, 1, 0.0),
    ]
    sc = _assemble("c4", dim, dx, lo, hi, groups, mats, bodies, max_bodies=len(bodies),
                   wall_A=A, wall_Omega=math.pi / Tp, wall_dir=(1.0, 0.0, 0.0))
    sc.x = jitter(sc.x, sc.kind == FLUID, dx, rng, dim)
    sc.meta.update(seed=seed, c=c, steps=500)
    return sc


def config_gastric(seed: int = 0, dx: float = 0.1, size=(40.0, 16.0), n_bolus: int = 60,
                   d_range=(1.6, 2.8), c: float = 1.0e3, C_t: float = 0.8, pb_factor: float = 5.0,
                   opening: float = 0.5, amplitude: float = 14.5, period: float = 2.0) -> Scene:
    """2D box (size[0] x size[1], 3 wall layers) with a moving constriction
    and rigid food boluses dissolving by a concentration, shaped like the
    gastric example (Sec. "Gastric disintegration of food boluses"):
    boluses (rigid discs of diameters U(d_range), density 1, D = 0.25,
    C = 0, dissolving into chyme above C_t) placed by random sequential
    addition; gastric juice (fluid, density 1, nu = 100, D = 1, C held at 1);
    chyme (fluid, nu = 200, D = 0.25, no further transition); no-flux walls.
    The constriction is a 3-layer wall plate normal to x with a central
    opening of `opening` x height, starting at x = size[0]/2 + amplitude and
    moving by amplitude (cos(2 pi t / period) - 1).  The concentration is
    carried by the scalar solver (cp = 1, kappa = D); the transport-velocity
    formulation is on with p_b = pb_factor p0."""
    dim = 2
    rng = np.random.default_rng(seed)
    nsites = (int(round(size[0] / dx)), int(round(size[1] / dx)))
    inner, walls, lo, hi = box_and_walls(dim, nsites, dx)
    ext = np.array([nsites[0] * dx, nsites[1] * dx])
    p0 = 1.0 * c * c
    mats = [
        Material(rho0=1.0, cp=1.0, kappa=0.25, T_t=C_t, switch_to=2),                    # 0 bolus (solid)
        Material(rho0=1.0, p0=p0, nu=100.0, cp=1.0, kappa=1.0, dirichlet=1),              # 1 gastric juice
        Material(rho0=1.0, p0=p0, nu=200.0, cp=1.0, kappa=0.25, T_t=C_t),                 # 2 chyme
        Material(rho0=1.0),                                                              # 3 wall (no flux)
    ]
    kind_of = np.full(inner.shape[0], FLUID, np.int32)
    phase_of = np.full(inner.shape[0], 1, np.int32)
    body_of = np.full(inner.shape[0], -1, np.int32)
    x0 = 0.5 * ext[0] + amplitude
    plate = np.abs(inner[:, 0] - x0) < 1.5 * dx
    plate &= ~(np.abs(inner[:, 1] - 0.5 * ext[1]) < 0.5 * opening * ext[1])
    kind_of[plate] = WALL
    phase_of[plate] = 3
    radii = np.sort(0.5 * rng.uniform(d_range[0], d_range[1], n_bolus))[::-1]
    placed = np.zeros((n_bolus, 2))
    placed_r = np.zeros(n_bolus)
    k = 0
    bodies = []
    for R in radii:
        for _ in range(500):
            cpos = np.array([rng.uniform(R + 2 * dx, ext[0] - R - 2 * dx), rng.uniform(R + 2 * dx, ext[1] - R - 2 * dx)])
            if abs(cpos[0] - x0) < R + 4 * dx:
                continue
            if np.any(np.sum((placed[:k] - cpos) ** 2, axis=1) < (placed_r[:k] + R + dx) ** 2):
                continue
            idx = ball_sites(nsites, dx, dim, np.array([cpos[0], cpos[1], 0.0]), R)
            idx = idx[kind_of[idx] == FLUID]
            if idx.size < 4:
                break
            placed[k] = cpos
            placed_r[k] = R
            k += 1
            kind_of[idx] = RIGID
            phase_of[idx] = 0
            body_of[idx] = len(bodies)
            bodies.append(BodyInit())
            break
    C = np.where(kind_of == RIGID, 0.0, 1.0)
    groups = [
        (inner[kind_of == FLUID], FLUID, 1, -1, 0, C[kind_of == FLUID]),
        (inner[kind_of == RIGID], RIGID, 0, body_of[kind_of == RIGID], 0, C[kind_of == RIGID]),
        (walls, WALL, 3, -1, 0, 0.0),
        (inner[kind_of == WALL], WALL, 3, -1, 1, 0.0),
    ]
    sc = _assemble("gastric", dim, dx, lo, hi, groups, mats, bodies, max_bodies=len(bodies),
                   thermal=1, phase_switch=1, wall_A=amplitude, wall_Omega=2.0 * math.pi / period,
                   wall_dir=(1.0, 0.0, 0.0))
    sc.x = jitter(sc.x, sc.kind == FLUID, dx, rng, dim)
    sc.p_b = pb_factor * p0
    sc.meta.update(seed=seed, c=c)
    return sc


def periodic_channel(dim: int = 2, n_sites=(20, 12, 9), dx: float = 0.05, g: float = 1.0, nu: float = 0.5,
                     c: float = 2.5, rho0: float = 1.0, seed: int = 0, jitter_amp: float = 0.01,
                     body_radius: float = 0.0, body_centre=None, body_density: float = 2.0) -> Scene:
    """Channel between two 3-layer walls normal to x (at x = 0 and x = n_x dx),
    periodic along y (and z in 3D) with periods n_y dx (n_z dx), which must
    be multiples of 3 sites (whole cells of edge 3 dx); body force g along y
    (a Poiseuille flow).  Optionally one rigid disc / sphere of body_radius
    around body_centre (which may straddle a periodic boundary)."""
    rng = np.random.default_rng(seed)
    nx, ny = int(n_sites[0]), int(n_sites[1])
    nz = int(n_sites[2]) if dim == 3 else 1
    if ny % 3 or (dim == 3 and nz % 3):
        raise ValueError("periodic extents must be whole cells (multiples of 3 sites)")
    layers = 3
    lo_idx = [0, 0, 0][:dim]
    hi_idx = [nx, ny, nz][:dim]
    inner = lattice_sites(dim, lo_idx, hi_idx, dx)
    wl = lattice_sites(dim, [-layers] + lo_idx[1:], [0] + hi_idx[1:], dx)
    wr = lattice_sites(dim, [nx] + lo_idx[1:], [nx + layers] + hi_idx[1:], dx)
    walls = np.concatenate([wl, wr])
    gvec = [0.0, 0.0, 0.0]
    gvec[1] = g
    mats = [Material(rho0=rho0, p0=rho0 * c * c, nu=nu, b=tuple(gvec)), Material(rho0=rho0),
            Material(rho0=body_density * rho0, b=tuple(gvec))]
    kind_of = np.full(inner.shape[0], FLUID, np.int32)
    bodies = []
    groups = []
    if body_radius > 0.0:
        cen = np.zeros(3)
        cen[:dim] = np.asarray(body_centre, dtype=np.float64)[:dim]
        per = np.array([0.0, ny * dx, nz * dx])
        # the body's sites, taken by minimum image, listed contiguously (they
        # may reach beyond the periodic box; set-up wraps them)
        d = inner - cen
        for a in (1, 2)[:dim - 1]:
            d[:, a] -= per[a] * np.round(d[:, a] / per[a])
        sel = np.sum(d[:, :dim] ** 2, axis=1) <= body_radius ** 2
        kind_of[sel] = RIGID
        groups.append((cen + d[sel], RIGID, 2, 0, 0, 0.0))
        bodies.append(BodyInit())
    groups.insert(0, (inner[kind_of == FLUID], FLUID, 0, -1, 0, 0.0))
    groups.append((walls, WALL, 1, -1, 0, 0.0))
    lo = np.zeros(3)
    hi = np.zeros(3)
    lo[0], hi[0] = -layers * dx, (nx + layers) * dx
    lo[1], hi[1] = 0.0, ny * dx
    if dim == 3:
        lo[2], hi[2] = 0.0, nz * dx
    sc = _assemble(f"channel{dim}d", dim, dx, lo, hi, groups, mats, bodies, max_bodies=len(bodies))
    sc.periodic = (0, 1, 1 if dim == 3 else 0)
    if jitter_amp > 0:
        sc.x = jitter(sc.x, sc.kind == FLUID, dx, rng, dim, jitter_amp)
    sc.meta.update(seed=seed, c=c)
    return sc


def config_e7(dx: float = 0.2) -> Scene:
    """Strong-scaling scene of Sec. "Strong scaling analysis": cubic box
    L = 30, 216 spheres D = 2.5 (density 10) on a regular grid with centres
    2.5 + 5 k, fluid density 1, nu = 1, c = 50, g = 1 downwards, 3-layer
    walls, cells of edge 0.65."""
    dim = 3
    n_side = int(round(30.0 / dx))
    inner, walls, lo, hi = box_and_walls(dim, (n_side,) * 3, dx)
    c = 50.0
    gvec = (0.0, 0.0, -1.0)
    mats = [Material(rho0=1.0, p0=c * c, nu=1.0, b=gvec), Material(rho0=1.0), Material(rho0=10.0, b=gvec)]
    kind_of = np.full(inner.shape[0], FLUID, np.int32)
    body_of = np.full(inner.shape[0], -1, np.int32)
    bodies = []
    for iz in range(6):
        for iy in range(6):
            for ix in range(6):
                centre = (2.5 + 5.0 * ix, 2.5 + 5.0 * iy, 2.5 + 5.0 * iz)
                sel = in_ball(inner, centre, 1.25, dim)
                kind_of[sel] = RIGID
                body_of[sel] = len(bodies)
                bodies.append(BodyInit())
    groups = [
        (inner[kind_of == FLUID], FLUID, 0, -1, 0, 0.0),
        (inner[kind_of == RIGID], RIGID, 2, body_of[kind_of == RIGID], 0, 0.0),
        (walls, WALL, 1, -1, 0, 0.0),
    ]
    # 48 cells of 0.65 cover [-0.6, 30.6] from lo = -0.6
    sc = _assemble("e7", dim, dx, lo, hi, groups, mats, bodies, cell_edge=0.65, max_bodies=len(bodies))
    sc.meta.update(c=c)
    return sc


# ----------------------------------------------------------------------------
# small scenes for tests
# ----------------------------------------------------------------------------

def fluid_box(dim: int, n_side: int, dx: float = 0.1, seed: int = 0, jitter_amp: float = 0.01,
              g: float = 0.0, nu: float = 0.1, c: float = 10.0, rho0: float = 1.0, walls: bool = True,
              shape=None) -> Scene:
    rng = np.random.default_rng(seed)
    shape = tuple(shape) if shape is not None else (n_side,) * dim
    inner, wall, lo, hi = box_and_walls(dim, shape, dx)
    gvec = [0.0, 0.0, 0.0]
    gvec[dim - 1] = -g
    mats = [Material(rho0=rho0, p0=rho0 * c * c, nu=nu, b=tuple(gvec)), Material(rho0=rho0)]
    groups = [(inner, FLUID, 0, -1, 0, 0.0)]
    if walls:
        groups.append((wall, WALL, 1, -1, 0, 0.0))
    sc = _assemble(f"fluid_box{dim}d", dim, dx, lo, hi, groups, mats, [], max_bodies=0)
    if jitter_amp > 0:
        sc.x = jitter(sc.x, sc.kind == FLUID, dx, rng, dim, jitter_amp)
    return sc


def random_cloud(dim: int, n: int, extent: float, dx: float, seed: int = 0, clustered: bool = False) -> Scene:
    """Random fluid cloud (optionally clustered) for neighbour-search checks."""
    rng = np.random.default_rng(seed)
    if clustered:
        centres = rng.uniform(0.2 * extent, 0.8 * extent, size=(max(1, n // 50), 3))
        pick = rng.integers(0, centres.shape[0], size=n)
        x = centres[pick] + rng.normal(0.0, 0.05 * extent, size=(n, 3))
        x = np.clip(x, 0.0, extent * 0.999)
    else:
        x = rng.uniform(0.0, extent, size=(n, 3))
    if dim == 2:
        x[:, 2] = 0.0
    lo = np.zeros(3)
    hi = np.zeros(3)
    hi[:dim] = extent
    mats = [Material(rho0=1.0, p0=100.0, nu=0.1)]
    sc = _assemble(f"cloud{dim}d", dim, dx, lo, hi, [(x, FLUID, 0, -1, 0, 0.0)], mats, [], max_bodies=0)
    return sc


def isolated_blob_with_body(dim: int = 2, n_side: int = 16, dx: float = 0.1, seed: int = 0,
                            body_radius: float = 0.25, u0=(0.3, -0.2, 0.1), w0=(0.0, 0.0, 2.0)) -> Scene:
    """Fluid blob in free space (no walls, no body force) containing one
    freely moving rigid body: an isolated system for momentum checks."""
    rng = np.random.default_rng(seed)
    inner = lattice_sites(dim, [0] * dim, [n_side] * dim, dx)
    ext = n_side * dx
    centre = np.array([0.5 * ext] * 3)
    if dim == 2:
        centre[2] = 0.0
    disc = in_ball(inner, centre, body_radius, dim)
    mats = [Material(rho0=1.0, p0=100.0, nu=0.05), Material(rho0=1.0), Material(rho0=2.0)]
    groups = [(inner[~disc], FLUID, 0, -1, 0, 0.0), (inner[disc], RIGID, 2, 0, 0, 0.0)]
    lo = np.zeros(3)
    hi = np.zeros(3)
    lo[:dim] = -ext
    hi[:dim] = 2.0 * ext
    sc = _assemble("blob", dim, dx, lo, hi, groups, mats,
                   [BodyInit(u=tuple(u0), w=tuple(w0))], max_bodies=1)
    sc.x = jitter(sc.x, sc.kind == FLUID, dx, rng, dim)
    sc.u[sc.kind == FLUID, :dim] = rng.normal(0.0, 0.1, size=(int(np.sum(sc.kind == FLUID)), dim))
    return sc


def single_body(dim: int, radius_sites: float = 3.0, dx: float = 0.1, g: float = 9.81,
                u0=(0.0, 0.0, 0.0), w0=(0.0, 0.0, 0.0), q0=(1.0, 0.0, 0.0, 0.0), extent: float = 3.0) -> Scene:
    """One rigid ball (site-centred) in empty space: free fall and spin checks."""
    r = int(math.ceil(radius_sites)) + 1
    sites = lattice_sites(dim, [-r] * dim, [r] * dim, dx)
    centre = np.zeros(3)
    centre[:dim] = 0.5 * dx
    sel = in_ball(sites, centre, radius_sites * dx, dim)
    x = sites[sel]
    gvec = [0.0, 0.0, 0.0]
    gvec[dim - 1] = -g
    mats = [Material(rho0=1.0, p0=1.0, nu=0.0), Material(rho0=1.0), Material(rho0=3.0, b=tuple(gvec))]
    lo = np.zeros(3)
    hi = np.zeros(3)
    lo[:dim] = -extent
    hi[:dim] = extent
    return _assemble("single_body", dim, dx, lo, hi, [(x, RIGID, 2, 0, 0, 0.0)], mats,
                     [BodyInit(u=tuple(u0), w=tuple(w0), q=tuple(q0))], max_bodies=1, contact=0)


def two_particle_bodies(dim: int = 2, dx: float = 0.1, gap: float = 0.5, speed: float = 1.0,
                        k_c: float = 1e4, d_c: float = 0.0) -> Scene:
    """Two one-particle bodies approaching head-on along x (contact check)."""
    x = np.zeros((2, 3))
    x[0, 0] = -0.5 * (dx + gap)
    x[1, 0] = 0.5 * (dx + gap)
    mats = [Material(rho0=1.0, p0=1.0), Material(rho0=1.0), Material(rho0=1.0)]
    lo = np.zeros(3)
    hi = np.zeros(3)
    lo[:dim] = -10.0
    hi[:dim] = 10.0
    sc = _assemble("two_bodies", dim, dx, lo, hi,
                   [(x[:1], RIGID, 2, 0, 0, 0.0), (x[1:], RIGID, 2, 1, 0, 0.0)], mats,
                   [BodyInit(u=(speed, 0.0, 0.0)), BodyInit(u=(-speed, 0.0, 0.0))],
                   max_bodies=2, k_c=k_c, d_c=d_c)
    return sc


def frozen_lattice(dim: int, n_side: int, dx: float = 0.1, rho0: float = 1.0, cp: float = 1.0,
                   kappa: float = 1.0, nu: float = 0.0, p0: float = 1.0) -> Scene:
    """Unjittered fluid lattice in free space, for operator checks on frozen
    particles (interior particles have full kernel support)."""
    x = lattice_sites(dim, [0] * dim, [n_side] * dim, dx)
    mats = [Material(rho0=rho0, p0=p0, nu=nu, cp=cp, kappa=kappa)]
    lo = np.zeros(3)
    hi = np.zeros(3)
    lo[:dim] = -1.0
    hi[:dim] = n_side * dx + 1.0
    return _assemble(f"frozen{dim}d", dim, dx, lo, hi, [(x, FLUID, 0, -1, 0, 0.0)], mats, [],
                     max_bodies=0, thermal=1)


def disc_sites(dim: int, diameter: float, dx: float, centre_on: str = "vertex") -> np.ndarray:
    """Lattice sites inside a disc (2D) or ball (3D) of the given diameter,
    the lattice aligned so that the centre is a lattice vertex or a site."""
    R = 0.5 * diameter
    r = int(math.ceil(R / dx)) + 2
    sites = lattice_sites(dim, [-r] * dim, [r] * dim, dx)
    centre = np.zeros(3)
    if centre_on == "site":
        centre[:dim] = 0.5 * dx
    return sites[in_ball(sites, centre, R, dim)]
