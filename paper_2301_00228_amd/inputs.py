"""Seeded synthetic inputs for the plane-strain LBM.

This module only builds problem data -- masks, material constants, time
steps, initial displacement pulses and boundary-node lists -- in the shapes
of the paper's problem statement (Sec. 2: body, Dirichlet part, Neumann part,
Lame parameters; Sec. 3: lattice spacing, time step).  It holds none of the
method's arithmetic and is the only module shared by the GPU library's tests
and the CPU oracle's tests.

Units are lattice units: dh = 1, mu = 1, rho = 1, lambda = 2 nu / (1 - 2 nu).
The time step follows from the equilibrium weight a0_phi through
dt = dh sqrt(2 a_phi) / c_d with a_phi = (1 - a0_phi) / 4 (Sec. 3, eq.
conditions-parameters), c_d = sqrt(lambda + 2 mu) (Sec. 2).
"""
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

MASTER_SEED = 0x230100228

# Edge codes for rectangular plates.
LEFT, RIGHT, BOTTOM, TOP = 0, 1, 2, 3

NEUMANN, DIRICHLET = 0, 1


@dataclass
class BoundaryData:
    """Boundary data for a set of boundary nodes (one ``set_bc`` call)."""
    xy: np.ndarray                       # (n, 2) int32 node coordinates (i, j)
    kind: np.ndarray                     # (n,) uint8: 0 Neumann, 1 Dirichlet
    val: np.ndarray                      # (n, 2) float64: u* or integrated external force
    cell: Optional[np.ndarray] = None    # (n, 5) float64 (V, lE, lN, lW, lS) or None
    knots: Optional[np.ndarray] = None   # (k, 2) float64 (t, g) amplitude knots or None


@dataclass
class Case:
    """One plate: geometry, material, time step, initial data, boundary data."""
    name: str
    nx: int
    ny: int
    mask: Optional[np.ndarray]           # (ny, nx) uint8, 1 = body; None = full rectangle
    periodic: Tuple[bool, bool]
    lam: float
    mu: float
    rho: float
    dh: float
    dt: float
    sync_every: int
    u0: Optional[np.ndarray]             # (2, ny, nx)
    v0: Optional[np.ndarray]
    e0: Optional[np.ndarray]             # (ny, nx) direct initial dilatation, or None
    w0: Optional[np.ndarray]             # (ny, nx) direct initial rotation, or None
    bcs: List[BoundaryData] = field(default_factory=list)
    steps: int = 0
    nu: float = 0.3
    a0_phi: float = 0.0
    # ellipses that carved the mask: (cx, cy, a, b, angle, kind), kind 0 =
    # hole (interior removed), 1 = bound (exterior removed); a node is in the
    # body iff its position is (points on an ellipse are)
    shapes: list = field(default_factory=list)
    # displacement update: 0 as printed in the paper, 1 central difference
    integrator: int = 0
    # readings of Sec. 3.1: (flux of eq. correction-f: 0 = R1 the boundary
    # node's own populations, 1 = R2 the populations streamed in from its
    # body neighbours; equilibrium of eq. LBE_mod: 0 = M1 the averaged
    # populations' own, 1 = M2 the boundary node's populations at t)
    readings: Tuple[int, int] = (0, 0)

    def in_body_nodes(self) -> int:
        return int(self.nx * self.ny if self.mask is None else int(np.count_nonzero(self.mask)))


def lame_lambda(nu: float, mu: float = 1.0) -> float:
    return 2.0 * nu * mu / (1.0 - 2.0 * nu)


def time_step(nu: float, a0_phi: float, dh: float = 1.0, mu: float = 1.0, rho: float = 1.0) -> float:
    lam = lame_lambda(nu, mu)
    cd = np.sqrt((lam + 2.0 * mu) / rho)
    a_phi = (1.0 - a0_phi) / 4.0
    return float(dh * np.sqrt(2.0 * a_phi) / cd)


def rng_for(config_index: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng([MASTER_SEED + config_index, sub])


def gaussian_pulse(nx, ny, cx, cy, sigma, amp, theta):
    """Displacement pulse u0 = A exp(-|x-x0|^2 / 2 sigma^2) (cos theta, sin theta)."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    g = amp * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * sigma * sigma))
    return np.stack([g * np.cos(theta), g * np.sin(theta)])


def edge_nodes(nx, ny, edge):
    if edge == LEFT:
        return np.stack([np.zeros(ny, np.int32), np.arange(ny, dtype=np.int32)], 1)
    if edge == RIGHT:
        return np.stack([np.full(ny, nx - 1, np.int32), np.arange(ny, dtype=np.int32)], 1)
    if edge == BOTTOM:
        return np.stack([np.arange(nx, dtype=np.int32), np.zeros(nx, np.int32)], 1)
    return np.stack([np.arange(nx, dtype=np.int32), np.full(nx, ny - 1, np.int32)], 1)


def dirichlet_edges_bc(nx, ny, edges):
    """Homogeneous Dirichlet data (u* = 0) on the listed rectangle edges.
    Corner nodes shared with a free edge are Dirichlet."""
    if not edges:
        return None
    pts = np.unique(np.concatenate([edge_nodes(nx, ny, e) for e in edges]), axis=0)
    n = pts.shape[0]
    return BoundaryData(pts.astype(np.int32), np.full(n, DIRICHLET, np.uint8), np.zeros((n, 2)))


def _clear_dirichlet(u0, bcs):
    for bc in bcs:
        d = bc.kind == DIRICHLET
        u0[:, bc.xy[d, 1], bc.xy[d, 0]] = bc.val[d].T
    return u0


# --------------------------------------------------------------------------
# Workloads.  Each function returns a Case (or a list of Cases for batches).
# --------------------------------------------------------------------------

def periodic_square(n=64, nu=0.3, a0_phi=0.0, steps=500, seed_index=0, sigma=4.0, amp=1e-3):
    """Periodic n x n square: e0 = sin(2 pi x/n) sin(2 pi y/n), omega0 a
    Gaussian (minimum-image distance to a seeded centre), u0 = v0 = 0."""
    rng = rng_for(seed_index)
    cx, cy = rng.uniform(0, n, size=2)
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    e0 = np.sin(2 * np.pi * x / n) * np.sin(2 * np.pi * y / n)
    dx = np.abs(x - cx)
    dx = np.minimum(dx, n - dx)
    dy = np.abs(y - cy)
    dy = np.minimum(dy, n - dy)
    w0 = amp * np.exp(-(dx * dx + dy * dy) / (2 * sigma * sigma))
    return Case(name=f"periodic{n}", nx=n, ny=n, mask=None, periodic=(True, True),
                lam=lame_lambda(nu), mu=1.0, rho=1.0, dh=1.0, dt=time_step(nu, a0_phi),
                sync_every=0, u0=None, v0=None, e0=e0, w0=w0, bcs=[], steps=steps, nu=nu,
                a0_phi=a0_phi)


def clamped_plate(n=1024, nu=0.3, a0_phi=0.9999, steps=5000, sync_every=50, sigma=16.0,
                  amp=1e-3, seed_index=1, ny=None):
    """Square plate, left edge Dirichlet u* = 0, other edges traction free,
    one seeded Gaussian displacement pulse released from rest."""
    nx, ny = n, (n if ny is None else ny)
    rng = rng_for(seed_index)
    lo = 6 * sigma
    cx = rng.uniform(min(lo, nx / 2), max(nx - 1 - lo, nx / 2))
    cy = rng.uniform(min(lo, ny / 2), max(ny - 1 - lo, ny / 2))
    theta = rng.uniform(0, 2 * np.pi)
    u0 = gaussian_pulse(nx, ny, cx, cy, sigma, amp, theta)
    bcs = [dirichlet_edges_bc(nx, ny, [LEFT])]
    _clear_dirichlet(u0, bcs)
    return Case(name=f"clamped{nx}x{ny}", nx=nx, ny=ny, mask=None, periodic=(False, False),
                lam=lame_lambda(nu), mu=1.0, rho=1.0, dh=1.0, dt=time_step(nu, a0_phi),
                sync_every=sync_every, u0=u0, v0=np.zeros_like(u0), e0=None, w0=None, bcs=bcs,
                steps=steps, nu=nu, a0_phi=a0_phi)


SHAPE_HOLE, SHAPE_BOUND = 0, 1


def shape_mask(nx, ny, shapes):
    """Mask of the lattice nodes inside the body bounded by the shapes."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    mask = np.ones((ny, nx), np.uint8)
    for cx, cy, a, b, ang, kind in shapes:
        ca, sa = np.cos(ang), np.sin(ang)
        xr = ca * (x - cx) + sa * (y - cy)
        yr = -sa * (x - cx) + ca * (y - cy)
        r2 = (xr / a) ** 2 + (yr / b) ** 2
        mask[(r2 < 1.0) if kind == SHAPE_HOLE else (r2 > 1.0)] = 0
    return mask


def boundary_nodes(mask, periodic=(False, False)):
    """(n, 2) coordinates of the body nodes with a missing D2Q5 neighbour
    (the lattice edge of a non-periodic axis counts as missing)."""
    m = mask.astype(bool)
    ny, nx = m.shape
    miss = np.zeros_like(m)
    for ax, per in ((1, periodic[0]), (0, periodic[1])):
        for sh in (1, -1):
            nb = np.roll(m, sh, axis=ax)
            if not per:
                idx = [slice(None)] * 2
                idx[ax] = 0 if sh == 1 else -1
                nb[tuple(idx)] = False
            miss |= ~nb
    j, i = np.nonzero(m & miss)
    return np.stack([i, j], 1).astype(np.int32)


def plate_with_ellipse_hole(nx=96, ny=80, hole=(47.3, 38.6, 15.0, 9.5, 0.5), nu=0.3, a0_phi=0.5,
                            steps=300, sync_every=50, sigma=4.0, amp=1e-3, seed_index=5,
                            clamped=(LEFT,)):
    """Rectangular plate with one elliptic hole (cx, cy, a, b, angle), the
    listed outer edges Dirichlet u* = 0, every other boundary node traction
    free; one seeded pulse between the hole and the plate edges."""
    rng = rng_for(seed_index)
    shapes = [tuple(hole) + (SHAPE_HOLE,)]
    mask = shape_mask(nx, ny, shapes)
    for _ in range(1000):
        cx, cy = rng.uniform(3 * sigma, nx - 1 - 3 * sigma), rng.uniform(3 * sigma, ny - 1 - 3 * sigma)
        if mask[int(round(cy)), int(round(cx))]:
            break
    theta = rng.uniform(0, 2 * np.pi)
    u0 = gaussian_pulse(nx, ny, cx, cy, sigma, amp, theta) * mask[None]
    bc = dirichlet_edges_bc(nx, ny, list(clamped))
    bcs = [bc] if bc is not None else []
    _clear_dirichlet(u0, bcs)
    return Case(name=f"ellipse_hole{nx}x{ny}", nx=nx, ny=ny, mask=mask, periodic=(False, False),
                lam=lame_lambda(nu), mu=1.0, rho=1.0, dh=1.0, dt=time_step(nu, a0_phi),
                sync_every=sync_every, u0=u0, v0=np.zeros_like(u0), e0=None, w0=None, bcs=bcs,
                steps=steps, nu=nu, a0_phi=a0_phi, shapes=shapes)


def hole_mask(n, radius, cx=None, cy=None):
    cx = (n - 1) / 2.0 if cx is None else cx
    cy = (n - 1) / 2.0 if cy is None else cy
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    return (((x - cx) ** 2 + (y - cy) ** 2) >= radius * radius).astype(np.uint8)


def plate_with_hole(n=8192, radius=1024, nu=0.3, a0_phi=0.9999, steps=2000, sync_every=50,
                    sigma=16.0, amp=1e-3, seed_index=2):
    """Square plate with a central circular hole (traction-free rim), outer
    edges Dirichlet u* = 0, one seeded pulse on the annulus around the hole."""
    rng = rng_for(seed_index)
    c = (n - 1) / 2.0
    r_lo = radius + 6 * sigma
    r_hi = min(1.5 * radius, c - 6 * sigma)
    r = rng.uniform(r_lo, max(r_hi, r_lo))
    ang = rng.uniform(0, 2 * np.pi)
    theta = rng.uniform(0, 2 * np.pi)
    mask = hole_mask(n, radius)
    u0 = gaussian_pulse(n, n, c + r * np.cos(ang), c + r * np.sin(ang), sigma, amp, theta)
    u0 *= mask[None]
    bcs = [dirichlet_edges_bc(n, n, [LEFT, RIGHT, BOTTOM, TOP])]
    _clear_dirichlet(u0, bcs)
    return Case(name=f"hole{n}r{radius}", nx=n, ny=n, mask=mask, periodic=(False, False),
                lam=lame_lambda(nu), mu=1.0, rho=1.0, dh=1.0, dt=time_step(nu, a0_phi),
                sync_every=sync_every, u0=u0, v0=np.zeros_like(u0), e0=None, w0=None, bcs=bcs,
                steps=steps, nu=nu, a0_phi=a0_phi,
                shapes=[(c, c, float(radius), float(radius), 0.0, SHAPE_HOLE)])


def plate_batch(count=256, side_lo=64, side_hi=1024, nu_lo=0.1, nu_hi=0.45, a0_phi=0.9999,
                steps=1000, sync_every=50, amp=1e-3, seed_index=3):
    """Independent rectangular plates of seeded uneven sizes and materials,
    each edge Dirichlet (u* = 0) or traction free with probability 1/2, one
    seeded pulse each (sigma = max(2, min(nx, ny)/32))."""
    rng = rng_for(seed_index)
    cases = []
    for p in range(count):
        nx = int(rng.integers(side_lo, side_hi + 1))
        ny = int(rng.integers(side_lo, side_hi + 1))
        nu = float(rng.uniform(nu_lo, nu_hi))
        edges = [e for e in (LEFT, RIGHT, BOTTOM, TOP) if rng.random() < 0.5]
        sigma = max(2.0, min(nx, ny) / 32.0)
        lo = 6 * sigma
        cx = rng.uniform(lo, nx - 1 - lo)
        cy = rng.uniform(lo, ny - 1 - lo)
        theta = rng.uniform(0, 2 * np.pi)
        u0 = gaussian_pulse(nx, ny, cx, cy, sigma, amp, theta)
        bc = dirichlet_edges_bc(nx, ny, edges)
        bcs = [bc] if bc is not None else []
        _clear_dirichlet(u0, bcs)
        cases.append(Case(name=f"batch{p}", nx=nx, ny=ny, mask=None, periodic=(False, False),
                          lam=lame_lambda(nu), mu=1.0, rho=1.0, dh=1.0, dt=time_step(nu, a0_phi),
                          sync_every=sync_every, u0=u0, v0=np.zeros_like(u0), e0=None, w0=None,
                          bcs=bcs, steps=steps, nu=nu, a0_phi=a0_phi))
    return cases


def ellipse_holes_mask(nx, ny, area_frac, rng, a_lo=8.0, a_hi=64.0, clearance=4.0,
                       max_tries=200000):
    """Random non-overlapping elliptic holes until their area reaches
    area_frac of the plate.  Semi-axes a ~ U[a_lo, a_hi], b ~ U[a/4, a],
    angle ~ U[0, pi); holes keep `clearance` nodes from each other and from
    the plate edges (tested on bounding circles).  Returns the mask and the
    holes as shapes (cx, cy, a, b, angle, SHAPE_HOLE)."""
    mask = np.ones((ny, nx), np.uint8)
    shapes = []
    target = area_frac * nx * ny
    area = 0.0
    placed = []  # (cx, cy, R)
    tries = 0
    a_hi = min(a_hi, (min(nx, ny) - 1) / 2.0 - clearance - 3.0)
    a_lo = min(a_lo, a_hi)
    while area < target and tries < max_tries:
        tries += 1
        a = rng.uniform(a_lo, a_hi)
        b = rng.uniform(a / 4, a)
        ang = rng.uniform(0, np.pi)
        R = a + clearance
        cx = rng.uniform(R + 2, nx - 1 - R - 2)
        cy = rng.uniform(R + 2, ny - 1 - R - 2)
        if any((cx - px) ** 2 + (cy - py) ** 2 < (R + pr) ** 2 for px, py, pr in placed):
            continue
        placed.append((cx, cy, R))
        x0, x1 = int(np.floor(cx - a)) - 1, int(np.ceil(cx + a)) + 2
        y0, y1 = int(np.floor(cy - a)) - 1, int(np.ceil(cy + a)) + 2
        yy, xx = np.mgrid[y0:y1, x0:x1].astype(np.float64)
        dx, dy = xx - cx, yy - cy
        ca, sa = np.cos(ang), np.sin(ang)
        xr, yr = ca * dx + sa * dy, -sa * dx + ca * dy
        inside = (xr / a) ** 2 + (yr / b) ** 2 < 1.0
        mask[y0:y1, x0:x1][inside] = 0
        area += np.pi * a * b
        shapes.append((cx, cy, a, b, ang, SHAPE_HOLE))
    return mask, shapes


def strip_with_holes(nx=65536, ny=2048, area_frac=0.05, nu=0.3, a0_phi=0.9999, steps=2000,
                     sync_every=50, sigma=32.0, amp=1e-3, pulses=8, seed_index=4, a_lo=8.0,
                     a_hi=64.0):
    """Long strip with seeded elliptic traction-free holes (area_frac of the
    plate), outer edges Dirichlet u* = 0 or free with probability 1/2,
    several seeded pulses."""
    rng = rng_for(seed_index, 1)
    mask, shapes = ellipse_holes_mask(nx, ny, area_frac, rng, a_lo=a_lo, a_hi=a_hi)
    edges = [e for e in (LEFT, RIGHT, BOTTOM, TOP) if rng.random() < 0.5]
    u0 = np.zeros((2, ny, nx))
    lo = 6 * sigma
    for _ in range(pulses):
        cx = rng.uniform(lo, nx - 1 - lo)
        cy = rng.uniform(lo, ny - 1 - lo)
        th = rng.uniform(0, 2 * np.pi)
        x0, x1 = int(max(0, cx - 8 * sigma)), int(min(nx, cx + 8 * sigma + 1))
        y0, y1 = int(max(0, cy - 8 * sigma)), int(min(ny, cy + 8 * sigma + 1))
        u0[:, y0:y1, x0:x1] += gaussian_pulse(x1 - x0, y1 - y0, cx - x0, cy - y0, sigma, amp, th)
    u0 *= mask[None]
    bc = dirichlet_edges_bc(nx, ny, edges)
    bcs = [bc] if bc is not None else []
    _clear_dirichlet(u0, bcs)
    return Case(name=f"strip{nx}x{ny}", nx=nx, ny=ny, mask=mask, periodic=(False, False),
                lam=lame_lambda(nu), mu=1.0, rho=1.0, dh=1.0, dt=time_step(nu, a0_phi),
                sync_every=sync_every, u0=u0, v0=np.zeros_like(u0), e0=None, w0=None, bcs=bcs,
                steps=steps, nu=nu, a0_phi=a0_phi, shapes=shapes)


def mixed_plate(nx, ny, rng, nu=0.3, a0_phi=0.9999, steps=2000, sync_every=50, sigma=32.0,
                amp=1e-3, name="plate", with_v0=False):
    """Rectangular plate, each edge Dirichlet (u* = 0) or traction free with
    probability 1/2, one seeded pulse."""
    edges = [e for e in (LEFT, RIGHT, BOTTOM, TOP) if rng.random() < 0.5]
    lo = 6 * sigma
    cx = rng.uniform(lo, nx - 1 - lo)
    cy = rng.uniform(lo, ny - 1 - lo)
    theta = rng.uniform(0, 2 * np.pi)
    u0 = gaussian_pulse(nx, ny, cx, cy, sigma, amp, theta)
    bc = dirichlet_edges_bc(nx, ny, edges)
    bcs = [bc] if bc is not None else []
    _clear_dirichlet(u0, bcs)
    return Case(name=name, nx=nx, ny=ny, mask=None, periodic=(False, False),
                lam=lame_lambda(nu), mu=1.0, rho=1.0, dh=1.0, dt=time_step(nu, a0_phi),
                sync_every=sync_every, u0=u0, v0=np.zeros_like(u0) if with_v0 else None, e0=None,
                w0=None, bcs=bcs, steps=steps, nu=nu, a0_phi=a0_phi)


def large_batch(count=64, side=4096, strip=(65536, 2048), steps=2000, seed_index=4):
    """count plates of side x side (mixed edges, one pulse each, sigma 32)
    plus one strip with seeded elliptic holes; v0 = 0 (not materialized)."""
    rng = rng_for(seed_index)
    cases = [mixed_plate(side, side, rng, steps=steps, name=f"sq{k}") for k in range(count)]
    if strip is not None:
        st = strip_with_holes(nx=strip[0], ny=strip[1], steps=steps, seed_index=seed_index)
        st.v0 = None
        cases.append(st)
    return cases


def mixed_batch(steps=2000, seed_index=6):
    """A small mixed batch for precision checks of the batched path against
    the oracle: five rectangular plates of the 256-plate recipe (sides
    U{128..320}, random clamped / free edges, one pulse each), a plate with
    one elliptic hole and a strip with seeded elliptic holes (5 % of its
    area, three pulses); a0_phi = 0.9999, synchronization every 50 steps."""
    cases = plate_batch(count=5, side_lo=128, side_hi=320, steps=steps, seed_index=seed_index)
    cases.append(plate_with_ellipse_hole(nx=200, ny=160, hole=(97.3, 81.6, 31.0, 17.5, 0.7),
                                         a0_phi=0.9999, steps=steps, sync_every=50, sigma=6.0,
                                         seed_index=seed_index))
    cases.append(strip_with_holes(nx=480, ny=120, sigma=8.0, pulses=3, steps=steps,
                                  seed_index=seed_index, a_lo=6.0, a_hi=20.0))
    return cases
