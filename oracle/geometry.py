"""Exact-geometry boundary cells, computed the slow way.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): the test-suite uses
it to check the library's ``lbm_exact_cells`` and to feed the same cell
tables to the oracle and the GPU library.

Sec. 3.1 builds, at each boundary lattice point, a cell that starts as the
square of side dh centred on the point and is cut to the body's boundary;
its volume V_C and the lengths of its sides towards its neighbours enter the
Neumann acceleration (eq. acc_neumann).  A side towards a neighbour outside
the body has no length in the table: the sliver of body beyond it (where
the boundary passes beyond the square) is taken as massless, passing the
boundary's traction to the cell, so the closure of the cell's normals gives
the rim normal integral of the cell and its slivers.

The body here is the lattice rectangle [0, nx-1] x [0, ny-1] (lattice
units, node (i, j) at (i, j); a periodic axis is not bounded) minus the open
interiors of "hole" ellipses and the open exteriors of "bound" ellipses, the
removed sets pairwise disjoint.

Method (independent of the library's, which sums triangle and sector areas
in the coordinates where an ellipse is a circle): the length of a straight
line's part inside the body is found by solving the quadratic of the
ellipse along that line; the area of a clipped square is the integral over
x of the inside length of the vertical line through x, by adaptive
quadrature (scipy.integrate.quad) with the kinks (where a chord end crosses
the square's bottom or top, or the line is tangent to an ellipse) passed as
break points.
"""
import math

import numpy as np
from scipy.integrate import quad

HOLE, BOUND = 0, 1


def _chord(px, py, dx, dy, shape):
    """Parameter interval [t0, t1] (possibly empty: None) of the line
    (px, py) + t (dx, dy) inside the closed ellipse."""
    cx, cy, a, b, ang, _ = shape
    c, s = math.cos(ang), math.sin(ang)
    # ellipse frame coordinates along the line: u = u0 + t du, v = v0 + t dv
    u0 = c * (px - cx) + s * (py - cy)
    v0 = -s * (px - cx) + c * (py - cy)
    du = c * dx + s * dy
    dv = -s * dx + c * dy
    # (u/a)^2 + (v/b)^2 - 1 = A t^2 + B t + C
    A = (du / a) ** 2 + (dv / b) ** 2
    B = 2.0 * (u0 * du / a ** 2 + v0 * dv / b ** 2)
    C = (u0 / a) ** 2 + (v0 / b) ** 2 - 1.0
    disc = B * B - 4.0 * A * C
    if A == 0.0 or disc <= 0.0:
        return None
    r = math.sqrt(disc)
    t0, t1 = (-B - r) / (2.0 * A), (-B + r) / (2.0 * A)
    return (min(t0, t1), max(t0, t1))


def inside_length(p0, p1, shapes):
    """Length of the segment p0 -> p1 that lies in the body (the segment is
    already inside the lattice rectangle)."""
    dx, dy = p1[0] - p0[0], p1[1] - p0[1]
    full = math.hypot(dx, dy)
    if full == 0.0:
        return 0.0
    removed = 0.0
    for sh in shapes:
        ch = _chord(p0[0], p0[1], dx, dy, sh)
        inside = 0.0
        if ch is not None:
            inside = max(0.0, min(ch[1], 1.0) - max(ch[0], 0.0)) * full
        removed += inside if sh[5] == HOLE else full - inside
    return full - removed


def _kinks(x0, x1, y0, y1, shapes):
    """x positions in (x0, x1) where the inside length of a vertical line is
    not smooth."""
    pts = []
    for sh in shapes:
        cx, cy, a, b, ang, _ = sh
        c, s = math.cos(ang), math.sin(ang)
        half = math.sqrt((a * c) ** 2 + (b * s) ** 2)  # half extent in x
        pts += [cx - half, cx + half]
        for yy in (y0, y1):  # crossings of the horizontal lines y0, y1
            ch = _chord(x0, yy, 1.0, 0.0, sh)
            if ch is not None:
                pts += [x0 + ch[0], x0 + ch[1]]
    return sorted(p for p in pts if x0 < p < x1)


def cell_of(i, j, nx, ny, shapes, periodic=(False, False), sides="body"):
    """(V, l_E, l_N, l_W, l_S) of node (i, j) in lattice units; sides =
    "body": lengths of the sides towards neighbours in the body (others 0),
    "all": the inside length of every side of the square."""
    def clip(lo, hi, n, per):
        return (lo, hi) if per else (max(lo, 0.0), min(hi, float(n - 1)))

    x0, x1 = clip(i - 0.5, i + 0.5, nx, periodic[0])
    y0, y1 = clip(j - 0.5, j + 0.5, ny, periodic[1])
    if x1 <= x0 or y1 <= y0:
        return (0.0, 0.0, 0.0, 0.0, 0.0)

    def h(x):
        return inside_length((x, y0), (x, y1), shapes)

    V, _ = quad(h, x0, x1, points=_kinks(x0, x1, y0, y1, shapes) or None, epsabs=1e-14,
                epsrel=1e-13, limit=200)
    # a side exists where the square is not cut at the node by a lattice edge
    lE = inside_length((i + 0.5, y0), (i + 0.5, y1), shapes) if (periodic[0] or i + 0.5 <= nx - 1) else 0.0
    lW = inside_length((i - 0.5, y0), (i - 0.5, y1), shapes) if (periodic[0] or i - 0.5 >= 0) else 0.0
    lN = inside_length((x0, j + 0.5), (x1, j + 0.5), shapes) if (periodic[1] or j + 0.5 <= ny - 1) else 0.0
    lS = inside_length((x0, j - 0.5), (x1, j - 0.5), shapes) if (periodic[1] or j - 0.5 >= 0) else 0.0
    if sides == "body":
        def nb(ii, jj):
            if periodic[0]:
                ii %= nx
            if periodic[1]:
                jj %= ny
            return 0 <= ii < nx and 0 <= jj < ny and in_body(ii, jj, nx, ny, shapes, periodic)
        lE = lE if nb(i + 1, j) else 0.0
        lN = lN if nb(i, j + 1) else 0.0
        lW = lW if nb(i - 1, j) else 0.0
        lS = lS if nb(i, j - 1) else 0.0
    return (max(V, 0.0), max(lE, 0.0), max(lN, 0.0), max(lW, 0.0), max(lS, 0.0))


def cells(nx, ny, shapes, xy, dh=1.0, periodic=(False, False), sides="body"):
    """Cell table (n, 5): V_C (dh^2 units), l_E, l_N, l_W, l_S (dh units) of
    the nodes xy (n, 2)."""
    out = np.array([cell_of(int(i), int(j), nx, ny, shapes, periodic, sides) for i, j in np.asarray(xy)],
                   dtype=np.float64).reshape(-1, 5)
    out[:, 0] *= dh * dh
    out[:, 1:] *= dh
    return out


def in_body(x, y, nx, ny, shapes, periodic=(False, False)):
    """Whether the point (x, y) (lattice units) belongs to the body."""
    if not periodic[0] and not (0.0 <= x <= nx - 1):
        return False
    if not periodic[1] and not (0.0 <= y <= ny - 1):
        return False
    for cx, cy, a, b, ang, kind in shapes:
        c, s = math.cos(ang), math.sin(ang)
        u = c * (x - cx) + s * (y - cy)
        v = -s * (x - cx) + c * (y - cy)
        r2 = (u / a) ** 2 + (v / b) ** 2
        if (kind == HOLE and r2 < 1.0) or (kind == BOUND and r2 > 1.0):
            return False
    return True


def rim_normal(cell):
    """Integral of the outward normal over the body boundary of each cell
    (and of the slivers beyond its sides towards missing neighbours):
    minus the normals of its sides times their lengths (closure)."""
    cell = np.asarray(cell, dtype=np.float64).reshape(-1, 5)
    return np.stack([-(cell[:, 1] - cell[:, 3]), -(cell[:, 2] - cell[:, 4])], 1)
