"""Physics checks of the GPU library beyond parity with the oracle, and the
paper's numerical examples (Sec. 4) rerun on synthetic setups.

    python -m paper_2301_00228_amd.experiments disc --radii 16 32 64
    python -m paper_2301_00228_amd.experiments paper --L 128

paper: the three examples of Sec. 4 -- a square of side L under a tensile
traction on its top and bottom edges (ramped to 0.005 mu over L / c_s, then
held), under a shear traction on its top edge growing as 0.005 mu c_s t / L
with the bottom edge clamped, and the tension case with a central circular
hole of diameter 0.266 L -- with c_s / c_d = 1 / sqrt(3) (lambda = mu),
a0_phi = 0.9999, with and without the synchronization every 50 steps.  It
records the displacement of the top-left corner P and (hole) of the point Q
at (-0.175 L, 0.025 L) from the hole's centre, the consistency error map at
t = 0.002 L / c_s and, for tension, the late-time mean displacement of P
against the static plane-strain solution.  The paper's FEM curves are not
available, so the comparison with them stays qualitative.

disc: the first axisymmetric (breathing) mode of a traction-free elastic
disc in plane strain.  Its radial displacement is u_r = J1(k r) with k R = x
the first root of (lambda + 2 mu) x J0(x) - 2 mu J1(x) = 0 (sigma_rr = 0 at
r = R), and it oscillates at omega = x c_d / R.  The disc (a bounding circle
of radius R on the lattice) starts in that shape at rest; the amplitude of
the shape in u(t) is fitted to a cos(omega t + phi) + b over one period
(longer runs on curved boundaries grow a grid-scale instability).  The
relative error of omega compares the mask-rule boundary cells with the
exact-geometry cells of lbm_exact_cells (Sec. 3.1).

Prints one JSON line per run.  Inputs are synthetic and deterministic.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import inputs as I
from . import lbm


def breathing_root(lam, mu):
    from scipy.optimize import brentq
    from scipy.special import j0, j1
    f = lambda x: (lam + 2 * mu) * x * j0(x) - 2 * mu * j1(x)
    xs = np.linspace(0.1, 4.0, 400)
    v = f(xs)
    k = int(np.nonzero(v[:-1] * v[1:] < 0)[0][0])
    return brentq(f, xs[k], xs[k + 1], xtol=1e-15)


def disc_case(R, nu=0.3, a0_phi=0.9999, sync_every=50, amp=1e-4, cells="mask"):
    from scipy.special import j1
    n = 2 * R + 6
    c = (n - 1) / 2.0
    shapes = [(c, c, float(R), float(R), 0.0, I.SHAPE_BOUND)]
    mask = I.shape_mask(n, n, shapes)
    lam = I.lame_lambda(nu)
    x1 = breathing_root(lam, 1.0)
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    r = np.hypot(x - c, y - c)
    ur = amp * j1(x1 * r / R)
    with np.errstate(invalid="ignore", divide="ignore"):
        cx, cy = np.where(r > 0, (x - c) / r, 0.0), np.where(r > 0, (y - c) / r, 0.0)
    u0 = np.stack([ur * cx, ur * cy]) * mask[None]
    xy = I.boundary_nodes(mask)
    cell = None
    if cells == "exact":
        cell, _ = lbm.exact_cells(n, n, shapes, xy)
    bcs = [I.BoundaryData(xy, np.zeros(len(xy), np.uint8), np.zeros((len(xy), 2)), cell=cell)]
    case = I.Case(name=f"disc{R}", nx=n, ny=n, mask=mask, periodic=(False, False), lam=lam, mu=1.0,
                  rho=1.0, dh=1.0, dt=I.time_step(nu, a0_phi), sync_every=sync_every, u0=u0,
                  v0=np.zeros_like(u0), e0=None, w0=None, bcs=bcs, nu=nu, a0_phi=a0_phi,
                  shapes=shapes)
    omega = x1 * np.sqrt(lam + 2.0) / R
    return case, omega


def disc_mode(R, cells, storage="f64", periods=1.0, samples=200, **kw):
    from scipy.optimize import curve_fit
    case, omega = disc_case(R, cells=cells, **kw)
    T = 2 * np.pi / omega
    total = int(round(periods * T / case.dt))
    every = max(1, total // samples)
    u0 = case.u0
    norm = float(np.sum(u0 * u0))
    ts, amps = [0.0], [1.0]
    t0 = time.perf_counter()
    with lbm.context_for(case, storage) as ctx:
        done = 0
        while done < total:
            ctx.step(every)
            done += every
            u = ctx.fields(0, want=("u",))["u"]
            ts.append(done * case.dt)
            amps.append(float(np.sum(u * u0)) / norm)
    wall = time.perf_counter() - t0
    ts, amps = np.array(ts), np.array(amps)
    f = lambda t, a, w, ph, b: a * np.cos(w * t + ph) + b
    p, _ = curve_fit(f, ts, amps, p0=(1.0, omega, 0.0, 0.0))
    resid = float(np.sqrt(np.mean((f(ts, *p) - amps) ** 2)))
    return {"experiment": "disc_breathing_mode", "R": R, "cells": cells, "storage": storage,
            "nodes": case.in_body_nodes(), "steps": done, "dt": case.dt, "omega_exact": omega,
            "omega_fit": float(p[1]), "rel_error": float(p[1] / omega - 1.0),
            "fit_amplitude": float(p[0]), "fit_rms_residual": resid, "wall_s": wall}


def paper_case(kind, L, sync_every, cells="mask", t_end=2.0, cell_fn=None):
    """One of the Sec. 4 examples on an (L+1)^2 lattice (dh = 1, mu = 1,
    rho = 1, c_s = 1).  kind: "tension", "shear" or "hole".  cells: "mask"
    or "exact" (the hole's rim; cell_fn(nx, ny, shapes, xy) -> cell table,
    default lbm_exact_cells).  Times are in units of L / c_s."""
    nu = 0.25  # lambda = mu: c_s / c_d = 1 / sqrt(3)
    n = L + 1
    lam = I.lame_lambda(nu)
    dt = I.time_step(nu, 0.9999)
    shapes = []
    if kind == "hole":
        c = L / 2.0
        shapes = [(c, c, 0.133 * L, 0.133 * L, 0.0, I.SHAPE_HOLE)]
    mask = I.shape_mask(n, n, shapes) if shapes else None
    m = mask if mask is not None else np.ones((n, n), np.uint8)
    top = I.edge_nodes(n, n, I.TOP)
    bot = I.edge_nodes(n, n, I.BOTTOM)
    # cell width along the edge (mask rule: half at the corners)
    wx = np.where((top[:, 0] == 0) | (top[:, 0] == n - 1), 0.5, 1.0)
    T = t_end * L  # c_s = 1
    bcs = []
    if kind in ("tension", "hole"):
        knots = np.array([[0.0, 0.0], [float(L), 0.005], [max(T, float(L)) + 1.0, 0.005]])
        bcs.append(I.BoundaryData(top, np.zeros(len(top), np.uint8), np.stack([0 * wx, wx], 1),
                                  knots=knots))
        bcs.append(I.BoundaryData(bot, np.zeros(len(bot), np.uint8), np.stack([0 * wx, -wx], 1),
                                  knots=knots))
    else:
        bcs.append(I.BoundaryData(bot, np.full(len(bot), I.DIRICHLET, np.uint8),
                                  np.zeros((len(bot), 2))))
        inner = top[(top[:, 0] > 0) & (top[:, 0] < n - 1)]
        knots = np.array([[0.0, 0.0], [T + 1.0, 0.005 * (T + 1.0) / L]])
        bcs.append(I.BoundaryData(inner, np.zeros(len(inner), np.uint8),
                                  np.stack([np.ones(len(inner)), np.zeros(len(inner))], 1),
                                  knots=knots))
        corners = np.array([[0, n - 1], [n - 1, n - 1]], np.int32)
        bcs.append(I.BoundaryData(corners, np.zeros(2, np.uint8), np.array([[0.5, 0.0], [0.5, 0.0]]),
                                  knots=knots))
    if kind == "hole" and cells == "exact":
        xy = I.boundary_nodes(m)
        rim = xy[(xy[:, 0] > 0) & (xy[:, 0] < n - 1) & (xy[:, 1] > 0) & (xy[:, 1] < n - 1)]
        cell = (cell_fn or (lambda *a: lbm.exact_cells(*a)[0]))(n, n, shapes, rim)
        bcs.append(I.BoundaryData(rim, np.zeros(len(rim), np.uint8), np.zeros((len(rim), 2)), cell=cell))
    return I.Case(name=f"{kind}{L}", nx=n, ny=n, mask=mask, periodic=(False, False), lam=lam, mu=1.0,
                  rho=1.0, dh=1.0, dt=dt, sync_every=sync_every, u0=None, v0=None, e0=None,
                  w0=None, bcs=bcs, steps=int(round(T / dt)), nu=nu, a0_phi=0.9999, shapes=shapes)


def static_tension_corner(nu, sigma0=0.005, mu=1.0):
    """Plane-strain uniaxial stress sigma_yy = sigma0 on a free square: the
    displacement of the top-left corner relative to the centre, per unit L."""
    E = 2 * mu * (1 + nu)
    eyy = (1 - nu * nu) * sigma0 / E
    exx = -nu * (1 + nu) * sigma0 / E
    return (-0.5 * exx, 0.5 * eyy)


def paper_run(kind, L, sync_every, cells="mask", storage="f64", samples=200, t_end=2.0):
    case = paper_case(kind, L, sync_every, cells=cells, t_end=t_end)
    n = case.nx
    P = (0, n - 1)
    Q = None
    if kind == "hole":
        c = L / 2.0
        Q = (int(round(c - 0.175 * L)), int(round(c + 0.025 * L)))
    total = case.steps
    every = max(1, total // samples)
    err_step = max(1, int(round(0.002 * L / case.dt)))
    t0 = time.perf_counter()
    ts, uP, uQ = [0.0], [(0.0, 0.0)], [(0.0, 0.0)]
    blew = None
    cons = None
    with lbm.context_for(case, storage) as ctx:
        ctx.step(err_step)
        err = ctx.consistency_error(0)
        k = np.unravel_index(int(np.argmax(err)), err.shape)
        cls = "boundary" if k[0] in (0, n - 1) or k[1] in (0, n - 1) else (
            "second row" if k[0] in (1, n - 2) or k[1] in (1, n - 2) else "interior")
        rows = np.sort(np.unique(np.nonzero(err > 0.5 * err.max())[0]))
        cons = {"t": err_step * case.dt / L, "max": float(err.max()), "argmax_ij": [int(k[1]), int(k[0])],
                "argmax_class": cls, "rows_above_half_max": rows.tolist()[:12]}
        done = err_step
        try:
            while done < total:
                m = min(every, total - done)
                ctx.step(m)
                done += m
                u = ctx.fields(0, want=("u",))["u"]
                ts.append(done * case.dt / L)
                uP.append((u[0, P[1], P[0]] / L, u[1, P[1], P[0]] / L))
                if Q:
                    uQ.append((u[0, Q[1], Q[0]] / L, u[1, Q[1], Q[0]] / L))
                if not np.isfinite(u).all() or np.abs(u).max() > 10.0 * L:
                    blew = done * case.dt / L
                    break
        except lbm.LbmError:
            blew = done * case.dt / L
    wall = time.perf_counter() - t0
    ts, uP = np.array(ts), np.array(uP)
    out = {"experiment": f"paper_{kind}", "L": L, "sync_every": sync_every, "cells": cells,
           "storage": storage, "nodes": case.in_body_nodes(), "steps": done, "dt": case.dt,
           "t_end": float(ts[-1]), "blew_up_at": blew, "cons_err": cons, "wall_s": wall,
           "t": np.round(ts, 4).tolist(), "uP": np.round(uP, 9).tolist()}
    if Q:
        out["uQ"] = np.round(np.array(uQ), 9).tolist()
    late = (ts >= 1.0) & (ts <= 2.0)
    if kind in ("tension", "hole") and late.sum() > 10:
        out["uP_mean_t1_2"] = uP[late].mean(0).tolist()
        # high-frequency content: rms of the second difference of u_y(P)
        d2 = np.diff(uP[late, 1], 2)
        out["uyP_rough_t1_2"] = float(np.sqrt(np.mean(d2 * d2)))
        if kind == "tension":
            out["static_uP"] = static_tension_corner(case.nu)
    return out


def plane_wave_case(n, a0_phi, k=1, amp=1e-3, nu=0.25, periods=1.0):
    """Periodic n x n square with the dilatational plane wave
    u = (A sin(2 pi k x / n) cos(c_d kappa t), 0) at rest at t = 0 (fields
    from the initial u by the method's finite differences).  Returns the
    case and the exact u(t) as a function."""
    lam = I.lame_lambda(nu)
    cd = np.sqrt(lam + 2.0)
    kappa = 2 * np.pi * k / n
    dt = I.time_step(nu, a0_phi)
    T = 2 * np.pi / (cd * kappa)
    steps = int(round(periods * T / dt))
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    u0 = np.stack([amp * np.sin(kappa * x), 0 * x])
    case = I.Case(name=f"wave{n}", nx=n, ny=n, mask=None, periodic=(True, True), lam=lam, mu=1.0,
                  rho=1.0, dh=1.0, dt=dt, sync_every=0, u0=u0, v0=np.zeros_like(u0), e0=None,
                  w0=None, bcs=[], steps=steps, nu=nu, a0_phi=a0_phi)
    exact = lambda t: np.stack([amp * np.sin(kappa * x) * np.cos(cd * kappa * t), 0 * x])
    return case, exact


def orders(sizes=(16, 32, 64, 128), a0s=(0.0, 0.5, 0.99), storage="f64", integrators=(0, 1)):
    """Convergence of the interior scheme on a periodic plane wave: the
    relative max error of u after one period against the exact solution, at
    a fixed a0_phi (so dt scales with dh), for growing lattices (the wave is
    the same on every lattice: its wavelength is the plate size), with the
    paper's displacement update (integrator 0) and the central difference
    (integrator 1)."""
    out = []
    for integ in integrators:
        out += _orders(sizes, a0s, storage, integ)
    return out


def _orders(sizes, a0s, storage, integ):
    out = []
    for a0 in a0s:
        errs = []
        for n in sizes:
            case, exact = plane_wave_case(n, a0)
            case.integrator = integ
            with lbm.context_for(case, storage) as ctx:
                ctx.step(case.steps)
                u = ctx.fields(0, want=("u",))["u"]
            ue = exact(case.steps * case.dt)
            errs.append(float(np.abs(u - ue).max() / np.abs(ue).max()))
        rates = [float(np.log2(errs[i] / errs[i + 1])) for i in range(len(errs) - 1)]
        out.append({"experiment": "plane_wave_orders", "integrator": integ, "a0_phi": a0,
                    "sizes": list(sizes), "rel_max_err_u": errs, "observed_orders": rates})
    return out


def stability_sweep(L=64, a0s=(0.9999, 0.999, 0.99, 0.9), syncs=(0, 10, 50, 200), t_end=2.0,
                    storage="f64", readings=(0, 0)):
    """Blow-up time (units of L / c_s; None = stable to t_end) of the
    tension example for each (a0_phi, synchronization period), with the
    given readings of eqs. correction-f / LBE_mod ((0, 0) = R1, M1)."""
    out = []
    for a0 in a0s:
        for l in syncs:
            case = paper_case("tension", L, l, t_end=t_end)
            case.readings = tuple(readings)
            nu = case.nu
            case.dt = I.time_step(nu, a0)
            case.a0_phi = a0
            case.steps = int(round(t_end * L / case.dt))
            every = max(1, case.steps // 40)
            blew = None
            with lbm.context_for(case, storage) as ctx:
                done = 0
                try:
                    while done < case.steps:
                        m = min(every, case.steps - done)
                        ctx.step(m)
                        done += m
                        u = ctx.fields(0, want=("u",))["u"]
                        if not np.isfinite(u).all() or np.abs(u).max() > 10.0 * L:
                            blew = done * case.dt / L
                            break
                except lbm.LbmError:
                    blew = done * case.dt / L
            out.append({"experiment": "stability_tension", "L": L, "a0_phi": a0, "sync_every": l,
                        "readings": "R%dM%d" % (readings[0] + 1, readings[1] + 1),
                        "dt": case.dt, "steps": done, "blew_up_at": blew})
            print(json.dumps(out[-1]), file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("experiment", choices=["disc", "paper", "orders", "stability"])
    ap.add_argument("--L", type=int, default=128)
    ap.add_argument("--t-end", type=float, default=2.0)
    ap.add_argument("--radii", type=int, nargs="+", default=[8, 12, 16, 24, 32])
    ap.add_argument("--periods", type=float, default=1.0)
    ap.add_argument("--storage", default="f64")
    ap.add_argument("--readings", default="R1M1", choices=["R1M1", "R2M1", "R1M2", "R2M2", "all"],
                    help="stability: readings of eqs. correction-f (R1 own flux, R2 streamed-in "
                         "flux) and LBE_mod (M1 own moments, M2 old state's equilibrium)")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    if args.experiment == "orders":
        for r in orders(storage=args.storage):
            print(json.dumps(r), flush=True)
        return
    if args.experiment == "stability":
        names = ["R1M1", "R2M1", "R1M2", "R2M2"] if args.readings == "all" else [args.readings]
        for name in names:
            rd = (int(name[1]) - 1, int(name[3]) - 1)
            for r in stability_sweep(L=args.L, storage=args.storage, t_end=args.t_end, readings=rd):
                print(json.dumps(r), flush=True)
        return
    if args.experiment == "disc":
        for R in args.radii:
            for cells in ("mask", "exact"):
                print(f"disc R={R} cells={cells}", file=sys.stderr, flush=True)
                print(json.dumps(disc_mode(R, cells, storage=args.storage, periods=args.periods)),
                      flush=True)
        return
    runs = [("tension", 0, "mask"), ("tension", 50, "mask"), ("shear", 50, "mask"), ("shear", 0, "mask"),
            ("hole", 50, "mask"), ("hole", 0, "mask"), ("hole", 50, "exact"), ("hole", 0, "exact")]
    for kind, l, cells in runs:
        print(f"paper {kind} L={args.L} sync={l} cells={cells}", file=sys.stderr, flush=True)
        print(json.dumps(paper_run(kind, args.L, l, cells=cells, storage=args.storage,
                                   t_end=args.t_end)), flush=True)


if __name__ == "__main__":
    main()
