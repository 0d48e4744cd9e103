"""Physics checks of the GPU library beyond parity with the oracle.

    python -m paper_2301_00228_amd.experiments disc --radii 16 32 64

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("experiment", choices=["disc"])
    ap.add_argument("--radii", type=int, nargs="+", default=[8, 12, 16, 24, 32])
    ap.add_argument("--periods", type=float, default=1.0)
    ap.add_argument("--storage", default="f64")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    for R in args.radii:
        for cells in ("mask", "exact"):
            print(f"disc R={R} cells={cells}", file=sys.stderr, flush=True)
            print(json.dumps(disc_mode(R, cells, storage=args.storage, periods=args.periods)),
                  flush=True)


if __name__ == "__main__":
    main()
