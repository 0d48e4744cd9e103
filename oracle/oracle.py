"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

Test infrastructure only (tests, smoke check, CPU-baseline timing).  Arrays
are numpy, row-major with x fastest: scalar fields have shape (ny, nx), vector
fields (2, ny, nx) with the x component first.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

ERRORS = {0: "OK", -1: "INVAL", -2: "UNSTABLE_DT", -3: "NOMEM", -6: "STATE"}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code} ({ERRORS.get(code, '?')})")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        up = C.POINTER(C.c_uint8)
        ip = C.POINTER(C.c_int32)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, up, C.c_int, C.c_int, C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.c_int, dp, dp, dp, dp,
                                 C.POINTER(C.c_int)]
        L.orc_set_integrator.restype = C.c_int
        L.orc_set_integrator.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_readings.restype = C.c_int
        L.orc_set_readings.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_set_bc.restype = C.c_int
        L.orc_set_bc.argtypes = [C.c_void_p, C.c_int, ip, up, dp, dp, C.c_int, dp]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_fields.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_pops.argtypes = [C.c_void_p, dp]
        L.orc_set_pops.argtypes = [C.c_void_p, dp]
        L.orc_last_accel.argtypes = [C.c_void_p, dp]
        L.orc_cons_err.argtypes = [C.c_void_p, dp]
        L.orc_classes.argtypes = [C.c_void_p, up]
        L.orc_params.argtypes = [C.c_void_p, dp]
        L.orc_step_count.restype = C.c_int64
        L.orc_step_count.argtypes = [C.c_void_p]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_threads.restype = C.c_int
        L.orc_threads.argtypes = []
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


class OraclePlate:
    """One plate advanced by the oracle."""

    def __init__(self, nx, ny, mask=None, periodic=(False, False), lam=1.0, mu=1.0, rho=1.0,
                 dh=1.0, dt=0.5, sync_every=0, u0=None, v0=None, e0=None, w0=None, integrator=0,
                 readings=(0, 0)):
        L = lib()
        self.nx, self.ny = int(nx), int(ny)
        shp, vshp = (self.ny, self.nx), (2, self.ny, self.nx)
        self._keep = [
            None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(shp),
            _f64(u0, vshp), _f64(v0, vshp), _f64(e0, shp), _f64(w0, shp)]
        m, u0a, v0a, e0a, w0a = self._keep
        err = C.c_int(0)
        h = L.orc_create(self.nx, self.ny,
                         None if m is None else m.ctypes.data_as(C.POINTER(C.c_uint8)),
                         int(periodic[0]), int(periodic[1]), float(lam), float(mu), float(rho),
                         float(dh), float(dt), int(sync_every), _dp(u0a), _dp(v0a), _dp(e0a),
                         _dp(w0a), C.byref(err))
        if not h:
            raise OracleError(err.value, "orc_create")
        self._h = C.c_void_p(h)
        if integrator:
            rc = L.orc_set_integrator(self._h, int(integrator))
            if rc:
                raise OracleError(rc, "orc_set_integrator")
        if tuple(readings) != (0, 0):
            # (flux reading of eq. correction-f: 0 R1 / 1 R2, equilibrium of
            # eq. LBE_mod: 0 M1 / 1 M2)
            rc = L.orc_set_readings(self._h, int(readings[0]), int(readings[1]))
            if rc:
                raise OracleError(rc, "orc_set_readings")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    def set_bc(self, xy, kind, val, cell=None, knots=None):
        xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
        n = xy.shape[0]
        kind = np.ascontiguousarray(kind, dtype=np.uint8).reshape(n)
        val = np.ascontiguousarray(val, dtype=np.float64).reshape(n, 2)
        cell = None if cell is None else np.ascontiguousarray(cell, dtype=np.float64).reshape(n, 5)
        kn = None if knots is None else np.ascontiguousarray(knots, dtype=np.float64).reshape(-1, 2)
        rc = lib().orc_set_bc(self._h, n, xy.ctypes.data_as(C.POINTER(C.c_int32)),
                              kind.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(val), _dp(cell),
                              0 if kn is None else kn.shape[0], _dp(kn))
        if rc:
            raise OracleError(rc, "orc_set_bc")

    def step(self, n=1):
        rc = lib().orc_step(self._h, int(n))
        if rc:
            raise OracleError(rc, "orc_step")

    def fields(self):
        shp = (self.ny, self.nx)
        e, w = np.zeros(shp), np.zeros(shp)
        u, v = np.zeros((2,) + shp), np.zeros((2,) + shp)
        lib().orc_fields(self._h, _dp(e), _dp(w), _dp(u), _dp(v))
        return {"e": e, "omega": w, "u": u, "v": v}

    def pops(self):
        f = np.zeros((2, 5, self.ny, self.nx))
        lib().orc_pops(self._h, _dp(f))
        return f

    def set_pops(self, f):
        f = _f64(f, (2, 5, self.ny, self.nx))
        lib().orc_set_pops(self._h, _dp(f))

    def last_accel(self):
        a = np.zeros((2, self.ny, self.nx))
        lib().orc_last_accel(self._h, _dp(a))
        return a

    def cons_err(self):
        e = np.zeros((self.ny, self.nx))
        lib().orc_cons_err(self._h, _dp(e))
        return e

    def classes(self):
        c = np.zeros((self.ny, self.nx), dtype=np.uint8)
        lib().orc_classes(self._h, c.ctypes.data_as(C.POINTER(C.c_uint8)))
        return c

    def params(self):
        o = np.zeros(7)
        lib().orc_params(self._h, _dp(o))
        return dict(zip(["a_phi", "a0_phi", "a_psi", "a0_psi", "c_d", "c_s", "c"], o.tolist()))

    @property
    def steps_done(self):
        return int(lib().orc_step_count(self._h))


def threads():
    """OpenMP threads used by the oracle's loops."""
    return int(lib().orc_threads())


def set_threads(n):
    """Set the OpenMP threads of the oracle's loops."""
    lib().orc_set_threads(int(n))


def run_case(case, steps=None):
    """Run a seeded input case (see ``paper_2301_00228_amd.inputs``) on the
    oracle and return its fields and the plate."""
    p = OraclePlate(case.nx, case.ny, mask=case.mask, periodic=case.periodic, lam=case.lam,
                    mu=case.mu, rho=case.rho, dh=case.dh, dt=case.dt, sync_every=case.sync_every,
                    u0=case.u0, v0=case.v0, e0=case.e0, w0=case.w0,
                    integrator=getattr(case, "integrator", 0),
                    readings=getattr(case, "readings", (0, 0)))
    for bc in case.bcs:
        p.set_bc(bc.xy, bc.kind, bc.val, cell=bc.cell, knots=bc.knots)
    p.step(case.steps if steps is None else steps)
    return p.fields(), p
