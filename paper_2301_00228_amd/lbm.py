"""Python binding of the C ABI in ``include/lbm.h`` (ctypes; marshalling only).

Every step of the method runs in the HIP library ``liblbm.so``; this module
only converts arguments.  PyTorch, when present, supplies the HIP stream
(and optionally the device allocator).  If the library has not been built
the import of this module succeeds but creating a context raises
``LbmError`` -- there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

OK, E_INVAL, E_UNSTABLE_DT, E_NOMEM, E_DEVICE, E_NONFINITE, E_STATE = 0, -1, -2, -3, -4, -5, -6
STATUS = {0: "OK", -1: "INVAL", -2: "UNSTABLE_DT", -3: "NOMEM", -4: "DEVICE", -5: "NONFINITE",
          -6: "STATE"}

STORE_F64, STORE_F32, STORE_F32DEV, STORE_F16DEV, STORE_BF16DEV = 0, 1, 2, 3, 4
STORAGES = {"f64": 0, "f32": 1, "f32dev": 2, "f16dev": 3, "bf16dev": 4}
BC_NEUMANN, BC_DIRICHLET = 0, 1
READ_FLUX_STREAMED, READ_EQ_OLD = 1, 2

# Every entry point declared in include/lbm.h.
EXPORTS = ["lbm_create", "lbm_set_bc", "lbm_step", "lbm_fields", "lbm_fields_device", "lbm_info",
           "lbm_set_tiling", "lbm_autotune", "lbm_profile", "lbm_use_graphs", "lbm_use_overlap", "lbm_destroy",
           "lbm_last_error", "lbm_version", "lbm_exact_cells", "lbm_consistency_error",
           "lbm_fields_noalloc", "lbm_prepare_steps", "lbm_copy_rate",
           "lbm_layout_copy_rate"]
SHAPE_HOLE, SHAPE_BOUND = 0, 1


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class lbm_plate(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("mask", C.POINTER(C.c_uint8)),
                ("periodic_x", C.c_uint8), ("periodic_y", C.c_uint8),
                ("lam", C.c_double), ("mu", C.c_double), ("rho_m", C.c_double),
                ("dh", C.c_double), ("dt", C.c_double), ("sync_every", C.c_int32),
                ("u0", C.POINTER(C.c_double)), ("v0", C.POINTER(C.c_double)),
                ("e0", C.POINTER(C.c_double)), ("w0", C.POINTER(C.c_double)),
                ("integrator", C.c_int32), ("readings", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class lbm_alloc(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class lbm_info_t(C.Structure):
    _fields_ = [("nodes_in_body", C.c_int64), ("nodes_allocated", C.c_int64),
                ("boundary_nodes", C.c_int64), ("second_row_nodes", C.c_int64),
                ("nodes_two_step", C.c_int64),
                ("steps_done", C.c_int64), ("device_bytes", C.c_int64),
                ("bytes_per_update", C.c_double), ("n_plates", C.c_int32),
                ("storage", C.c_int32), ("tile_lanes", C.c_int32), ("tile_rows", C.c_int32),
                ("tile_order", C.c_int32), ("tile_edge_rows", C.c_int32),
                ("tile_align", C.c_int32), ("tile_steps", C.c_int32), ("n_tiles", C.c_int32),
                ("tile_edge_cols", C.c_int32), ("nodes_deep", C.c_int64), ("overlap", C.c_int32),
                ("graphs_cached", C.c_int32), ("steps_in_graphs", C.c_int64),
                ("syncs_done", C.c_int64), ("tile_stream_stores", C.c_int32), ("pad", C.c_int32)]


class lbm_tiling(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("rows", C.c_int32), ("order", C.c_int32),
                ("edge_rows", C.c_int32), ("align", C.c_int32), ("steps", C.c_int32),
                ("edge_cols", C.c_int32), ("stream_stores", C.c_int32)]


class lbm_shape(C.Structure):
    _fields_ = [("cx", C.c_double), ("cy", C.c_double), ("a", C.c_double), ("b", C.c_double),
                ("angle", C.c_double), ("kind", C.c_int32), ("pad", C.c_int32)]


_lib = None


def library():
    """Load liblbm.so (raises LbmError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LbmError(E_DEVICE, f"{LIB_PATH} is missing: build the HIP library first "
                                 "(python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip, up = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_uint8)
    L.lbm_create.restype = C.c_int
    L.lbm_create.argtypes = [C.POINTER(lbm_plate), C.c_int32, C.c_int, vp, C.POINTER(lbm_alloc),
                             C.POINTER(vp)]
    L.lbm_set_bc.restype = C.c_int
    L.lbm_set_bc.argtypes = [vp, C.c_int32, C.c_int32, ip, up, dp, dp, C.c_int32, dp]
    L.lbm_step.restype = C.c_int
    L.lbm_step.argtypes = [vp, C.c_int64]
    L.lbm_copy_rate.restype = C.c_int
    L.lbm_copy_rate.argtypes = [C.c_size_t, C.c_int32, dp]
    L.lbm_layout_copy_rate.restype = C.c_int
    L.lbm_layout_copy_rate.argtypes = [C.c_int32, C.c_int64, C.c_int32, dp]
    L.lbm_prepare_steps.restype = C.c_int
    L.lbm_prepare_steps.argtypes = [vp, C.c_int64]
    L.lbm_fields.restype = C.c_int
    L.lbm_fields.argtypes = [vp, C.c_int32, dp, dp, dp, dp]
    L.lbm_fields_noalloc.restype = C.c_int
    L.lbm_fields_noalloc.argtypes = [vp, C.c_int32, dp, dp, dp, dp]
    L.lbm_fields_device.restype = C.c_int
    L.lbm_fields_device.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    L.lbm_info.restype = C.c_int
    L.lbm_info.argtypes = [vp, C.POINTER(lbm_info_t)]
    L.lbm_set_tiling.restype = C.c_int
    L.lbm_set_tiling.argtypes = [vp, C.POINTER(lbm_tiling)]
    L.lbm_autotune.restype = C.c_int
    L.lbm_autotune.argtypes = [vp, C.c_int32, dp]
    L.lbm_profile.restype = C.c_int
    L.lbm_profile.argtypes = [vp, C.c_int64, dp, C.POINTER(C.c_int64)]
    L.lbm_use_graphs.restype = C.c_int
    L.lbm_use_graphs.argtypes = [vp, C.c_int32]
    L.lbm_use_overlap.restype = C.c_int
    L.lbm_use_overlap.argtypes = [vp, C.c_int32]
    L.lbm_destroy.restype = None
    L.lbm_destroy.argtypes = [vp]
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_last_error.argtypes = [vp]
    L.lbm_version.restype = C.c_char_p
    L.lbm_version.argtypes = []
    L.lbm_consistency_error.restype = C.c_int
    L.lbm_consistency_error.argtypes = [vp, C.c_int32, dp]
    L.lbm_exact_cells.restype = C.c_int
    L.lbm_exact_cells.argtypes = [C.c_int32, C.c_int32, C.c_uint8, C.c_uint8, C.c_double, C.c_int32,
                                  C.POINTER(lbm_shape), C.c_int32, ip, dp, dp]
    _lib = L
    return L


def _dptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape, what):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != int(np.prod(shape)):
        raise LbmError(E_INVAL, f"{what}: expected {shape}, got {a.shape}")
    return a.reshape(shape)


def exact_cells(nx, ny, shapes, xy, dh=1.0, periodic=(False, False)):
    """lbm_exact_cells: cell table (n, 5) = V_C, l_E, l_N, l_W, l_S and the
    external normal integrals (n, 2) of nodes xy (n, 2) of an nx x ny lattice
    bounded by ellipses; shapes = [(cx, cy, a, b, angle, kind), ...]."""
    L = library()
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    n = xy.shape[0]
    arr = (lbm_shape * max(len(shapes), 1))()
    for q, (cx, cy, a, b, ang, kind) in enumerate(shapes):
        arr[q] = lbm_shape(cx, cy, a, b, ang, kind, 0)
    cell = np.zeros((n, 5), dtype=np.float64)
    ext = np.zeros((n, 2), dtype=np.float64)
    st = L.lbm_exact_cells(nx, ny, int(periodic[0]), int(periodic[1]), float(dh), len(shapes), arr, n,
                           xy.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(cell), _dptr(ext))
    if st != OK:
        raise LbmError(st, "lbm_exact_cells rejected its arguments")
    return cell, ext


def layout_copy_rate(storage, nodes, reps=10):
    """lbm_layout_copy_rate: GB/s of a copy with the array structure of the
    storage's state over `nodes` nodes."""
    st = STORAGES[storage] if isinstance(storage, str) else int(storage)
    out = C.c_double(0)
    rc = library().lbm_layout_copy_rate(st, int(nodes), int(reps), C.byref(out))
    if rc != OK:
        raise LbmError(rc, library().lbm_last_error(None).decode())
    return out.value


def copy_rate(nbytes=2 << 30, reps=10):
    """lbm_copy_rate: GB/s of a plain device copy of nbytes bytes."""
    out = C.c_double(0)
    rc = library().lbm_copy_rate(int(nbytes), int(reps), C.byref(out))
    if rc != OK:
        raise LbmError(rc, library().lbm_last_error(None).decode())
    return out.value


def default_stream():
    """The current torch HIP stream handle, or 0 (null stream)."""
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return 0


def torch_allocator():
    """An lbm_alloc backed by torch's caching allocator on the current device."""
    import torch

    dev = torch.cuda.current_device()
    live = {}

    @ALLOC_FN
    def _alloc(nbytes, user):
        p = torch.cuda.caching_allocator_alloc(int(nbytes), dev)
        live[p] = nbytes
        return p

    @FREE_FN
    def _free(ptr, user):
        if ptr in live:
            del live[ptr]
            torch.cuda.caching_allocator_delete(ptr)

    a = lbm_alloc(_alloc, _free, None)
    a._keep = (_alloc, _free, live)
    return a


class Context:
    """One lbm_ctx: a batch of plates advanced together."""

    def __init__(self, plates, storage="f64", stream=None, allocator=None):
        L = library()
        st = STORAGES[storage] if isinstance(storage, str) else int(storage)
        n = len(plates)
        arr = (lbm_plate * n)()
        self._keep = []
        self.shapes = []
        for k, p in enumerate(plates):
            nx, ny = int(p["nx"]), int(p["ny"])
            self.shapes.append((nx, ny))
            d = arr[k]
            d.nx, d.ny = nx, ny
            m = p.get("mask")
            if m is not None:
                m = np.ascontiguousarray(m, dtype=np.uint8)
                if m.size != nx * ny:
                    raise LbmError(E_INVAL, "mask size")
                self._keep.append(m)
                d.mask = m.ctypes.data_as(C.POINTER(C.c_uint8))
            per = p.get("periodic", (False, False))
            d.periodic_x, d.periodic_y = int(bool(per[0])), int(bool(per[1]))
            d.lam, d.mu, d.rho_m = float(p["lam"]), float(p["mu"]), float(p["rho"])
            d.dh, d.dt = float(p["dh"]), float(p["dt"])
            d.sync_every = int(p.get("sync_every", 0))
            d.integrator = int(p.get("integrator", 0))
            rd = p.get("readings", (0, 0))
            # (flux reading of eq. correction-f: 0 R1 / 1 R2; equilibrium of
            # eq. LBE_mod: 0 M1 / 1 M2) -> LBM_READ_* bits
            d.readings = int(rd[0]) * READ_FLUX_STREAMED + int(rd[1]) * READ_EQ_OLD
            for name, shape in (("u0", (2, ny, nx)), ("v0", (2, ny, nx)), ("e0", (ny, nx)),
                                ("w0", (ny, nx))):
                a = _f64(p.get(name), shape, name)
                if a is not None:
                    self._keep.append(a)
                    setattr(d, name, _dptr(a))
        self.storage = st
        self.stream = default_stream() if stream is None else int(stream)
        self._alloc = allocator
        h = C.c_void_p()
        rc = L.lbm_create(arr, n, st, C.c_void_p(self.stream),
                          None if allocator is None else C.byref(allocator), C.byref(h))
        if rc != OK:
            raise LbmError(rc, L.lbm_last_error(None).decode())
        self._h = h
        self._keep = []

    def _check(self, rc):
        if rc != OK:
            raise LbmError(rc, library().lbm_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            library().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_bc(self, plate, xy, kind, val, cell=None, knots=None):
        xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
        n = xy.shape[0]
        kind = np.ascontiguousarray(kind, dtype=np.uint8).reshape(n)
        val = np.ascontiguousarray(val, dtype=np.float64).reshape(n, 2)
        cell = None if cell is None else np.ascontiguousarray(cell, np.float64).reshape(n, 5)
        kn = None if knots is None else np.ascontiguousarray(knots, np.float64).reshape(-1, 2)
        self._check(library().lbm_set_bc(
            self._h, int(plate), n, xy.ctypes.data_as(C.POINTER(C.c_int32)),
            kind.ctypes.data_as(C.POINTER(C.c_uint8)), _dptr(val), _dptr(cell),
            0 if kn is None else kn.shape[0], _dptr(kn)))

    def step(self, n=1):
        self._check(library().lbm_step(self._h, int(n)))

    def prepare_steps(self, n):
        """lbm_prepare_steps: capture the graphs step(n) would replay from the
        current state, without running them."""
        self._check(library().lbm_prepare_steps(self._h, int(n)))

    def _shape(self, plate):
        # (the output arrays are sized from the plate: an index outside the
        # context is the library's LBM_E_INVAL, not a Python IndexError)
        if not 0 <= int(plate) < len(self.shapes):
            raise LbmError(E_INVAL, f"bad plate index {plate}")
        return self.shapes[int(plate)]

    def fields(self, plate=0, want=("e", "omega", "u", "v")):
        nx, ny = self._shape(plate)
        e = np.zeros((ny, nx)) if "e" in want else None
        w = np.zeros((ny, nx)) if "omega" in want else None
        u = np.zeros((2, ny, nx)) if "u" in want else None
        v = np.zeros((2, ny, nx)) if "v" in want else None
        self._check(library().lbm_fields(self._h, int(plate), _dptr(e), _dptr(w), _dptr(u),
                                         _dptr(v)))
        out = {"e": e, "omega": w, "u": u, "v": v}
        return {k: out[k] for k in want}

    def fields_noalloc(self, plate=0, want=("e", "omega", "u", "v")):
        """lbm_fields_noalloc: as fields(), staged through the library's fixed
        device area (no device allocation)."""
        nx, ny = self._shape(plate)
        e = np.zeros((ny, nx)) if "e" in want else None
        w = np.zeros((ny, nx)) if "omega" in want else None
        u = np.zeros((2, ny, nx)) if "u" in want else None
        v = np.zeros((2, ny, nx)) if "v" in want else None
        self._check(library().lbm_fields_noalloc(self._h, int(plate), _dptr(e), _dptr(w),
                                                 _dptr(u), _dptr(v)))
        out = {"e": e, "omega": w, "u": u, "v": v}
        return {k: out[k] for k in want}

    def consistency_error(self, plate=0):
        """lbm_consistency_error: (ny, nx) array of the consistency error."""
        nx, ny = self._shape(plate)
        err = np.zeros((ny, nx))
        self._check(library().lbm_consistency_error(self._h, int(plate), _dptr(err)))
        return err

    def fields_device(self, plate, e=None, omega=None, u=None, v=None):
        """Write fields into caller device buffers (torch float64 tensors or raw ints)."""
        def ptr(t):
            if t is None:
                return None
            return C.c_void_p(t if isinstance(t, int) else t.data_ptr())
        self._check(library().lbm_fields_device(self._h, int(plate), ptr(e), ptr(omega), ptr(u),
                                                ptr(v)))

    def info(self):
        i = lbm_info_t()
        self._check(library().lbm_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in lbm_info_t._fields_}

    def set_tiling(self, lanes, rows, order=0, edge_rows=0, align=0, steps=1, edge_cols=0,
                   stream_stores=0):
        t = lbm_tiling(int(lanes), int(rows), int(order), int(edge_rows), int(align), int(steps),
                       int(edge_cols), int(stream_stores))
        self._check(library().lbm_set_tiling(self._h, C.byref(t)))

    def autotune(self, steps=5):
        best = C.c_double(0)
        self._check(library().lbm_autotune(self._h, int(steps), C.byref(best)))
        return best.value

    def profile(self, n):
        """lbm_profile: {kind: (ms, launches)} over n eager steps, kinds
        interior (single-step), boundary, sync, two_step (first launch of a
        pair), deep (deep tiles of overlapped pairs)."""
        ms = (C.c_double * 5)()
        cnt = (C.c_int64 * 5)()
        self._check(library().lbm_profile(self._h, int(n), ms, cnt))
        names = ("interior", "boundary", "sync", "two_step", "deep")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(names)}

    def use_graphs(self, on=True):
        """lbm_use_graphs: captured HIP graphs in step (default on)."""
        self._check(library().lbm_use_graphs(self._h, int(bool(on))))

    def use_overlap(self, on=True):
        """lbm_use_overlap: deep two-step tiles on a second stream beside the
        single-step launches (default on; bitwise the same results)."""
        self._check(library().lbm_use_overlap(self._h, int(bool(on))))


def plate_dict(case):
    """lbm_plate fields of an input case (see ``inputs.Case``)."""
    return {"nx": case.nx, "ny": case.ny, "mask": case.mask, "periodic": case.periodic,
            "lam": case.lam, "mu": case.mu, "rho": case.rho, "dh": case.dh, "dt": case.dt,
            "sync_every": case.sync_every, "u0": case.u0, "v0": case.v0, "e0": case.e0,
            "w0": case.w0, "integrator": getattr(case, "integrator", 0),
            "readings": getattr(case, "readings", (0, 0))}


def context_for(cases, storage="f64", **kw):
    """Create a context for one case or a list of cases and apply their
    boundary data."""
    if not isinstance(cases, (list, tuple)):
        cases = [cases]
    ctx = Context([plate_dict(c) for c in cases], storage=storage, **kw)
    for p, c in enumerate(cases):
        for bc in c.bcs:
            ctx.set_bc(p, bc.xy, bc.kind, bc.val, cell=bc.cell, knots=bc.knots)
    return ctx
