"""Ghost-cell reconstruction on MI355X: Python binding of libgcr.so.

Argument marshalling only -- every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and streams.  The names follow
the C-ABI in ``include/gcr.h`` (``gcr_plan_create`` -> ``Plan(...)``,
``gcr_fill`` -> ``Plan.fill`` ...).  There is no fallback: if the library is
missing, importing works but every call raises ``GcrError``.
"""
from __future__ import annotations

import ctypes
import sys
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libgcr.so")

CGC, CGC_ES, HGC = 0, 1, 2
LAYER2 = 4   # flag or-ed into a scheme: a second ghost layer
DIRICHLET, NEUMANN, MIXED = 0, 1, 2
SPHERE, STAR2D, SHSTAR, AIRFOIL = 0, 1, 2, 3
SCHED_AUTO, SCHED_LEVELS, SCHED_WORKGROUP, SCHED_GRAPH = 0, 1, 2, 3
SYMBOLS = [
    "gcr_plan_create", "gcr_plan_destroy", "gcr_plan_stats", "gcr_plan_level_offsets",
    "gcr_plan_export", "gcr_plan_foot_points", "gcr_plan_fresh_cells", "gcr_plan_update",
    "gcr_set_schedule",
    "gcr_fill", "gcr_surface_ghost", "gcr_surface",
    "gcr_forces", "gcr_forces_noalloc", "gcr_surface_adjoint", "gcr_forces_adjoint", "gcr_fill_adjoint",
    "gcr_batch_create", "gcr_batch_destroy", "gcr_batch_plan", "gcr_batch_counts",
    "gcr_batch_foot_points",
    "gcr_batch_forward", "gcr_batch_status",
    "gcr_set_profiling", "gcr_set_batch_tiling", "gcr_set_batch_shape", "gcr_set_batch_spin",
    "gcr_batch_tiled", "gcr_batch_shape", "gcr_last_build_times", "gcr_forward_times", "gcr_set_wide_layering",
    "gcr_set_wave_residual", "gcr_set_wide_buffer",
    "gcr_status_str", "gcr_version",
]


class GcrError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = _lib.gcr_status_str(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("lo", ctypes.c_double * 3),
                ("h", ctypes.c_double * 3), ("faces", ctypes.c_void_p * 3)]


class _Shape(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("ncoef", ctypes.c_int32),
                ("center", ctypes.c_double * 3), ("r0", ctypes.c_double),
                ("coef", ctypes.POINTER(ctypes.c_double)),
                ("chord", ctypes.c_double), ("thickness", ctypes.c_double),
                ("incidence", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("n_cells", ctypes.c_int64), ("n_interface", ctypes.c_int64),
                ("n_ghost", ctypes.c_int64), ("n_ghost_fluid_side", ctypes.c_int64),
                ("n_units_coupled", ctypes.c_int32), ("max_unit", ctypes.c_int32),
                ("max_level_width", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("max_alpha", ctypes.c_double * 3), ("n_band_segments", ctypes.c_int64)]


_lib = None


def lib():
    """Load libgcr.so (raises GcrError-like OSError if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"libgcr.so not built ({LIB_PATH}); run paper_2609_10165_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        L.gcr_status_str.restype = ctypes.c_char_p
        L.gcr_status_str.argtypes = [ctypes.c_int]
        L.gcr_version.restype = ctypes.c_char_p
        L.gcr_plan_create.argtypes = [P(_Grid), P(_Shape), i32, vp, P(vp)]
        L.gcr_plan_destroy.argtypes = [vp]
        L.gcr_plan_destroy.restype = None
        L.gcr_plan_stats.argtypes = [vp, P(_Stats)]
        L.gcr_plan_level_offsets.argtypes = [vp, vp]
        L.gcr_plan_export.argtypes = [vp] + [vp] * 8 + [vp]
        L.gcr_plan_foot_points.argtypes = [vp, vp, vp, vp]
        L.gcr_plan_fresh_cells.argtypes = [vp, vp, vp, vp, i64, vp]
        L.gcr_plan_update.argtypes = [vp, P(_Shape), vp]
        L.gcr_set_schedule.argtypes = [vp, i32, i32]
        L.gcr_fill.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.gcr_surface_ghost.argtypes = [vp, i32, vp, vp, vp, vp]
        L.gcr_surface.argtypes = [vp, i64, vp, i32, vp, vp, vp, vp, vp]
        L.gcr_forces.argtypes = [vp, i64, vp, vp, vp, vp, vp, dbl, vp, vp]
        L.gcr_forces_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp, dbl, vp, vp]
        L.gcr_surface_adjoint.argtypes = [vp, i64, vp, i32, vp, vp, vp, vp]
        L.gcr_forces_adjoint.argtypes = [vp, i64, vp, vp, vp, dbl, vp, vp, vp, vp]
        L.gcr_fill_adjoint.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.gcr_batch_create.argtypes = [i32, P(_Grid), P(_Shape), vp, vp, P(vp)]
        L.gcr_batch_destroy.argtypes = [vp]
        L.gcr_batch_destroy.restype = None
        L.gcr_batch_plan.argtypes = [vp, i32, P(vp)]
        L.gcr_batch_counts.argtypes = [vp, vp, vp]
        L.gcr_batch_foot_points.argtypes = [vp, vp, vp, vp]
        L.gcr_set_profiling.argtypes = [i32]
        L.gcr_set_batch_tiling.argtypes = [i32]
        L.gcr_set_batch_shape.argtypes = [i32, i32]
        L.gcr_set_batch_spin.argtypes = [i32]
        L.gcr_batch_status.argtypes = [vp]
        L.gcr_batch_tiled.argtypes = [vp, vp]
        L.gcr_batch_shape.argtypes = [vp, vp, vp]
        L.gcr_set_wide_layering.argtypes = [ctypes.c_int64]
        L.gcr_set_wave_residual.argtypes = [i32]
        L.gcr_set_wide_buffer.argtypes = [i32]
        L.gcr_forward_times.argtypes = [vp]
        L.gcr_last_build_times.argtypes = [vp]
        L.gcr_batch_forward.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, dbl,
                                        vp, vp, vp, vp]
        for name in SYMBOLS:
            getattr(L, name)
            if getattr(L, name).restype is ctypes.c_int and name not in ("gcr_status_str",):
                pass
        _lib = L
    return _lib


def _check(code: int, what: str):
    if code != 0:
        raise GcrError(code, what)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t: Optional[torch.Tensor], dtype=torch.float64) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor, got {t.dtype} "
                         f"on {t.device} (contiguous={t.is_contiguous()})")
    return t.data_ptr()


def _ptr_array(ts, dtype=torch.float64):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = _dptr(t, dtype)
    return arr


def make_grid(grid) -> _Grid:
    """The ctypes grid.  A stretched axis (grid.faces[a] not None) passes its
    n + 1 faces; the arrays are kept alive on the returned object."""
    import numpy as np
    g = _Grid()
    g.dim = int(grid.dim)
    faces = getattr(grid, "faces", None)
    g._keep = []
    for i in range(3):
        g.n[i] = int(grid.n[i]) if i < grid.dim else 1
        g.lo[i] = float(grid.lo[i]) if i < grid.dim else 0.0
        g.h[i] = float(grid.h[i]) if i < grid.dim else 1.0
        g.faces[i] = None
        if faces is not None and i < grid.dim and faces[i] is not None:
            f = np.ascontiguousarray(faces[i], dtype=np.float64)
            g._keep.append(f)
            g.faces[i] = f.ctypes.data
    return g


def make_shape(shape):
    """Returns the ctypes shape and the coefficient buffer it points into."""
    s = _Shape()
    s.kind = int(shape.kind)
    coef = [float(v) for v in getattr(shape, "coef", [])]
    buf = (ctypes.c_double * max(1, len(coef)))(*coef) if coef else None
    s.ncoef = int(getattr(shape, "ncoef", 0))
    for i in range(3):
        s.center[i] = float(shape.center[i]) if i < len(shape.center) else 0.0
    s.r0 = float(getattr(shape, "r0", 0.0))
    s.coef = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double)) if buf is not None else None
    s.chord = float(getattr(shape, "chord", 1.0))
    s.thickness = float(getattr(shape, "thick", getattr(shape, "thickness", 0.12)))
    s.incidence = float(getattr(shape, "incidence", 0.0))
    return s, buf


class Plan:
    """gcr_plan_create: ghost tags, levels and geometry of one grid + body."""

    def __init__(self, grid, shape, scheme: int, stream=None, _handle=None, _owner=None):
        L = lib()
        self._owner = _owner
        if _handle is not None:
            self._h = _handle
        else:
            g = make_grid(grid)
            s, keep = make_shape(shape)
            h = ctypes.c_void_p()
            _check(L.gcr_plan_create(ctypes.byref(g), ctypes.byref(s), int(scheme),
                                     _stream(stream), ctypes.byref(h)), "gcr_plan_create")
            self._h = h
        st = _Stats()
        _check(L.gcr_plan_stats(self._h, ctypes.byref(st)), "gcr_plan_stats")
        self._sizes(st)

    def _sizes(self, st):
        self.dim = st.dim
        self.n_cells = st.n_cells
        self.n_ghost = st.n_ghost
        self.n_levels = st.n_levels
        self.n_interface = st.n_interface

    def update(self, shape, stream=None):
        """gcr_plan_update: the plan re-made in place for the body `shape`
        (same grid and scheme), classifying again only the chunks the move
        can change."""
        s, keep = make_shape(shape)
        _check(lib().gcr_plan_update(self._h, ctypes.byref(s), _stream(stream)), "gcr_plan_update")
        st = _Stats()
        _check(lib().gcr_plan_stats(self._h, ctypes.byref(st)), "gcr_plan_stats")
        self._sizes(st)
        return self

    def __del__(self, _finalizing=sys.is_finalizing):
        h = getattr(self, "_h", None)
        # at interpreter exit the HIP runtime may already be torn down: the
        # process is ending, so the plan's memory is left to it
        if h is not None and self._owner is None and _lib is not None and not _finalizing():
            _lib.gcr_plan_destroy(h)
        self._h = None

    def stats(self) -> dict:
        st = _Stats()
        _check(lib().gcr_plan_stats(self._h, ctypes.byref(st)), "gcr_plan_stats")
        return {f: (list(getattr(st, f))[: st.dim] if f == "max_alpha" else getattr(st, f))
                for f, _ in _Stats._fields_}

    def level_offsets(self):
        buf = (ctypes.c_int32 * (self.n_levels + 1))()
        _check(lib().gcr_plan_level_offsets(self._h, buf), "gcr_plan_level_offsets")
        return list(buf)

    def set_schedule(self, schedule: int):
        _check(lib().gcr_set_schedule(self._h, int(schedule), 0), "gcr_set_schedule")

    EXPORTS = ("tags", "cell", "level", "delta", "normal", "psi", "r", "unit")

    def export(self, which: Sequence[str] = EXPORTS, stream=None) -> dict:
        """Device copies of the plan arrays named in `which`."""
        dev = torch.device("cuda")
        ng, d = self.n_ghost, self.dim
        shapes = dict(tags=(self.n_cells, torch.int8), cell=(ng, torch.int32),
                      level=(ng, torch.int32), delta=((d, ng), torch.float64),
                      normal=((d, ng), torch.float64), psi=(ng, torch.float64),
                      r=((d, ng), torch.int32), unit=(ng, torch.int32))
        out = {}
        for k in which:
            if k not in shapes:
                raise KeyError(f"unknown plan array {k!r}")
            shp, dt = shapes[k]
            out[k] = torch.empty(shp, dtype=dt, device=dev)
        ptr = [_dptr(out.get(k), shapes[k][1]) for k in self.EXPORTS]
        _check(lib().gcr_plan_export(self._h, *ptr, _stream(stream)), "gcr_plan_export")
        return out

    def foot_points(self, stream=None):
        """(S, normal), each f64 [dim][n_ghost]: where boundary data is due."""
        dev = torch.device("cuda")
        S = torch.empty((self.dim, self.n_ghost), dtype=torch.float64, device=dev)
        n = torch.empty((self.dim, self.n_ghost), dtype=torch.float64, device=dev)
        _check(lib().gcr_plan_foot_points(self._h, _dptr(S), _dptr(n), _stream(stream)),
               "gcr_plan_foot_points")
        return S, n

    def fresh_cells(self, after: "Plan", cap: Optional[int] = None, stream=None):
        """gcr_plan_fresh_cells: cells exposed when this plan's body moves to
        `after`'s (same grid).  Returns (device int32 list of the first `cap`
        fresh cells, ascending; device int64 counts [fresh, uncovered]); cap
        None: up to every interface cell of `after`."""
        dev = torch.device("cuda")
        if cap is None:
            cap = max(1, self.n_interface + after.n_interface)
        counts = torch.empty(2, dtype=torch.int64, device=dev)
        lst = torch.empty(cap, dtype=torch.int32, device=dev)
        _check(lib().gcr_plan_fresh_cells(self._h, after._h, counts.data_ptr(), lst.data_ptr(),
                                          int(cap), _stream(stream)), "gcr_plan_fresh_cells")
        return lst, counts

    def fill(self, fields: Sequence[torch.Tensor], bc_kind: Sequence[int],
             bc_val: Sequence[torch.Tensor], bc_type: Optional[Sequence] = None, stream=None):
        nf = len(fields)
        kinds = (ctypes.c_int32 * nf)(*[int(k) for k in bc_kind])
        bt = None
        if bc_type is not None:
            bt = (ctypes.c_void_p * nf)()
            for i, t in enumerate(bc_type):
                bt[i] = _dptr(t, torch.uint8) if t is not None else None
        _check(lib().gcr_fill(self._h, nf, _ptr_array(fields), kinds, bt, _ptr_array(bc_val),
                              _stream(stream)), "gcr_fill")

    def surface_ghost(self, fields: Sequence[torch.Tensor], stream=None):
        nf = len(fields)
        dev = fields[0].device
        val = torch.empty((nf, self.n_ghost), dtype=torch.float64, device=dev)
        grad = torch.empty((nf, self.dim, self.n_ghost), dtype=torch.float64, device=dev)
        _check(lib().gcr_surface_ghost(self._h, nf, _ptr_array(fields), _dptr(val), _dptr(grad),
                                       _stream(stream)), "gcr_surface_ghost")
        return val, grad

    def surface(self, xq: torch.Tensor, fields: Sequence[torch.Tensor], stream=None):
        nf = len(fields)
        nq = xq.shape[1]
        dev = xq.device
        val = torch.empty((nf, nq), dtype=torch.float64, device=dev)
        grad = torch.empty((nf, self.dim, nq), dtype=torch.float64, device=dev)
        anchor = torch.empty(nq, dtype=torch.int32, device=dev)
        _check(lib().gcr_surface(self._h, nq, _dptr(xq), nf, _ptr_array(fields), _dptr(val),
                                 _dptr(grad), _dptr(anchor, torch.int32), _stream(stream)),
               "gcr_surface")
        return val, grad, anchor

    def forces(self, xq, nrm, wq, p, u: Sequence[torch.Tensor], mu: float, out=None,
               stream=None):
        F = out if out is not None else torch.empty(self.dim, dtype=torch.float64,
                                                    device=xq.device)
        _check(lib().gcr_forces(self._h, xq.shape[1], _dptr(xq), _dptr(nrm), _dptr(wq), _dptr(p),
                                _ptr_array(u), float(mu), _dptr(F), _stream(stream)),
               "gcr_forces")
        return F

    def surface_adjoint(self, xq, gval, ggrad, lam: Sequence[torch.Tensor], stream=None):
        _check(lib().gcr_surface_adjoint(self._h, xq.shape[1], _dptr(xq), len(lam), _dptr(gval),
                                         _dptr(ggrad), _ptr_array(lam), _stream(stream)),
               "gcr_surface_adjoint")

    def forces_adjoint(self, xq, nrm, wq, mu, gF, lam_p, lam_u, stream=None):
        _check(lib().gcr_forces_adjoint(self._h, xq.shape[1], _dptr(xq), _dptr(nrm), _dptr(wq),
                                        float(mu), _dptr(gF), _dptr(lam_p), _ptr_array(lam_u),
                                        _stream(stream)), "gcr_forces_adjoint")

    def fill_adjoint(self, lam: Sequence[torch.Tensor], bc_kind: Sequence[int],
                     lam_bc: Sequence[torch.Tensor], bc_type=None, stream=None):
        nf = len(lam)
        kinds = (ctypes.c_int32 * nf)(*[int(k) for k in bc_kind])
        bt = None
        if bc_type is not None:
            bt = (ctypes.c_void_p * nf)()
            for i, t in enumerate(bc_type):
                bt[i] = _dptr(t, torch.uint8) if t is not None else None
        _check(lib().gcr_fill_adjoint(self._h, nf, _ptr_array(lam), kinds, bt,
                                      _ptr_array(lam_bc), _stream(stream)), "gcr_fill_adjoint")


class _BatchHandle:
    """Owner of a gcr_batch: destroyed when neither the Batch nor any of its
    plans refers to it (plans keep it, not the Batch, so that no reference
    cycle delays the release of the batch's device memory to the pool)."""

    def __init__(self, h):
        self.h = h

    def __del__(self, _finalizing=sys.is_finalizing):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None and not _finalizing():
            _lib.gcr_batch_destroy(h)
        self.h = None


class BatchSpec:
    """The instances of a batch packed once into the C-ABI's host structs,
    for building the same kind of batch repeatedly (a static or moving body
    rebuilt every step) without converting every grid and shape again."""

    def __init__(self, grids, shapes, schemes):
        n = len(grids)
        self.n = n
        gs = [make_grid(g) for g in grids]   # keeps stretched faces alive
        self._keep = ([getattr(g, "_keep", None) for g in gs],
                      [make_shape(s) for s in shapes])
        self.G = (_Grid * n)(*gs)
        self.S = (_Shape * n)(*[k[0] for k in self._keep[1]])
        self.sch = (ctypes.c_int32 * n)(*[int(s) for s in schemes])


class Batch:
    """gcr_batch_create: plans of many uneven instances built together.
    `spec` (a BatchSpec) replaces grids, shapes and schemes."""

    def __init__(self, grids=None, shapes=None, schemes=None, stream=None, spec=None):
        L = lib()
        if spec is None:
            spec = BatchSpec(grids, shapes, schemes)
        h = ctypes.c_void_p()
        _check(L.gcr_batch_create(spec.n, spec.G, spec.S, spec.sch, _stream(stream),
                                  ctypes.byref(h)), "gcr_batch_create")
        self._owner = _BatchHandle(h)
        self._h = h
        self.n = spec.n
        self.dim = int(spec.G[0].dim)
        self._plans = None

    @property
    def plans(self):
        """Plan of every instance (wrappers made on first use)."""
        if self._plans is None:
            L = lib()
            plans = []
            for i in range(self.n):
                ph = ctypes.c_void_p()
                _check(L.gcr_batch_plan(self._h, i, ctypes.byref(ph)), "gcr_batch_plan")
                plans.append(Plan(None, None, 0, _handle=ph, _owner=self._owner))
            self._plans = plans
        return self._plans

    def counts(self):
        """gcr_batch_counts: ghosts per instance, a tuple of ints."""
        buf = (ctypes.c_int64 * self.n)()
        _check(lib().gcr_batch_counts(self._h, buf, None), "gcr_batch_counts")
        return tuple(buf)

    def status(self):
        """gcr_batch_status: waits for the batch's forward launches; raises
        GcrError (GCR_E_TIMEOUT) if a split sweep's wait gave up since the
        last query."""
        _check(lib().gcr_batch_status(self._h), "gcr_batch_status")

    def tiled(self) -> int:
        """gcr_batch_tiled: -1 sweep, 0 undecided, 1 tiled fill, 2 sweep after
        the closures did not fit (synchronises the device)."""
        st = ctypes.c_int32()
        _check(lib().gcr_batch_tiled(self._h, ctypes.byref(st)), "gcr_batch_tiled")
        return st.value

    def shape(self):
        """gcr_batch_shape: (threads, grid) of the forward's launches; grid < 0
        the split sweep (k_batch_split), > 0 per-item workgroups
        (k_batch_forward); (0, 0) before the first forward call."""
        t, g = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().gcr_batch_shape(self._h, ctypes.byref(t), ctypes.byref(g)),
               "gcr_batch_shape")
        return t.value, g.value

    def foot_points(self, stream=None, out=None):
        """gcr_batch_foot_points: (S, normal), each f64 [dim][total ghosts],
        the instances' ghosts one after another (into `out` = (S, normal)
        if given)."""
        dim, ng = self.dim, sum(self.counts())
        if out is not None:
            S, n = out
            if tuple(S.shape) != (dim, ng) or tuple(n.shape) != (dim, ng):
                raise ValueError(f"out: two ({dim}, {ng}) tensors expected")
        else:
            dev = torch.device("cuda")
            S = torch.empty((dim, ng), dtype=torch.float64, device=dev)
            n = torch.empty((dim, ng), dtype=torch.float64, device=dev)
        _check(lib().gcr_batch_foot_points(self._h, _dptr(S), _dptr(n), _stream(stream)),
               "gcr_batch_foot_points")
        return S, n

    def forward(self, nf=None, fields=None, bc_kind=None, bc_val=None, bc_type=None, nq=None,
                xq=None, nrm=None, wq=None, p_field=-1, u_first=-1, mu=1.0, F=None, sval=None,
                sgrad=None, stream=None, args=None):
        """gcr_batch_forward; per-field lists are instance-major [ninst*nf]
        (fields, bc_val, bc_type, sval, sgrad; None entries allowed in the
        last three).  `args`: a ForwardArgs packed once for repeated calls
        with the same tensors, in place of the other arguments."""
        a = args if args is not None else ForwardArgs(
            nf, fields, bc_kind, bc_val, bc_type, nq, xq, nrm, wq, p_field, u_first, mu, F,
            sval, sgrad)
        if a.ninst != self.n:
            raise ValueError(f"arguments packed for {a.ninst} instances, batch has {self.n}")
        _check(lib().gcr_batch_forward(self._h, a.nf, a.fields, a.kinds, a.bt, a.bcv, a.nqa,
                                       a.xa, a.na, a.wa, a.p_field, a.u_first, a.mu, a.F,
                                       a.sval, a.sgrad, _stream(stream)),
               "gcr_batch_forward")
        return a.F_tensor


class ForwardArgs:
    """Arguments of Batch.forward checked and packed into the C-ABI's pointer
    tables once, for repeated calls on the same tensors (the tensors are kept
    alive here; their contents may change between calls)."""

    def __init__(self, nf, fields, bc_kind, bc_val, bc_type=None, nq=None, xq=None, nrm=None,
                 wq=None, p_field=-1, u_first=-1, mu=1.0, F=None, sval=None, sgrad=None):
        if len(fields) % nf or len(bc_val) != len(fields):
            raise ValueError("fields and bc_val: ninst * nf tensors each")
        self.nf = int(nf)
        self.ninst = len(fields) // nf
        for name, ts, n in (("bc_type", bc_type, len(fields)), ("sval", sval, len(fields)),
                            ("sgrad", sgrad, len(fields)), ("nq", nq, self.ninst),
                            ("xq", xq, self.ninst), ("nrm", nrm, self.ninst),
                            ("wq", wq, self.ninst)):
            if ts is not None and len(ts) != n:
                raise ValueError(f"{name}: {n} entries expected, got {len(ts)}")
        self.kinds = (ctypes.c_int32 * nf)(*[int(k) for k in bc_kind])
        self.bt = None
        if bc_type is not None:
            self.bt = (ctypes.c_void_p * len(bc_type))()
            for i, t in enumerate(bc_type):
                self.bt[i] = _dptr(t, torch.uint8) if t is not None else None
        self.nqa = self.xa = self.na = self.wa = None
        if nq is not None:
            self.nqa = (ctypes.c_int64 * len(nq))(*[int(v) for v in nq])
            self.xa, self.na, self.wa = _ptr_array(xq), _ptr_array(nrm), _ptr_array(wq)

        def opt(ts):
            if ts is None:
                return None
            a = (ctypes.c_void_p * len(ts))()
            for k, t in enumerate(ts):
                a[k] = _dptr(t) if t is not None else None
            return a
        self.fields, self.bcv = _ptr_array(fields), _ptr_array(bc_val)
        self.sval, self.sgrad = opt(sval), opt(sgrad)
        self.p_field, self.u_first, self.mu = int(p_field), int(u_first), float(mu)
        self.F = _dptr(F)
        self.F_tensor = F
        self._keep = (fields, bc_val, bc_type, xq, nrm, wq, F, sval, sgrad)


STAGES = ["classify", "interface_scan", "interface_compact", "geometry_tags",
          "ghost_compact", "dependencies", "levels_order", "finalize",
          "classify_prepass", "classify_store", "classify_band", "sizing_wait", "call_host"]


def set_wave_residual(max_ghosts: int = 64):
    """Largest remainder of a stalled Kahn layering (ghosts reading a cycle)
    that one wave resolves; larger ones go to the workgroup (0..64)."""
    _check(lib().gcr_set_wave_residual(int(max_ghosts)), "gcr_set_wave_residual")


def set_wide_buffer(entries: int = 0):
    """Slots of the whole-GPU layering's per-workgroup release buffer
    (1..4096; 0 the default)."""
    _check(lib().gcr_set_wide_buffer(int(entries)), "gcr_set_wide_buffer")


def set_wide_layering(min_interface: int = 0):
    """Interface-cell count from which a plan built alone is layered by the
    whole GPU (0: the default)."""
    _check(lib().gcr_set_wide_layering(int(min_interface)), "gcr_set_wide_layering")


PROFILE_BUILD = 1     # stage timing of plan builds
PROFILE_FORWARD = 2   # timing of the batched forward's kernels


def set_batch_shape(threads: int = 0, grid: int = 0):
    """Launch shape of the batched forward's level sweep: (0, 0) the tuned
    choice; else threads a power of two in 64..1024 and grid 1..4 (per-item
    workgroups) or -1..-128 (split sweep, -grid workgroups per instance)."""
    _check(lib().gcr_set_batch_shape(int(threads), int(grid)), "gcr_set_batch_shape")


def set_batch_spin(polls: int = 0):
    """Polls of a split sweep's wait before it gives up (0: the default)."""
    _check(lib().gcr_set_batch_spin(int(polls)), "gcr_set_batch_spin")


def set_batch_tiling(mode: int):
    """Tiled batched fill: 0 off (level-by-level sweep), 1 from a batch's
    second forward call (the default), 2 from its first."""
    _check(lib().gcr_set_batch_tiling(int(mode)), "gcr_set_batch_tiling")


def set_profiling(on):
    """True: every timing on; False: off; an int: a mask of PROFILE_*."""
    mask = (PROFILE_BUILD | PROFILE_FORWARD) if on is True else (0 if on is False else int(on))
    _check(lib().gcr_set_profiling(mask), "gcr_set_profiling")


def forward_times() -> dict:
    """Mean ms of the batched forward's anchor search and fill + force
    kernels over the calls made with profiling on since the last query."""
    buf = (ctypes.c_float * 3)()
    _check(lib().gcr_forward_times(buf), "gcr_forward_times")
    return {"anchor": buf[0], "forward": buf[1], "calls": int(buf[2])}


def last_build_times() -> dict:
    buf = (ctypes.c_float * len(STAGES))()
    _check(lib().gcr_last_build_times(buf), "gcr_last_build_times")
    return dict(zip(STAGES, list(buf)))


def version() -> str:
    return lib().gcr_version().decode()
