"""CPU oracle for the direct ghost-cell method (ctypes wrapper over oracle.c).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.  It
shares no code with the GPU path.  Every function follows the paper section
cited in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

SPHERE, STAR2D, SHSTAR, AIRFOIL = 0, 1, 2, 3
CGC, CGC_ES, HGC = 0, 1, 2
DIRICHLET, NEUMANN = 0, 1
STATUS = {0: "ok", 1: "bad argument", 3: "out of memory", 4: "cycle",
          5: "stencil", 6: "degenerate", 7: "geometry", 8: "unsupported"}


def build(force: bool = True) -> str:
    """Compile oracle.c into _build/liboracle.so (gcc, FP64, no contraction)."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-o", tmp, os.path.join(_HERE, "oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("lo", ctypes.c_double * 3),
                ("h", ctypes.c_double * 3), ("faces", ctypes.c_void_p * 3)]


class _Shape(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("ncoef", ctypes.c_int32),
                ("c", ctypes.c_double * 3), ("r0", ctypes.c_double),
                ("coef", ctypes.POINTER(ctypes.c_double)),
                ("chord", ctypes.c_double), ("thick", ctypes.c_double),
                ("incidence", ctypes.c_double)]


def _P(a, t=ctypes.c_double):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(t))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        vp = ctypes.c_void_p
        L.orc_plan_create.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Shape),
                                      ctypes.c_int, ctypes.POINTER(vp)]
        L.orc_plan_destroy.argtypes = [vp]
        for f in ("orc_n_cells", "orc_n_ghost", "orc_n_interface"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = ctypes.c_int64
        L.orc_n_levels.argtypes = [vp]
        L.orc_n_levels.restype = ctypes.c_int32
        L.orc_dim.argtypes = [vp]
        L.orc_export.argtypes = [vp] + [vp] * 8
        L.orc_stencil.argtypes = [vp, ctypes.c_int64, vp]
        L.orc_margins.argtypes = [vp, vp]
        L.orc_units.argtypes = [vp, vp, vp, vp]
        L.orc_weights.argtypes = [vp, ctypes.c_int64, ctypes.c_int, vp, vp]
        L.orc_weights_raw.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp]
        L.orc_weight_bounds.argtypes = [vp, ctypes.c_int64, ctypes.c_int, vp, vp]
        L.orc_weight_bounds_raw.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp]
        L.orc_fill.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.orc_fresh_cells.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64]
        L.orc_fill_jacobi.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_int]
        L.orc_fill_scale.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
        L.orc_surface_ghost.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.orc_surface_query.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int, vp, vp,
                                        vp, vp, vp, vp]
        L.orc_forces.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp,
                                 ctypes.c_double, vp]
        L.orc_surface_query_adjoint.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int,
                                                vp, vp, vp]
        L.orc_fill_adjoint.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.orc_surface_query_adjoint_scale.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int,
                                                      vp, vp, vp]
        L.orc_fill_adjoint_scale.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.orc_shape_project.argtypes = [ctypes.POINTER(_Shape), ctypes.c_int, vp,
                                        ctypes.c_int, vp, vp, vp]
        L.orc_shape_inside.argtypes = [ctypes.POINTER(_Shape), ctypes.c_int, vp]
        L.orc_shape_radius.argtypes = [ctypes.POINTER(_Shape), ctypes.c_int, vp]
        L.orc_shape_radius.restype = ctypes.c_double
        L.orc_sh_basis.argtypes = [ctypes.c_int, ctypes.c_int, vp]
        L.orc_sh_basis.restype = ctypes.c_double
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


def _vp(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def make_grid(grid) -> _Grid:
    """The ctypes grid; a stretched grid's face arrays are kept alive on it."""
    g = _Grid()
    g.dim = grid.dim
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
    s = _Shape()
    s.kind = shape.kind
    coef = np.ascontiguousarray(np.asarray(shape.coef, dtype=np.float64).ravel())
    s.ncoef = shape.ncoef
    for i in range(3):
        s.c[i] = float(shape.center[i]) if i < len(shape.center) else 0.0
    s.r0 = float(shape.r0)
    s.coef = _P(coef) if coef.size else None
    s.chord, s.thick, s.incidence = float(shape.chord), float(shape.thick), float(shape.incidence)
    return s, coef


def project(shape, dim, x, solid):
    s, keep = make_shape(shape)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3) if len(x) == 3
                             else np.r_[np.asarray(x, dtype=np.float64), 0.0])
    S = np.zeros(3)
    n = np.zeros(3)
    psi = np.zeros(1)
    st = lib().orc_shape_project(ctypes.byref(s), dim, _vp(x), int(solid), _vp(S), _vp(n), _vp(psi))
    if st:
        raise OracleError(st, "project")
    return S[:dim], n[:dim], float(psi[0])


def inside(shape, dim, x):
    s, keep = make_shape(shape)
    x = np.zeros(3) + np.r_[np.asarray(x, dtype=np.float64), np.zeros(3 - len(x))]
    return bool(lib().orc_shape_inside(ctypes.byref(s), dim, _vp(x)))


def weights_raw(dim, bc, x2, xs, n):
    """Closed-form weights from local geometry (x_1 = 0)."""
    a = [np.ascontiguousarray(np.r_[np.asarray(v, dtype=np.float64), np.zeros(3 - len(v))])
         for v in (x2, xs, n)]
    w = np.zeros(7)
    ws = np.zeros(1)
    lib().orc_weights_raw(int(dim), int(bc), *[_vp(v) for v in a], _vp(w), _vp(ws))
    return w[: (3 if dim == 2 else 7)], float(ws[0])


def weight_bounds_raw(dim, bc, x2, xs, n):
    """Tolerance bounds of the closed-form weights (magnitude plus
    sensitivity to the foot point and the normal)."""
    a = [np.ascontiguousarray(np.r_[np.asarray(v, dtype=np.float64), np.zeros(3 - len(v))])
         for v in (x2, xs, n)]
    w = np.zeros(7)
    ws = np.zeros(1)
    lib().orc_weight_bounds_raw(int(dim), int(bc), *[_vp(v) for v in a], _vp(w), _vp(ws))
    return w[: (3 if dim == 2 else 7)], float(ws[0])


def sh_basis(l, m, v):
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    return lib().orc_sh_basis(l, m, _vp(v))


class OraclePlan:
    """Ghost-cell plan built by the oracle from (grid, shape, scheme)."""

    def __init__(self, grid, shape, scheme):
        self.grid = grid
        g = make_grid(grid)
        s, self._coef = make_shape(shape)
        h = ctypes.c_void_p()
        st = lib().orc_plan_create(ctypes.byref(g), ctypes.byref(s), int(scheme), ctypes.byref(h))
        if st:
            raise OracleError(st, "orc_plan_create")
        self._h = h
        L = lib()
        self.dim = grid.dim
        self.n_cells = L.orc_n_cells(h)
        self.n_ghost = L.orc_n_ghost(h)
        self.n_interface = L.orc_n_interface(h)
        self.n_levels = L.orc_n_levels(h)
        ng, d = self.n_ghost, self.dim
        self.tags = np.zeros(self.n_cells, np.int8)
        self.ghost_cell = np.zeros(ng, np.int64)
        self.level_off = np.zeros(self.n_levels + 1, np.int32)
        self.level = np.zeros(ng, np.int32)
        self.delta = np.zeros((d, ng))
        self.normal = np.zeros((d, ng))
        self.psi = np.zeros(ng)
        self.r = np.zeros((d, ng), np.int32)
        L.orc_export(h, *[_vp(a) for a in (self.tags, self.ghost_cell, self.level_off,
                                            self.level, self.delta, self.normal,
                                            self.psi, self.r)])
        m = np.zeros(7)
        L.orc_margins(h, _vp(m))
        self.margins = dict(classify=m[0], hgc=m[1], multiplier=m[2], normal_sign=m[3],
                            max_alpha=m[4:4 + d].copy())
        nb, mb = ctypes.c_int32(), ctypes.c_int32()
        self.unit = np.zeros(ng, np.int32)
        L.orc_units(h, ctypes.byref(nb), ctypes.byref(mb), _vp(self.unit))
        self.n_units_coupled, self.max_unit = nb.value, mb.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_plan_destroy(h)
            self._h = None

    @property
    def min_margin(self):
        return min(self.margins["classify"], self.margins["hgc"],
                   self.margins["multiplier"], self.margins["normal_sign"])

    def stencil(self, g):
        out = np.zeros(7, np.int64)
        lib().orc_stencil(self._h, int(g), _vp(out))
        return out[: (3 if self.dim == 2 else 7)]

    def weights(self, g, bc):
        w = np.zeros(7)
        ws = np.zeros(1)
        lib().orc_weights(self._h, int(g), int(bc), _vp(w), _vp(ws))
        return w[: (3 if self.dim == 2 else 7)], float(ws[0])

    def weight_bounds(self, g, bc):
        w = np.zeros(7)
        ws = np.zeros(1)
        lib().orc_weight_bounds(self._h, int(g), int(bc), _vp(w), _vp(ws))
        return w[: (3 if self.dim == 2 else 7)], float(ws[0])

    @staticmethod
    def _bc(bc_type, nf, ng):
        bc_type = np.asarray(bc_type, dtype=np.int8)
        if bc_type.ndim == 1 and bc_type.size == nf:
            bc_type = np.repeat(bc_type[:, None], ng, axis=1)
        return np.ascontiguousarray(bc_type.reshape(nf, ng))

    def fresh_cells(self, after):
        """Fresh cells when the body of this plan moves to that of `after`
        (same grid): (ascending linear indices, number uncovered)."""
        nf, nu = ctypes.c_int64(), ctypes.c_int64()
        st = lib().orc_fresh_cells(self._h, after._h, ctypes.byref(nf), ctypes.byref(nu), None, 0)
        if st:
            raise OracleError(st, "orc_fresh_cells")
        out = np.zeros(max(nf.value, 1), np.int64)
        lib().orc_fresh_cells(self._h, after._h, ctypes.byref(nf), ctypes.byref(nu), _vp(out),
                              nf.value)
        return out[:nf.value], nu.value

    def fill(self, fields, bc_type, bc_val):
        f = np.ascontiguousarray(np.array(fields, dtype=np.float64).reshape(-1, self.n_cells))
        nf = f.shape[0]
        bt = self._bc(bc_type, nf, self.n_ghost)
        bv = np.ascontiguousarray(np.asarray(bc_val, dtype=np.float64).reshape(nf, self.n_ghost))
        st = lib().orc_fill(self._h, nf, _vp(f), _vp(bt), _vp(bv))
        if st:
            raise OracleError(st, "orc_fill")
        return f

    def fill_jacobi(self, fields, bc_type, bc_val, max_sweeps=1000):
        f = np.ascontiguousarray(np.array(fields, dtype=np.float64).reshape(-1, self.n_cells))
        nf = f.shape[0]
        bt = self._bc(bc_type, nf, self.n_ghost)
        bv = np.ascontiguousarray(np.asarray(bc_val, dtype=np.float64).reshape(nf, self.n_ghost))
        sweeps = lib().orc_fill_jacobi(self._h, nf, _vp(f), _vp(bt), _vp(bv), int(max_sweeps))
        return f, sweeps

    def fill_scale(self, fields, bc_type, bc_val):
        f = np.ascontiguousarray(np.asarray(fields, dtype=np.float64).reshape(-1, self.n_cells))
        nf = f.shape[0]
        bt = self._bc(bc_type, nf, self.n_ghost)
        bv = np.ascontiguousarray(np.asarray(bc_val, dtype=np.float64).reshape(nf, self.n_ghost))
        sc = np.zeros((nf, self.n_ghost))
        st = lib().orc_fill_scale(self._h, nf, _vp(f), _vp(bt), _vp(bv), _vp(sc))
        if st:
            raise OracleError(st, "orc_fill_scale")
        return sc

    def cell_scale(self, fields, ghost_scale):
        """Dense per-cell scale: |phi| on non-ghost cells, s_G on ghosts."""
        f = np.abs(np.asarray(fields, dtype=np.float64).reshape(-1, self.n_cells)).copy()
        f[:, self.ghost_cell] = ghost_scale
        return f

    def surface_ghost(self, fields):
        f = np.ascontiguousarray(np.asarray(fields, dtype=np.float64).reshape(-1, self.n_cells))
        nf = f.shape[0]
        val = np.zeros((nf, self.n_ghost))
        grad = np.zeros((nf, self.dim, self.n_ghost))
        lib().orc_surface_ghost(self._h, nf, _vp(f), _vp(val), _vp(grad))
        return val, grad

    def surface_query(self, xq, fields, field_scale=None):
        xq = np.ascontiguousarray(np.asarray(xq, dtype=np.float64).reshape(self.dim, -1))
        nq = xq.shape[1]
        f = np.ascontiguousarray(np.asarray(fields, dtype=np.float64).reshape(-1, self.n_cells))
        nf = f.shape[0]
        val = np.zeros((nf, nq))
        grad = np.zeros((nf, self.dim, nq))
        anchor = np.zeros(nq, np.int64)
        fs = None if field_scale is None else np.ascontiguousarray(
            np.asarray(field_scale, dtype=np.float64).reshape(nf, self.n_cells))
        sc = None if fs is None else np.zeros((nf, self.dim + 1, nq))
        st = lib().orc_surface_query(self._h, nq, _vp(xq), nf, _vp(f), _vp(val), _vp(grad),
                                     _vp(anchor), _vp(fs), _vp(sc))
        if st:
            raise OracleError(st, "orc_surface_query")
        return (val, grad, anchor) if sc is None else (val, grad, anchor, sc)

    def forces(self, xq, nq_, wq, p, u, mu):
        xq = np.ascontiguousarray(np.asarray(xq, dtype=np.float64).reshape(self.dim, -1))
        nrm = np.ascontiguousarray(np.asarray(nq_, dtype=np.float64).reshape(self.dim, -1))
        wq = np.ascontiguousarray(np.asarray(wq, dtype=np.float64).ravel())
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float64).ravel())
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(self.dim, self.n_cells))
        F = np.zeros(self.dim)
        st = lib().orc_forces(self._h, xq.shape[1], _vp(xq), _vp(nrm), _vp(wq), _vp(p), _vp(u),
                              float(mu), _vp(F))
        if st:
            raise OracleError(st, "orc_forces")
        return F

    def surface_query_adjoint(self, xq, gval, ggrad, lam):
        xq = np.ascontiguousarray(np.asarray(xq, dtype=np.float64).reshape(self.dim, -1))
        nq = xq.shape[1]
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        nf = lam.reshape(-1, self.n_cells).shape[0]
        gv = None if gval is None else np.ascontiguousarray(np.asarray(gval, np.float64).reshape(nf, nq))
        gg = None if ggrad is None else np.ascontiguousarray(
            np.asarray(ggrad, np.float64).reshape(nf, self.dim, nq))
        st = lib().orc_surface_query_adjoint(self._h, nq, _vp(xq), nf, _vp(gv), _vp(gg), _vp(lam))
        if st:
            raise OracleError(st, "orc_surface_query_adjoint")
        return lam

    def fill_adjoint(self, lam, bc_type):
        lam = np.ascontiguousarray(np.array(lam, dtype=np.float64).reshape(-1, self.n_cells))
        nf = lam.shape[0]
        bt = self._bc(bc_type, nf, self.n_ghost)
        lam_bc = np.zeros((nf, self.n_ghost))
        st = lib().orc_fill_adjoint(self._h, nf, _vp(lam), _vp(bt), _vp(lam_bc))
        if st:
            raise OracleError(st, "orc_fill_adjoint")
        return lam, lam_bc

    def surface_query_adjoint_scale(self, xq, gval, ggrad, lam_scale):
        """Adds, per cell, the magnitudes of the terms that
        surface_query_adjoint would add there (the scale of its rounding)."""
        xq = np.ascontiguousarray(np.asarray(xq, dtype=np.float64).reshape(self.dim, -1))
        nq = xq.shape[1]
        lam_scale = np.ascontiguousarray(lam_scale, dtype=np.float64)
        nf = lam_scale.reshape(-1, self.n_cells).shape[0]
        gv = None if gval is None else np.ascontiguousarray(np.asarray(gval, np.float64).reshape(nf, nq))
        gg = None if ggrad is None else np.ascontiguousarray(
            np.asarray(ggrad, np.float64).reshape(nf, self.dim, nq))
        st = lib().orc_surface_query_adjoint_scale(self._h, nq, _vp(xq), nf, _vp(gv), _vp(gg),
                                                   _vp(lam_scale))
        if st:
            raise OracleError(st, "orc_surface_query_adjoint_scale")
        return lam_scale

    def fill_adjoint_scale(self, lam_scale, bc_type):
        """Scale of every output of fill_adjoint given the scale of its input
        (the reverse sweep on magnitudes; units by |A^-T|)."""
        lam = np.ascontiguousarray(np.array(lam_scale, dtype=np.float64).reshape(-1, self.n_cells))
        nf = lam.shape[0]
        bt = self._bc(bc_type, nf, self.n_ghost)
        lam_bc = np.zeros((nf, self.n_ghost))
        st = lib().orc_fill_adjoint_scale(self._h, nf, _vp(lam), _vp(bt), _vp(lam_bc))
        if st:
            raise OracleError(st, "orc_fill_adjoint_scale")
        return lam, lam_bc
