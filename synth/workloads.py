"""Seeded synthetic workloads (SplitMix64 -> 53-bit uniform doubles).

The workloads mirror the paper's setting -- a Cartesian grid cut by a smooth
embedded body, smooth fields, Dirichlet and Neumann data on the body -- at
the sizes named in ``WORKLOADS``:

  circle128   2D, 128^2 on [-2,2]^2, circle R=0.5 at a sub-cell offset,
              u = sin 2x cos 3y (Dirichlet), 256 surface points.
  sphere256   3D, 256^3 on [-1,1]^3, sphere R=0.3 at a sub-cell offset,
              ABC-type u,v,w (Dirichlet) and p = cos x cos y cos z (Neumann).
  airfoil4096 2D, 4096^2 on [-1,3]x[-2,2], 12%-thick symmetric four-digit
              section at 8 deg nose-up, potential-flow-like u,v,p.
  stars64     64 2D instances, n ~ U{128..2048} on [-1,1]^2, Fourier-star
              bodies, 3 fields with mixed Dirichlet/Neumann data.
  shstar384   3D, 384^3 on [-1,1]^3, spherical-harmonic star (l=2..4),
              u,v,w,p as sphere256.

No method arithmetic lives here: the boundary data are the analytic fields
evaluated at points the caller supplies (the foot points S of a plan).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

SPHERE, STAR2D, SHSTAR, AIRFOIL = 0, 1, 2, 3
CGC, CGC_ES, HGC = 0, 1, 2
LAYER2 = 4          # flag: a second ghost layer on top of any scheme
DIRICHLET, NEUMANN = 0, 1

_M64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea & Flood 2014); uniform() gives k/2^53."""

    def __init__(self, seed: int):
        self.state = seed & _M64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _M64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def uniform(self, a: float = 0.0, b: float = 1.0) -> float:
        return a + (b - a) * ((self.next_u64() >> 11) * (1.0 / 9007199254740992.0))

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi]."""
        return lo + int(self.uniform() * (hi - lo + 1))


@dataclass
class Grid:
    """Uniform spacing h per axis from lo, or, where faces[axis] is given, a
    stretched axis: its n + 1 cell faces (lo and h then nominal only)."""
    dim: int
    n: tuple
    lo: tuple
    h: tuple
    faces: tuple = None

    @property
    def n_cells(self) -> int:
        return int(np.prod(self.n[: self.dim]))

    def centres(self, axis: int) -> np.ndarray:
        if self.faces is not None and self.faces[axis] is not None:
            f = np.asarray(self.faces[axis], dtype=np.float64)
            return 0.5 * (f[:-1] + f[1:])
        return self.lo[axis] + (np.arange(self.n[axis]) + 0.5) * self.h[axis]

    def widths(self, axis: int) -> np.ndarray:
        if self.faces is not None and self.faces[axis] is not None:
            return np.diff(np.asarray(self.faces[axis], dtype=np.float64))
        return np.full(self.n[axis], float(self.h[axis]))

    def mesh(self):
        """Cell-centre coordinate arrays, flattened x-fastest."""
        if self.dim == 2:
            y, x = np.meshgrid(self.centres(1), self.centres(0), indexing="ij")
            return x.ravel(), y.ravel()
        z, y, x = np.meshgrid(self.centres(2), self.centres(1), self.centres(0), indexing="ij")
        return x.ravel(), y.ravel(), z.ravel()


@dataclass
class Shape:
    kind: int
    center: tuple
    r0: float = 0.0
    coef: np.ndarray = field(default_factory=lambda: np.zeros(0))
    ncoef: int = 0
    chord: float = 1.0
    thick: float = 0.12
    incidence: float = 0.0


@dataclass
class Field:
    """Analytic field: value f(*x) and gradient grad(*x) -> list of arrays."""
    name: str
    f: Callable
    grad: Callable
    bc: int  # DIRICHLET or NEUMANN (or -1: mixed, see bc_types)


@dataclass
class Queries:
    x: np.ndarray       # [dim][nq]
    n: np.ndarray       # [dim][nq] outward unit normals
    w: np.ndarray       # [nq] quadrature weights


@dataclass
class Instance:
    name: str
    grid: Grid
    shape: Shape
    scheme: int
    fields: List[Field]
    queries: Optional[Queries] = None
    mixed_beta: Optional[np.ndarray] = None  # per-field angle for mixed BCs
    mu: float = 1.0


# --------------------------------------------------------------------------
# analytic fields
# --------------------------------------------------------------------------

def _trig2d():
    f = lambda x, y: np.sin(2 * x) * np.cos(3 * y)
    g = lambda x, y: [2 * np.cos(2 * x) * np.cos(3 * y), -3 * np.sin(2 * x) * np.sin(3 * y)]
    return f, g


def abc_fields():
    """Divergence-free ABC-type velocity and a smooth pressure (3D)."""
    u = Field("u", lambda x, y, z: np.sin(z) + np.cos(y),
              lambda x, y, z: [0 * x, -np.sin(y), np.cos(z)], DIRICHLET)
    v = Field("v", lambda x, y, z: np.sin(x) + np.cos(z),
              lambda x, y, z: [np.cos(x), 0 * y, -np.sin(z)], DIRICHLET)
    w = Field("w", lambda x, y, z: np.sin(y) + np.cos(x),
              lambda x, y, z: [-np.sin(x), np.cos(y), 0 * z], DIRICHLET)
    p = Field("p", lambda x, y, z: np.cos(x) * np.cos(y) * np.cos(z),
              lambda x, y, z: [-np.sin(x) * np.cos(y) * np.cos(z),
                               -np.cos(x) * np.sin(y) * np.cos(z),
                               -np.cos(x) * np.cos(y) * np.sin(z)], NEUMANN)
    return [u, v, w, p]


def polynomial_field(dim: int, coeffs: Sequence[float], bc: int, name="poly") -> Field:
    """Bilinear (2D) / trilinear (3D) field C0 + C1 x + C2 y (+ C3 z) + ...

    2D: C0 + C1 x + C2 y + C3 xy.   3D: C0 + C1 x + C2 y + C3 z + C4 xy +
    C5 yz + C6 xz + C7 xyz.
    """
    c = list(coeffs)
    if dim == 2:
        f = lambda x, y: c[0] + c[1] * x + c[2] * y + c[3] * x * y
        g = lambda x, y: [c[1] + c[3] * y, c[2] + c[3] * x]
    else:
        f = lambda x, y, z: (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y +
                             c[5] * y * z + c[6] * x * z + c[7] * x * y * z)
        g = lambda x, y, z: [c[1] + c[4] * y + c[6] * z + c[7] * y * z,
                             c[2] + c[4] * x + c[5] * z + c[7] * x * z,
                             c[3] + c[5] * y + c[6] * x + c[7] * x * y]
    return Field(name, f, g, bc)


def potential_flow(center, a=0.03, U=1.0, gamma=None, alpha_deg=8.0):
    """Uniform stream + doublet + vortex about `center` (2D), p = (U^2-|w|^2)/2."""
    if gamma is None:
        gamma = math.pi * U * math.sin(math.radians(alpha_deg))
    z0 = complex(center[0], center[1])

    def wfun(x, y):
        z = x + 1j * y - z0
        return U * (1 - a * a / z ** 2) + 1j * gamma / (2 * math.pi * z)

    def dwfun(x, y):
        z = x + 1j * y - z0
        return U * 2 * a * a / z ** 3 - 1j * gamma / (2 * math.pi * z ** 2)

    # complex velocity w = u - i v ; dw/dz = du/dx - i dv/dx ; u_y = -v_x... use w'
    u = Field("u", lambda x, y: wfun(x, y).real,
              lambda x, y: [dwfun(x, y).real, -dwfun(x, y).imag], DIRICHLET)
    v = Field("v", lambda x, y: -wfun(x, y).imag,
              lambda x, y: [-dwfun(x, y).imag, -dwfun(x, y).real], DIRICHLET)

    def pf(x, y):
        w = wfun(x, y)
        return 0.5 * (U * U - (w.real ** 2 + w.imag ** 2))

    def pg(x, y):
        w = wfun(x, y)
        dw = dwfun(x, y)
        uu, vv = w.real, -w.imag
        ux, vx = dw.real, -dw.imag
        uy, vy = -dw.imag, -dw.real
        return [-(uu * ux + vv * vx), -(uu * uy + vv * vy)]

    p = Field("p", pf, pg, NEUMANN)
    return [u, v, p]


# --------------------------------------------------------------------------
# boundary data and field sampling
# --------------------------------------------------------------------------

def sample(fld: Field, grid: Grid) -> np.ndarray:
    return np.asarray(fld.f(*grid.mesh()), dtype=np.float64)


def bc_values(fld: Field, S: np.ndarray, n: np.ndarray, kind) -> np.ndarray:
    """Boundary data at foot points S [dim][N] with normals n: the field value
    (Dirichlet) or the normal derivative grad f . n (Neumann).  `kind` is a
    scalar or an array of per-point kinds."""
    S = np.asarray(S, dtype=np.float64)
    val = np.asarray(fld.f(*S), dtype=np.float64)
    g = fld.grad(*S)
    dn = sum(np.asarray(g[i], dtype=np.float64) * n[i] for i in range(S.shape[0]))
    kind = np.broadcast_to(np.asarray(kind), val.shape)
    return np.where(kind == NEUMANN, dn, val)


def mixed_kinds(S: np.ndarray, center, beta: float) -> np.ndarray:
    """Mixed data: Dirichlet where cos(theta_S - beta) >= 0, else Neumann."""
    th = np.arctan2(S[1] - center[1], S[0] - center[0])
    return np.where(np.cos(th - beta) >= 0.0, DIRICHLET, NEUMANN).astype(np.int8)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def circle_queries(center, R, nq=256):
    th = 2 * np.pi * np.arange(nq) / nq
    x = np.stack([center[0] + R * np.cos(th), center[1] + R * np.sin(th)])
    n = np.stack([np.cos(th), np.sin(th)])
    w = np.full(nq, 2 * np.pi * R / nq)
    return Queries(x, n, w)


def sphere_queries(center, R, nt=32, nph=64):
    ct, wt = np.polynomial.legendre.leggauss(nt)
    ph = 2 * np.pi * np.arange(nph) / nph
    CT, PH = np.meshgrid(ct, ph, indexing="ij")
    ST = np.sqrt(1 - CT ** 2)
    n = np.stack([ST * np.cos(PH), ST * np.sin(PH), CT]).reshape(3, -1)
    x = np.asarray(center, dtype=np.float64)[:, None] + R * n
    w = (np.repeat(wt, nph) * (2 * np.pi / nph) * R * R)
    return Queries(x, n, w)


def circle128(seed: int = 0, scheme: int = HGC, nq: int = 256) -> Instance:
    rng = SplitMix64(0xC1C1E000 + seed)
    h = 4.0 / 128
    grid = Grid(2, (128, 128, 1), (-2.0, -2.0, 0.0), (h, h, 1.0))
    c = (rng.uniform(0, h), rng.uniform(0, h), 0.0)
    shape = Shape(SPHERE, c, 0.5)
    f, g = _trig2d()
    return Instance("circle128", grid, shape, scheme, [Field("u", f, g, DIRICHLET)],
                    circle_queries(c, 0.5, nq))


def stretched_faces(n: int, lo: float, hi: float, ratio: float) -> np.ndarray:
    """n cells on [lo, hi] whose widths grow geometrically by `ratio` per
    cell from the middle of the axis outward (the paper's grids are
    stretched by a fixed ratio away from the body)."""
    k = np.abs(np.arange(n) - (n - 1) / 2.0)
    w = ratio ** k
    w *= (hi - lo) / w.sum()
    f = np.concatenate([[lo], lo + np.cumsum(w)])
    f[-1] = hi
    return f


def circle_stretched(seed: int = 0, scheme: int = HGC, n: int = 128, ratio: float = 1.02,
                     nq: int = 256) -> Instance:
    """The circle of circle128 on a grid stretched by `ratio` per cell."""
    rng = SplitMix64(0xC1C15700 + seed)
    fx, fy = stretched_faces(n, -2.0, 2.0, ratio), stretched_faces(n, -2.0, 2.0, ratio * 1.005)
    h = 4.0 / n
    grid = Grid(2, (n, n, 1), (-2.0, -2.0, 0.0), (h, h, 1.0), (fx, fy, None))
    c = (rng.uniform(0, h), rng.uniform(0, h), 0.0)
    shape = Shape(SPHERE, c, 0.5)
    f, g = _trig2d()
    return Instance("circle_stretched", grid, shape, scheme, [Field("u", f, g, DIRICHLET)],
                    circle_queries(c, 0.5, nq))


def sphere_stretched(seed: int = 0, scheme: int = HGC, n: int = 48,
                     ratio: float = 1.03) -> Instance:
    """The sphere of sphere256 on an n^3 grid stretched by `ratio` per cell."""
    rng = SplitMix64(0x5F357000 + seed)
    h = 2.0 / n
    faces = tuple(stretched_faces(n, -1.0, 1.0, ratio + 0.004 * a) for a in range(3))
    grid = Grid(3, (n, n, n), (-1.0, -1.0, -1.0), (h, h, h), faces)
    c = (rng.uniform(0, h), rng.uniform(0, h), rng.uniform(0, h))
    shape = Shape(SPHERE, c, 0.3)
    return Instance(f"sphere_stretched{n}", grid, shape, scheme, abc_fields(),
                    sphere_queries(c, 0.3))


def sphere256(seed: int = 0, scheme: int = HGC, n: int = 256) -> Instance:
    rng = SplitMix64(0x5F3E0000 + seed)
    h = 2.0 / n
    grid = Grid(3, (n, n, n), (-1.0, -1.0, -1.0), (h, h, h))
    c = (rng.uniform(0, h), rng.uniform(0, h), rng.uniform(0, h))
    shape = Shape(SPHERE, c, 0.3)
    return Instance(f"sphere{n}", grid, shape, scheme, abc_fields(), sphere_queries(c, 0.3))


def star_shape(rng: SplitMix64, center, kmax=5, amax=0.05, r0=None) -> Shape:
    """r(theta) = r0 (1 + sum_{k=2..kmax} a_k cos(k theta + phi_k)), stored as
    coefficients A_k = a_k cos phi_k, B_k = -a_k sin phi_k of cos/sin k theta."""
    if r0 is None:
        r0 = rng.uniform(0.3, 0.6)
    coef = np.zeros((kmax + 1, 2))
    for k in range(2, kmax + 1):
        a = rng.uniform(0, amax)
        ph = rng.uniform(0, 2 * np.pi)
        coef[k] = (a * math.cos(ph), -a * math.sin(ph))
    return Shape(STAR2D, tuple(center), r0, coef.ravel(), kmax + 1)


def star_radius(shape: Shape, th):
    coef = np.asarray(shape.coef).reshape(-1, 2)
    r = np.ones_like(th)
    dr = np.zeros_like(th)
    for k in range(coef.shape[0]):
        r = r + coef[k, 0] * np.cos(k * th) + coef[k, 1] * np.sin(k * th)
        dr = dr + k * (-coef[k, 0] * np.sin(k * th) + coef[k, 1] * np.cos(k * th))
    return shape.r0 * r, shape.r0 * dr


def star_queries(shape: Shape, nq=512):
    th = 2 * np.pi * np.arange(nq) / nq
    r, dr = star_radius(shape, th)
    c = shape.center
    x = np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th)])
    T = np.stack([dr * np.cos(th) - r * np.sin(th), dr * np.sin(th) + r * np.cos(th)])
    ds = np.hypot(T[0], T[1])
    n = np.stack([T[1], -T[0]]) / ds
    return Queries(x, n, ds * 2 * np.pi / nq)


def stars64(seed: int = 0, ninst: int = 64, nmin: int = 128, nmax: int = 2048,
            scheme: int = HGC) -> List[Instance]:
    rng = SplitMix64(0x57A45000 + seed)
    out = []
    f, g = _trig2d()
    for i in range(ninst):
        n = rng.randint(nmin, nmax)
        h = 2.0 / n
        grid = Grid(2, (n, n, 1), (-1.0, -1.0, 0.0), (h, h, 1.0))
        c = (rng.uniform(0, h), rng.uniform(0, h), 0.0)
        shape = star_shape(rng, c)
        flds = [Field("u", f, g, -1),
                Field("v", lambda x, y: np.cos(x + 2 * y), lambda x, y: [-np.sin(x + 2 * y), -2 * np.sin(x + 2 * y)], -1),
                Field("p", lambda x, y: np.exp(0.5 * x) * np.sin(y),
                      lambda x, y: [0.5 * np.exp(0.5 * x) * np.sin(y), np.exp(0.5 * x) * np.cos(y)], -1)]
        beta = np.array([rng.uniform(0, 2 * np.pi) for _ in range(3)])
        out.append(Instance(f"star{i}_{n}", grid, shape, scheme, flds, star_queries(shape, 256),
                            mixed_beta=beta))
    return out


def sh_shape(rng: SplitMix64, center, r0=0.3, L=4, amax=0.04) -> Shape:
    coef = np.zeros((L + 1) ** 2)
    for l in range(2, L + 1):
        for m in range(-l, l + 1):
            coef[l * l + l + m] = rng.uniform(0, amax)
    return Shape(SHSTAR, tuple(center), r0, coef, (L + 1) ** 2)


def _sh_real_schmidt(l, m, ct, ph):
    """Real Schmidt semi-normalised Y_lm (no Condon-Shortley phase), via scipy."""
    from scipy.special import lpmv
    am = abs(m)
    P = lpmv(am, l, ct) * ((-1.0) ** am)  # remove Condon-Shortley phase
    N = 1.0 if am == 0 else math.sqrt(2.0 * math.factorial(l - am) / math.factorial(l + am))
    return N * P * (np.cos(am * ph) if m >= 0 else np.sin(am * ph))


def sh_radius(shape: Shape, ct, ph):
    L = int(round(math.sqrt(shape.ncoef))) - 1
    r = np.ones_like(ct)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            a = shape.coef[l * l + l + m]
            if a != 0.0:
                r = r + a * _sh_real_schmidt(l, m, ct, ph)
    return shape.r0 * r


def sh_queries(shape: Shape, nt=64, nph=128, eps=1e-6):
    """Gauss-Legendre in cos(theta) x uniform phi on the SH star surface;
    normals and area elements from central differences of the surface map."""
    ct, wt = np.polynomial.legendre.leggauss(nt)
    ph = 2 * np.pi * np.arange(nph) / nph
    CT, PH = np.meshgrid(ct, ph, indexing="ij")
    CT, PH = CT.ravel(), PH.ravel()
    c = np.asarray(shape.center, dtype=np.float64)[:, None]

    def X(ct_, ph_):
        st_ = np.sqrt(np.maximum(0.0, 1 - ct_ ** 2))
        om = np.stack([st_ * np.cos(ph_), st_ * np.sin(ph_), ct_])
        return c + sh_radius(shape, ct_, ph_) * om

    Xc = X(CT, PH)
    Xt = (X(CT + eps, PH) - X(CT - eps, PH)) / (2 * eps)   # d/d(cos theta)
    Xp = (X(CT, PH + eps) - X(CT, PH - eps)) / (2 * eps)
    cr = np.cross(Xp.T, Xt.T).T   # outward for increasing phi x increasing cos
    area = np.linalg.norm(cr, axis=0)
    n = cr / area
    w = np.repeat(wt, nph) * (2 * np.pi / nph) * area
    # orient outward
    sgn = np.sign(np.sum(n * (Xc - c), axis=0))
    return Queries(Xc, n * sgn, w)


def shstar384(seed: int = 0, n: int = 384, scheme: int = HGC, nt=64, nph=128) -> Instance:
    rng = SplitMix64(0x5A5A0000 + seed)
    h = 2.0 / n
    grid = Grid(3, (n, n, n), (-1.0, -1.0, -1.0), (h, h, h))
    c = (rng.uniform(0, h), rng.uniform(0, h), rng.uniform(0, h))
    shape = sh_shape(rng, c)
    return Instance(f"shstar{n}", grid, shape, scheme, abc_fields(), sh_queries(shape, nt, nph))


def airfoil_queries(shape: Shape, m=1024):
    """Both surfaces sampled with x = s^2 (trapezoid weights |dX/ds| ds)."""
    s = np.linspace(-1.0, 1.0, 2 * m + 1)[:-1] + 1.0 / (2 * m)
    t = shape.thick
    s2 = s * s
    sg = np.sign(s)
    poly = 0.1260 * s2 + 0.3516 * s2 ** 2 - 0.2843 * s2 ** 3 + 0.1036 * s2 ** 4
    dpoly = 2 * 0.1260 * s + 4 * 0.3516 * s2 * s - 6 * 0.2843 * s2 ** 2 * s + 8 * 0.1036 * s2 ** 3 * s
    bx, by = s2, 5 * t * (0.2969 * s - sg * poly)
    tx, ty = 2 * s, 5 * t * (0.2969 - sg * dpoly)
    ca, sa = math.cos(shape.incidence), math.sin(shape.incidence)
    ch = shape.chord
    x = np.stack([shape.center[0] + ch * (ca * bx + sa * by), shape.center[1] + ch * (-sa * bx + ca * by)])
    T = np.stack([ca * tx + sa * ty, -sa * tx + ca * ty]) * ch
    ds = np.hypot(T[0], T[1])
    n = np.stack([-T[1], T[0]]) / ds   # contour is clockwise in s
    w = ds * (2.0 / (2 * m))
    return Queries(x, n, w)


def airfoil4096(seed: int = 0, n: int = 4096, scheme: int = HGC, m: int = 1024) -> Instance:
    rng = SplitMix64(0xA1F00000 + seed)
    h = 4.0 / n
    grid = Grid(2, (n, n, 1), (-1.0, -2.0, 0.0), (h, h, 1.0))
    le = (rng.uniform(0, h), rng.uniform(0, h), 0.0)
    shape = Shape(AIRFOIL, le, 0.0, np.zeros(0), 0, 1.0, 0.12, math.radians(8.0))
    qc = (le[0] + 0.25 * math.cos(shape.incidence), le[1] - 0.25 * math.sin(shape.incidence))
    return Instance(f"airfoil{n}", grid, shape, scheme, potential_flow(qc), airfoil_queries(shape, m))


WORKLOADS = {
    "circle128": circle128,
    "sphere256": sphere256,
    "airfoil4096": airfoil4096,
    "stars64": stars64,
    "shstar384": shstar384,
}
