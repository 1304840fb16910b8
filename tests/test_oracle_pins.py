"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it pins.  None of them compares the oracle with
itself: expected values come from the paper's worked example, Appendix A's
Vandermonde systems (solved here with numpy), polynomial reproduction,
special cases with textbook answers, closed-form integrals, brute force on
tiny inputs, or invariants the paper states.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from synth import CGC, CGC_ES, HGC, DIRICHLET, NEUMANN

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def quarter_plan(scheme):
    g = synth.Grid(2, (12, 12, 1), (-6.0, -6.0, 0.0), (1.0, 1.0, 1.0))
    s = synth.Shape(synth.SPHERE, (0.0, 0.0, 0.0), 3.75)
    return oracle.OraclePlan(g, s, scheme)


def quadrant_sets(p):
    T = p.tags.reshape(12, 12)
    ghosts, solid = set(), set()
    for j in range(6, 12):
        for i in range(6, 12):
            key = (i - 6 + 0.5, j - 6 + 0.5)
            if T[j, i] in (2, -2):
                ghosts.add(key)
            if T[j, i] == 1:
                solid.add(key)
    return ghosts, solid, T


# ---------------------------------------------------------------------------
# Sec. 3.1 / 3.3 worked example (circle R = 3.75 h about a grid vertex)
# ---------------------------------------------------------------------------

def test_fig3_cgc_tags():
    fx = json.load(open(os.path.join(GOLDEN, "fig3_quarter_circle.json")))
    for scheme in (CGC, CGC_ES):
        ghosts, solid, T = quadrant_sets(quarter_plan(scheme))
        assert ghosts == {tuple(c) for c in fx["cgc"]["ghosts"]}
        assert solid == {tuple(c) for c in fx["cgc"]["solid"]}
        # every CGC ghost centre is in the solid (tag +2)
        assert all(T[int(y + 6), int(x + 6)] == 2 for x, y in ghosts)


def test_fig3_hgc_tags():
    fx = json.load(open(os.path.join(GOLDEN, "fig3_quarter_circle.json")))
    p = quarter_plan(HGC)
    ghosts, solid, T = quadrant_sets(p)
    assert ghosts == {tuple(c) for c in fx["hgc"]["ghosts"]}
    fluid_side = {tuple(c) for c in fx["hgc"]["fluid_side_ghosts"]}
    # fluid-centred ghosts are -2, solid-centred ones +2
    for x, y in ghosts:
        t = T[int(y + 6), int(x + 6)]
        assert t == (-2 if (x, y) in fluid_side else 2)
    assert solid == {tuple(c) for c in fx["hgc"]["solid"]}


def test_fig3_foot_points():
    fx = json.load(open(os.path.join(GOLDEN, "fig3_quarter_circle.json")))
    tol = fx["foot_point_tolerance"]
    for scheme, key in ((CGC, "cgc"), (HGC, "hgc")):
        p = quarter_plan(scheme)
        for k, c in enumerate(p.ghost_cell):
            i, j = c % 12 - 6, c // 12 - 6
            name = f"{i + 0.5},{j + 0.5}"
            if name in fx[key]["foot_points"]:
                S = np.array([i + 0.5, j + 0.5]) + p.delta[:, k]
                assert np.abs(S - fx[key]["foot_points"][name]).max() < tol


def test_fig3_levels_by_hand():
    """Levels derived by hand from Sec. 3.2's rule on the worked example: the
    CGC ghost (1.5,2.5) reads ghost (2.5,2.5) through P1, so it sits in L2;
    the HGC ghost (0.5,3.5) reads the fluid-side ghost (1.5,3.5)."""
    def levels(p):
        out = {}
        for k, c in enumerate(p.ghost_cell):
            i, j = c % 12 - 6, c // 12 - 6
            if i >= 0 and j >= 0:
                out[(i + 0.5, j + 0.5)] = int(p.level[k])
        return out
    cgc = levels(quarter_plan(CGC))
    assert cgc == {(0.5, 3.5): 1, (2.5, 2.5): 1, (3.5, 0.5): 1, (1.5, 2.5): 2, (2.5, 1.5): 2}
    assert levels(quarter_plan(CGC_ES)) == cgc
    hgc = levels(quarter_plan(HGC))
    assert hgc == {(1.5, 3.5): 1, (2.5, 2.5): 1, (3.5, 1.5): 1, (0.5, 3.5): 2, (3.5, 0.5): 2}


def test_fig3_extended_multiplier():
    """Eq. stencil_anisotropic on ghost (1.5,2.5): |x_s - x_1| = psi |n| gives
    r = (1, 2) and alpha = (0.4294, 0.3578) (hand computation)."""
    p = quarter_plan(CGC_ES)
    for k, c in enumerate(p.ghost_cell):
        if (c % 12 - 6, c // 12 - 6) == (1, 2):
            assert list(p.r[:, k]) == [1, 2]
            psi = 3.75 - math.hypot(1.5, 2.5)
            assert abs(p.psi[k] - psi) < 1e-14
            alpha = np.abs(p.delta[:, k]) / p.r[:, k]
            assert np.allclose(alpha, [psi * 1.5 / math.hypot(1.5, 2.5),
                                       psi * 2.5 / math.hypot(1.5, 2.5) / 2], atol=1e-14)
            return
    pytest.fail("ghost not found")


# ---------------------------------------------------------------------------
# Appendix A: closed-form weights = first row of the inverse Vandermonde
# ---------------------------------------------------------------------------

def _basis(dim, x):
    if dim == 2:
        return np.array([1.0, x[0], x[1], x[0] * x[1]])
    X, Y, Z = x
    return np.array([1.0, X, Y, Z, X * Y, Y * Z, X * Z, X * Y * Z])


def _basis_grad(dim, x):
    if dim == 2:
        return np.array([[0, 1, 0, x[1]], [0, 0, 1, x[0]]], dtype=float)
    X, Y, Z = x
    return np.array([[0, 1, 0, 0, Y, 0, Z, Y * Z],
                     [0, 0, 1, 0, X, Z, 0, X * Z],
                     [0, 0, 0, 1, 0, Y, X, X * Y]], dtype=float)


def _subsets(dim):
    return ([(1, 0), (0, 1), (1, 1)] if dim == 2 else
            [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (0, 1, 1), (1, 0, 1), (1, 1, 1)])


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("bc", [DIRICHLET, NEUMANN])
def test_vandermonde_first_row(dim, bc):
    rng = np.random.default_rng(7 + dim + 10 * bc)
    for _ in range(200):
        e = rng.choice([-1.0, 1.0], size=dim)
        r = rng.integers(1, 3, size=dim)
        h = rng.uniform(0.5, 2.0, size=dim)
        x2 = e * r * h
        n = rng.normal(size=dim)
        n /= np.linalg.norm(n)
        psi = rng.uniform(-0.5, 0.9) * h.min()
        xs = psi * n
        V = np.array([_basis(dim, np.array(s) * x2) for s in _subsets(dim)] +
                     [_basis(dim, xs) if bc == DIRICHLET else _basis_grad(dim, xs).T @ n])
        if np.linalg.cond(V) > 1e8:
            continue
        row = np.linalg.inv(V)[0]
        w, ws = oracle.weights_raw(dim, bc, x2, xs, n)
        assert np.allclose(w, row[:-1], rtol=1e-9, atol=1e-9 * np.abs(row).max())
        assert abs(ws - row[-1]) <= 1e-9 * max(1.0, abs(row[-1]))


def test_3d_weights_reduce_to_2d():
    """With n_z = 0 and x_s on the ghost's z plane, the trilinear relations
    give the bilinear ones on (P1, P2, P4) and zero weight on z-displaced
    points (Sec. 5.1 remark, Sec. 3.2)."""
    rng = np.random.default_rng(3)
    for _ in range(100):
        e = rng.choice([-1.0, 1.0], size=2)
        h = rng.uniform(0.5, 2.0, size=3)
        th = rng.uniform(0, 2 * np.pi)
        n2 = np.array([math.cos(th), math.sin(th)])
        psi = rng.uniform(-0.4, 0.9) * h[:2].min()
        x2 = np.r_[e * h[:2], h[2]]
        xs = np.r_[psi * n2, 0.0]
        for bc in (DIRICHLET, NEUMANN):
            w3, ws3 = oracle.weights_raw(3, bc, x2, xs, np.r_[n2, 0.0])
            w2, ws2 = oracle.weights_raw(2, bc, x2[:2], xs[:2], n2)
            assert np.allclose([w3[0], w3[1], w3[3]], w2, rtol=1e-12, atol=1e-12)
            assert np.allclose([w3[2], w3[4], w3[5], w3[6]], 0.0, atol=0)
            assert abs(ws3 - ws2) <= 1e-12 * max(1, abs(ws2))


def test_zero_normal_reduces_to_1d():
    """n_x = 0: Dirichlet is the 1D linear extrapolation through P2 and S,
    Neumann is phi_G = phi_P2 - h dphi/dn (Sec. 4.1 note)."""
    h = 0.37
    for ny in (1.0, -1.0):
        for psi in (0.1, 0.3, -0.2):
            x2 = np.array([h, ny * h])
            xs = np.array([0.0, psi * ny])
            w, ws = oracle.weights_raw(2, DIRICHLET, x2, xs, np.array([0.0, ny]))
            # phi_G = phi_s + (phi_2 - phi_s) * (0 - y_s)/(y_2 - y_s)
            lam = (0 - xs[1]) / (x2[1] - xs[1])
            assert w[0] == 0 and w[2] == 0
            assert abs(w[1] - lam) < 1e-15 and abs(ws - (1 - lam)) < 1e-15
            w, ws = oracle.weights_raw(2, NEUMANN, x2, xs, np.array([0.0, ny]))
            assert w[0] == 0 and w[2] == 0 and w[1] == 1.0
            assert abs(ws - (-h)) < 1e-15


# ---------------------------------------------------------------------------
# polynomial reproduction (Sec. 4, 5, 6): exact for (bi/tri)linear fields
# ---------------------------------------------------------------------------

def _bc_from_plan(p, flds, kinds):
    S = ghost_centres(p) + p.delta
    return np.stack([synth.bc_values(f, S, p.normal, k) for f, k in zip(flds, kinds)])


def ghost_centres(p):
    g = p.grid
    c = p.ghost_cell
    idx = [c % g.n[0], (c // g.n[0]) % g.n[1]]
    if p.dim == 3:
        idx.append(c // (g.n[0] * g.n[1]))
    return np.stack([g.lo[i] + (idx[i] + 0.5) * g.h[i] for i in range(p.dim)])


def _plans_2d():
    inst = synth.circle128(seed=1)
    star = synth.stars64(seed=0, ninst=2, nmin=96, nmax=160)
    return [(inst.grid, inst.shape), (star[0].grid, star[0].shape), (star[1].grid, star[1].shape)]


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_exact_bilinear_2d(scheme):
    rng = np.random.default_rng(11 + scheme)
    for grid, shape in _plans_2d():
        p = oracle.OraclePlan(grid, shape, scheme)
        C = rng.normal(size=4)
        for bc in (DIRICHLET, NEUMANN):
            fld = synth.polynomial_field(2, C, bc)
            exact = synth.sample(fld, grid)
            phi = exact.copy()
            phi[p.tags != 0] = np.nan            # ghosts and solid cells poisoned
            b = _bc_from_plan(p, [fld], [bc])
            out = p.fill(phi[None], [bc], b)[0]
            sc = p.fill_scale(exact[None], [bc], b)[0]
            err = np.abs(out[p.ghost_cell] - exact[p.ghost_cell])
            assert np.all(err <= 1e-12 * np.maximum(sc, 1.0)), err.max()
            # boundary value and gradient at S from the same polynomial
            val, grad = p.surface_ghost(out[None])
            S = ghost_centres(p) + p.delta
            assert np.allclose(val[0], fld.f(*S), rtol=0, atol=1e-11 * np.abs(exact).max())
            gexact = np.stack(fld.grad(*S))
            assert np.allclose(grad[0], gexact, rtol=0, atol=1e-9 * np.abs(gexact).max())


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_exact_trilinear_3d(scheme):
    rng = np.random.default_rng(21 + scheme)
    cases = [synth.sphere256(seed=2, n=48), synth.shstar384(seed=1, n=40, nt=4, nph=8)]
    for inst in cases:
        p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
        C = rng.normal(size=8)
        for bc in (DIRICHLET, NEUMANN):
            fld = synth.polynomial_field(3, C, bc)
            exact = synth.sample(fld, inst.grid)
            phi = exact.copy()
            phi[p.tags != 0] = np.nan
            b = _bc_from_plan(p, [fld], [bc])
            out = p.fill(phi[None], [bc], b)[0]
            sc = p.fill_scale(exact[None], [bc], b)[0]
            err = np.abs(out[p.ghost_cell] - exact[p.ghost_cell])
            assert np.all(err <= 1e-12 * np.maximum(sc, 1.0)), err.max()
            val, grad = p.surface_ghost(out[None])
            S = ghost_centres(p) + p.delta
            assert np.allclose(val[0], fld.f(*S), rtol=0, atol=1e-11 * np.abs(exact).max())
            gexact = np.stack(fld.grad(*S))
            assert np.allclose(grad[0], gexact, rtol=0, atol=1e-9 * np.abs(gexact).max())


def test_query_points_exact_bilinear():
    inst = synth.circle128(seed=3)
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    fld = synth.polynomial_field(2, [0.3, -1.2, 0.7, 2.1], DIRICHLET)
    exact = synth.sample(fld, inst.grid)
    phi = exact.copy()
    phi[p.tags != 0] = np.nan
    out = p.fill(phi[None], [DIRICHLET], _bc_from_plan(p, [fld], [DIRICHLET]))
    val, grad, anchor = p.surface_query(inst.queries.x, out)
    assert np.allclose(val[0], fld.f(*inst.queries.x), atol=1e-12)
    assert np.allclose(grad[0], np.stack(fld.grad(*inst.queries.x)), atol=1e-10)
    # the anchor is the ghost whose S is nearest (brute force over all ghosts)
    S = ghost_centres(p) + p.delta
    for q in range(0, inst.queries.x.shape[1], 17):
        d2 = ((S - inst.queries.x[:, q:q + 1]) ** 2).sum(0)
        assert d2[anchor[q]] <= d2.min() + 1e-15


# ---------------------------------------------------------------------------
# Sec. 3.2: dependency graph and levels
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_levels_are_longest_paths(scheme):
    for grid, shape in _plans_2d()[:2] + [(synth.sphere256(seed=0, n=40).grid,
                                           synth.sphere256(seed=0, n=40).shape)]:
        p = oracle.OraclePlan(grid, shape, scheme)
        pos = {int(c): k for k, c in enumerate(p.ghost_cell)}
        for k in range(p.n_ghost):
            deps = [pos[int(c)] for c in p.stencil(k) if c >= 0 and int(c) in pos]
            if p.unit[k] >= 0:   # coupled unit: edges leaving the unit count
                mates = np.where(p.unit == p.unit[k])[0]
                deps = [pos[int(c)] for m in mates for c in p.stencil(m)
                        if c >= 0 and int(c) in pos and p.unit[pos[int(c)]] != p.unit[k]]
            want = 1 + max((p.level[d] for d in deps), default=0)
            assert p.level[k] == want
        # canonical order: level ascending, linear index ascending in a level
        assert np.all(np.diff(p.level) >= 0)
        for l in range(p.n_levels):
            seg = p.ghost_cell[p.level_off[l]:p.level_off[l + 1]]
            assert np.all(np.diff(seg) > 0)
            assert np.all(p.level[p.level_off[l]:p.level_off[l + 1]] == l + 1)


@pytest.mark.parametrize("scheme", [CGC, HGC])
def test_jacobi_needs_exactly_n_sweeps(scheme):
    """Synchronous sweeps need as many sweeps as there are levels, and reach
    the level-by-level values bit for bit (Sec. 3.2)."""
    inst = synth.circle128(seed=4)
    p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    u = synth.sample(inst.fields[0], inst.grid)
    b = _bc_from_plan(p, inst.fields, [DIRICHLET])
    lev = p.fill(u[None], [DIRICHLET], b)
    jac, sweeps = p.fill_jacobi(u[None], [DIRICHLET], b)
    assert sweeps == p.n_levels
    assert np.array_equal(lev, jac)


def _cyclic_star():
    """A star whose concave valley puts two CGC ghosts in a 2-cycle."""
    inst = synth.stars64(seed=0, ninst=1, nmin=96, nmax=160)[0]
    return inst


def test_cycle_units_solve_the_coupled_system():
    """Where two ghosts read each other (concave valley), the unit's value is
    the solution of the coupled relations: equal to a dense solve of the
    whole ghost system (numpy), for both boundary-condition types."""
    inst = _cyclic_star()
    for scheme in (CGC, HGC):
        p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
        assert p.n_units_coupled >= 1 and p.max_unit == 2
        u = synth.sample(inst.fields[0], inst.grid)
        for bc in (DIRICHLET, NEUMANN):
            b = _bc_from_plan(p, inst.fields[:1], [bc])[0]
            x = _dense_solve(p, u, b, bc)
            out = p.fill(u[None], [bc], b[None])[0]
            assert np.allclose(out[p.ghost_cell], x, rtol=1e-12, atol=1e-12)


def _dense_solve(p, u, b, bc):
    ng = p.n_ghost
    pos = {int(c): k for k, c in enumerate(p.ghost_cell)}
    A = np.eye(ng)
    rhs = np.zeros(ng)
    for g in range(ng):
        w, ws = p.weights(g, bc)
        rhs[g] = ws * b[g]
        for wk, c in zip(w, p.stencil(g)):
            if c < 0:
                continue
            if int(c) in pos:
                A[g, pos[int(c)]] -= wk
            else:
                rhs[g] += wk * u[c]
    return np.linalg.solve(A, rhs)


def test_dense_solve_equals_level_fill():
    """The coupled ghost system solved as one dense linear system (numpy)
    equals the level-by-level substitution (Sec. 3.2)."""
    inst = synth.circle128(seed=5)
    p = oracle.OraclePlan(inst.grid, inst.shape, CGC)
    u = synth.sample(inst.fields[0], inst.grid)
    for bc in (DIRICHLET, NEUMANN):
        b = _bc_from_plan(p, inst.fields, [bc])[0]
        ng = p.n_ghost
        pos = {int(c): k for k, c in enumerate(p.ghost_cell)}
        A = np.eye(ng)
        rhs = np.zeros(ng)
        for g in range(ng):
            w, ws = p.weights(g, bc)
            rhs[g] = ws * b[g]
            for wk, c in zip(w, p.stencil(g)):
                if c < 0:
                    continue
                if int(c) in pos:
                    A[g, pos[int(c)]] -= wk
                else:
                    rhs[g] += wk * u[c]
        x = np.linalg.solve(A, rhs)
        out = p.fill(u[None], [bc], b[None])[0]
        assert np.allclose(out[p.ghost_cell], x, rtol=1e-12, atol=1e-12)


def test_alpha_bounds():
    """HGC and CGC_ES keep alpha <= 1/2 (Eq. HGC_criterion with Eq. delta_n;
    Eq. stencil_anisotropic); CGC does not on a generic circle."""
    for seed in range(3):
        inst = synth.circle128(seed=seed)
        a = {s: oracle.OraclePlan(inst.grid, inst.shape, s).margins["max_alpha"].max()
             for s in (CGC, CGC_ES, HGC)}
        assert a[HGC] <= 0.5 and a[CGC_ES] <= 0.5
        assert a[CGC] > 0.77
    inst = synth.sphere256(seed=1, n=48)
    for s in (CGC_ES, HGC):
        assert oracle.OraclePlan(inst.grid, inst.shape, s).margins["max_alpha"].max() <= 0.5


def test_hgc_closure():
    """After HGC reclassification no fluid cell (0) touches a solid cell (1)
    across a face: the signed distance is 1-Lipschitz (Sec. 3.1)."""
    for inst in (synth.circle128(seed=0), synth.stars64(seed=1, ninst=1, nmin=200, nmax=300)[0]):
        p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
        T = p.tags.reshape(inst.grid.n[1], inst.grid.n[0])
        assert not np.any((T[:, 1:] == 0) & (T[:, :-1] == 1))
        assert not np.any((T[:, 1:] == 1) & (T[:, :-1] == 0))
        assert not np.any((T[1:, :] == 0) & (T[:-1, :] == 1))
        assert not np.any((T[1:, :] == 1) & (T[:-1, :] == 0))


def test_zero_normal_ghosts_skip_points():
    """Circle centred on a cell centre: ghosts on its axes have n_i = 0
    exactly; their displaced points get weight 0 and are not read (Sec. 3.2),
    so NaN there leaves the fill finite."""
    h = 1.0 / 32
    grid = synth.Grid(2, (128, 128, 1), (-2.0, -2.0, 0.0), (h, h, 1.0))
    c = (-2.0 + 64.5 * h, -2.0 + 64.5 * h, 0.0)
    p = oracle.OraclePlan(grid, synth.Shape(synth.SPHERE, c, 0.5), HGC)
    zero = np.where((p.normal == 0.0).any(axis=0))[0]
    assert len(zero) >= 4
    for g in zero:
        st = p.stencil(g)
        ax = int(np.where(p.normal[:, g] == 0.0)[0][0])
        skipped = [k for k, sb in enumerate(_subsets(2)) if sb[ax]]
        assert all(st[k] == -1 for k in skipped)
    f = synth.polynomial_field(2, [1.0, 0.5, -0.25, 0.1], DIRICHLET)
    u = synth.sample(f, grid)
    u[p.tags == 1] = np.nan
    out = p.fill(u[None], [DIRICHLET], _bc_from_plan(p, [f], [DIRICHLET]))[0]
    assert np.all(np.isfinite(out[p.ghost_cell]))


# ---------------------------------------------------------------------------
# geometry (Sec. 3.1): closest point and analytic normal
# ---------------------------------------------------------------------------

def test_star_closest_point_bruteforce():
    inst = synth.stars64(seed=2, ninst=1, nmin=400, nmax=400)[0]
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    th = np.linspace(0, 2 * np.pi, 400001)[:-1]
    r, dr = synth.star_radius(inst.shape, th)
    c = inst.shape.center
    curve = np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th)])
    xc = ghost_centres(p)
    S = xc + p.delta
    ds = np.hypot(*np.diff(curve, axis=1)).max()   # sample spacing
    for g in range(0, p.n_ghost, max(1, p.n_ghost // 60)):
        d = np.sqrt(((curve - xc[:, g:g + 1]) ** 2).sum(0)).min()
        assert abs(p.psi[g]) <= d + 1e-14             # never beaten by samples
        assert d * d <= p.psi[g] ** 2 + 1.01 * (ds / 2) ** 2   # within sampling
        # S on the curve, (x - S) along the normal
        ths = math.atan2(S[1, g] - c[1], S[0, g] - c[0])
        rs, _ = synth.star_radius(inst.shape, np.array([ths]))
        assert abs(math.hypot(S[0, g] - c[0], S[1, g] - c[1]) - rs[0]) < 1e-13
        v = xc[:, g] - S[:, g]
        assert abs(v[0] * p.normal[1, g] - v[1] * p.normal[0, g]) < 1e-13


def test_airfoil_closest_point_bruteforce():
    """Four-digit closed-trailing-edge contour (x = s^2 parametrisation):
    no dense contour sample is nearer than |psi|, S lies on the contour,
    and away from the trailing-edge corner (x - S) is along the normal."""
    inst = synth.airfoil4096(seed=1, n=512, m=64)
    sh = inst.shape
    p = oracle.OraclePlan(inst.grid, sh, HGC)
    s = np.linspace(-1.0, 1.0, 2_000_001)
    s2 = s * s
    yt = 5 * sh.thick * (0.2969 * np.abs(s) - (0.1260 * s2 + 0.3516 * s2 ** 2
                                                - 0.2843 * s2 ** 3 + 0.1036 * s2 ** 4))
    bx, by = s2, np.sign(s) * yt
    ca, sa = math.cos(sh.incidence), math.sin(sh.incidence)
    le = sh.center
    curve = np.stack([le[0] + sh.chord * (ca * bx + sa * by),
                      le[1] + sh.chord * (-sa * bx + ca * by)])
    ds = np.hypot(*np.diff(curve, axis=1)).max()
    xc = ghost_centres(p)
    S = xc + p.delta
    te = curve[:, -1]
    for g in range(0, p.n_ghost, max(1, p.n_ghost // 80)):
        d = np.sqrt(((curve - xc[:, g:g + 1]) ** 2).sum(0)).min()
        assert abs(p.psi[g]) <= d + 1e-14
        assert d * d <= p.psi[g] ** 2 + 1.01 * (ds / 2) ** 2
        dx, dy = (S[0, g] - le[0]) / sh.chord, (S[1, g] - le[1]) / sh.chord
        b0, b1 = ca * dx - sa * dy, sa * dx + ca * dy
        yb = 5 * sh.thick * (0.2969 * math.sqrt(max(b0, 0.0)) - 0.1260 * b0 - 0.3516 * b0 ** 2
                             + 0.2843 * b0 ** 3 - 0.1036 * b0 ** 4)
        assert abs(abs(b1) - yb) < 1e-12
        if np.hypot(*(S[:, g] - te)) > 1e-12:
            v = xc[:, g] - S[:, g]
            assert abs(v[0] * p.normal[1, g] - v[1] * p.normal[0, g]) < 1e-13


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(0)
    for _ in range(20):
        v = rng.normal(size=3)
        ct = v[2] / np.linalg.norm(v)
        ph = math.atan2(v[1], v[0])
        for l in range(5):
            for m in range(-l, l + 1):
                ref = synth.workloads._sh_real_schmidt(l, m, np.array([ct]), np.array([ph]))[0]
                assert abs(oracle.sh_basis(l, m, v) - ref) < 1e-13


def test_sh_closest_point():
    inst = synth.shstar384(seed=0, n=64, nt=4, nph=8)
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    xc = ghost_centres(p)
    S = xc + p.delta
    c = np.asarray(inst.shape.center)[:, None]
    v = S - c
    rr = np.linalg.norm(v, axis=0)
    ct = v[2] / rr
    ph = np.arctan2(v[1], v[0])
    assert np.allclose(rr, synth.sh_radius(inst.shape, ct, ph), atol=1e-13)
    d = xc - S
    cross = np.cross(d.T, p.normal.T)
    assert np.abs(cross).max() < 1e-13
    # local brute force: no surface sample nearer than |psi|
    rng = np.random.default_rng(1)
    for g in rng.choice(p.n_ghost, 20, replace=False):
        om = v[:, g] / rr[g]
        t1 = np.cross(om, [1.0, 0, 0]) if abs(om[0]) < 0.9 else np.cross(om, [0, 1.0, 0])
        t1 /= np.linalg.norm(t1)
        t2 = np.cross(om, t1)
        a, b = np.meshgrid(np.linspace(-0.05, 0.05, 201), np.linspace(-0.05, 0.05, 201))
        w = om[:, None] + a.ravel() * t1[:, None] + b.ravel() * t2[:, None]
        w /= np.linalg.norm(w, axis=0)
        pts = c + synth.sh_radius(inst.shape, w[2], np.arctan2(w[1], w[0])) * w
        dmin = np.sqrt(((pts - xc[:, g:g + 1]) ** 2).sum(0)).min()
        assert abs(p.psi[g]) <= dmin + 1e-14


# ---------------------------------------------------------------------------
# forces (Sec. 6): closed forms for exactly reproduced fields
# ---------------------------------------------------------------------------

def test_forces_closed_forms_circle():
    """p = x gives F = -(pi R^2, 0) (divergence theorem); u = (xy, 0) gives
    F = (0, mu pi R^2); both fields are bilinear, so reconstruction is exact,
    and the trapezoid rule is exact for the resulting trigonometric sums."""
    inst = synth.circle128(seed=6)
    R = inst.shape.r0
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    q = inst.queries
    x, y = inst.grid.mesh()

    def filled(fld, bc):
        v = synth.sample(fld, inst.grid)
        v[p.tags != 0] = np.nan
        return p.fill(v[None], [bc], _bc_from_plan(p, [fld], [bc]))[0]

    pf = filled(synth.polynomial_field(2, [0, 1, 0, 0], NEUMANN), NEUMANN)
    ux = filled(synth.polynomial_field(2, [0, 0, 0, 1], DIRICHLET), DIRICHLET)
    zero = filled(synth.polynomial_field(2, [0, 0, 0, 0], DIRICHLET), DIRICHLET)
    F = p.forces(q.x, q.n, q.w, pf, np.stack([zero, zero]), 1.0)
    assert np.allclose(F, [-math.pi * R * R, 0.0], atol=1e-12)
    mu = 0.7
    F = p.forces(q.x, q.n, q.w, zero, np.stack([ux, zero]), mu)
    assert np.allclose(F, [0.0, mu * math.pi * R * R], atol=1e-12)


def test_forces_closed_form_sphere():
    inst = synth.sphere256(seed=3, n=48)
    R = inst.shape.r0
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    q = inst.queries
    fld = synth.polynomial_field(3, [0, 0, 0, 1, 0, 0, 0, 0], NEUMANN)   # p = z
    v = synth.sample(fld, inst.grid)
    v[p.tags != 0] = np.nan
    pf = p.fill(v[None], [NEUMANN], _bc_from_plan(p, [fld], [NEUMANN]))[0]
    zero = np.zeros((3, p.n_cells))
    F = p.forces(q.x, q.n, q.w, pf, zero, 1.0)
    assert np.allclose(F, [0, 0, -4.0 / 3.0 * math.pi * R ** 3], atol=1e-12)


# ---------------------------------------------------------------------------
# adjoint: exact transpose, and central differences of an affine functional
# ---------------------------------------------------------------------------

def _forward(p, inst, phi, b, kinds):
    out = p.fill(phi, kinds, b)
    val, grad, _ = p.surface_query(inst.queries.x, out)
    return val, grad


@pytest.mark.parametrize("which", ["circle", "shstar"])
def test_adjoint_dot_product(which):
    inst = synth.circle128(seed=7) if which == "circle" else synth.shstar384(seed=2, n=40, nt=4, nph=8)
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    rng = np.random.default_rng(5)
    nf = 2
    kinds = np.array([DIRICHLET, NEUMANN], np.int8)
    phi = rng.normal(size=(nf, p.n_cells))
    b = rng.normal(size=(nf, p.n_ghost))
    nq = inst.queries.x.shape[1]
    gv = rng.normal(size=(nf, nq))
    gg = rng.normal(size=(nf, p.dim, nq))
    val, grad = _forward(p, inst, phi, b, kinds)
    lhs = (gv * val).sum() + (gg * grad).sum()
    lam = p.surface_query_adjoint(inst.queries.x, gv, gg, np.zeros((nf, p.n_cells)))
    lam, lam_bc = p.fill_adjoint(lam, kinds)
    rhs = (lam * phi).sum() + (lam_bc * b).sum()
    assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + np.abs(lam * phi).sum())
    # overwritten ghost slots carry no sensitivity
    assert np.all(lam[:, p.ghost_cell] == 0)


def test_adjoint_central_differences():
    """J = drag-like functional is affine in (field, boundary data): central
    differences have no truncation error, only rounding (step 1e-6)."""
    inst = synth.circle128(seed=8)
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    rng = np.random.default_rng(9)
    kinds = np.array([DIRICHLET], np.int8)
    phi = synth.sample(inst.fields[0], inst.grid)[None].copy()
    b = _bc_from_plan(p, inst.fields, [DIRICHLET])
    nq = inst.queries.x.shape[1]
    gv = rng.normal(size=(1, nq))
    gg = rng.normal(size=(1, 2, nq))

    def J(phi_, b_):
        val, grad = _forward(p, inst, phi_, b_, kinds)
        return (gv * val).sum() + (gg * grad).sum()

    lam = p.surface_query_adjoint(inst.queries.x, gv, gg, np.zeros((1, p.n_cells)))
    lam, lam_bc = p.fill_adjoint(lam, kinds)
    support = np.where(lam[0] != 0)[0]
    eps = 1e-6
    for c in rng.choice(support, 8, replace=False):
        a, m = phi.copy(), phi.copy()
        a[0, c] += eps
        m[0, c] -= eps
        fd = (J(a, b) - J(m, b)) / (2 * eps)
        assert abs(fd - lam[0, c]) < 1e-7 * max(1.0, abs(lam[0, c]))
    for g in rng.choice(p.n_ghost, 8, replace=False):
        a, m = b.copy(), b.copy()
        a[0, g] += eps
        m[0, g] -= eps
        fd = (J(phi, a) - J(phi, m)) / (2 * eps)
        assert abs(fd - lam_bc[0, g]) < 1e-7 * max(1.0, abs(lam_bc[0, g]))


def test_dirichlet_surface_value_returns_datum():
    """After a Dirichlet fill the interpolant at S equals the imposed datum
    (Sec. 6: the Dirichlet relation rearranged)."""
    inst = synth.circle128(seed=9)
    for scheme in (CGC_ES, HGC):
        p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
        u = synth.sample(inst.fields[0], inst.grid)
        b = _bc_from_plan(p, inst.fields, [DIRICHLET])
        out = p.fill(u[None], [DIRICHLET], b)
        val, _ = p.surface_ghost(out)
        assert np.allclose(val, b, rtol=0, atol=1e-13)


def test_margins_of_standard_seeds():
    """Decisions (inside test, HGC band, multipliers, normal signs) sit far
    from their thresholds on the standard seeds, so any correct evaluation
    order takes the same decisions."""
    for seed in range(3):
        inst = synth.circle128(seed=seed)
        for scheme in (CGC, CGC_ES, HGC):
            assert oracle.OraclePlan(inst.grid, inst.shape, scheme).min_margin > 1e-9


@pytest.mark.parametrize("which", ["circle", "star", "shstar", "airfoil"])
def test_normals_point_into_fluid(which):
    """n is the unit normal pointing into the fluid (Sec. 3.1): a step along
    +n from S leaves the body, a step along -n enters it."""
    if which == "circle":
        inst = synth.circle128(seed=0)
    elif which == "star":
        inst = synth.stars64(seed=3, ninst=1, nmin=300, nmax=300)[0]
    elif which == "shstar":
        inst = synth.shstar384(seed=0, n=48, nt=4, nph=8)
    else:
        inst = synth.airfoil4096(seed=0, n=512, m=64)
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    S = ghost_centres(p) + p.delta
    eps = 1e-7
    for g in range(0, p.n_ghost, max(1, p.n_ghost // 100)):
        assert not oracle.inside(inst.shape, p.dim, S[:, g] + eps * p.normal[:, g])
        assert oracle.inside(inst.shape, p.dim, S[:, g] - eps * p.normal[:, g])
        assert abs(np.linalg.norm(p.normal[:, g]) - 1) < 1e-14
    if which in ("circle", "star", "airfoil"):
        q = inst.queries
        for k in range(0, q.x.shape[1], max(1, q.x.shape[1] // 50)):
            assert not oracle.inside(inst.shape, p.dim, q.x[:, k] + 1e-6 * q.n[:, k])
