"""Pins of the oracle on stretched grids: cell faces given per axis, cell
centres midway between faces, and the local spacing of a cell (its width)
in Eq. delta_n and Eq. stencil_anisotropic; stencil spans x_2 - x_1 are
differences of cell centres.  The flows of Secs. 8.1 and 8.2 run on grids
uniform near the body and stretched by a fixed ratio toward the outer
boundaries; Sec. 7.1 takes the spacing in both equations as the local one.

Expected values come from brute force with the circle's closed-form
distance, polynomial reproduction (exact for any spacing), the level
properties of Sec. 3.2, and the uniform grid as the ratio-1 special case."""
import numpy as np
import pytest

import oracle
import synth
from synth import CGC, CGC_ES, HGC, LAYER2, DIRICHLET, NEUMANN


def ghost_centres(p):
    g = p.grid
    c = p.ghost_cell
    idx = [c % g.n[0], (c // g.n[0]) % g.n[1]]
    if p.dim == 3:
        idx.append(c // (g.n[0] * g.n[1]))
    return np.stack([g.centres(i)[idx[i]] for i in range(p.dim)])


def brute_force_circle(grid, centre, R, scheme, layer2=False):
    X, Y = grid.centres(0) - centre[0], grid.centres(1) - centre[1]
    WX, WY = grid.widths(0), grid.widths(1)
    x, y = np.meshgrid(X, Y)
    wx, wy = np.meshgrid(WX, WY)
    rho = np.hypot(x, y)
    psi = R - rho
    n = np.stack([x / rho, y / rho])
    dn = 1.0 / np.sqrt((n[0] / wx) ** 2 + (n[1] / wy) ** 2)   # Eq. delta_n, local widths
    solid = psi >= 0
    other = np.zeros_like(solid)
    other[:, 1:] |= solid[:, 1:] != solid[:, :-1]
    other[:, :-1] |= solid[:, :-1] != solid[:, 1:]
    other[1:, :] |= solid[1:, :] != solid[:-1, :]
    other[:-1, :] |= solid[:-1, :] != solid[1:, :]
    tags = solid.astype(np.int8)
    if scheme == HGC:
        tags[solid & other & (psi <= dn / 2)] = 2
        tags[~solid & other & (-psi < dn / 2)] = -2
    else:
        tags[solid & other] = 2
    # second layer (Sec. 7.1): every other solid cell with psi <= 1.5 delta n,
    # on the extended stencil
    added = solid & (tags != 2) & (psi <= 1.5 * dn) if layer2 else np.zeros_like(solid)
    tags[added] = 2
    r = np.ones((2,) + psi.shape, np.int64)
    ext = (tags == 2) if scheme == CGC_ES else added
    for a, w in ((0, wx), (1, wy)):
        q = np.maximum(1, np.ceil(2 * np.abs(psi * n[a]) / w)).astype(np.int64)
        r[a][ext] = q[ext]
    return tags.ravel(), r.reshape(2, -1)


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
@pytest.mark.parametrize("seed", [0, 1])
def test_stretched_tags_brute_force(scheme, seed):
    inst = synth.circle_stretched(seed=seed)
    p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    assert p.min_margin > 1e-9
    tags, r = brute_force_circle(inst.grid, inst.shape.center, inst.shape.r0, scheme)
    assert np.array_equal(p.tags, tags)
    assert np.array_equal(p.r, r[:, p.ghost_cell])


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_stretched_exact_bilinear_and_trilinear(scheme):
    rng = np.random.default_rng(41 + scheme)
    for dim, inst in ((2, synth.circle_stretched(seed=2)), (3, synth.sphere_stretched(seed=1))):
        p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
        C = rng.normal(size=4 if dim == 2 else 8)
        for bc in (DIRICHLET, NEUMANN):
            fld = synth.polynomial_field(dim, C, bc)
            exact = synth.sample(fld, inst.grid)
            phi = exact.copy()
            phi[p.tags != 0] = np.nan
            S = ghost_centres(p) + p.delta
            b = synth.bc_values(fld, S, p.normal, bc)[None]
            out = p.fill(phi[None], [bc], b)[0]
            sc = p.fill_scale(exact[None], [bc], b)[0]
            err = np.abs(out[p.ghost_cell] - exact[p.ghost_cell])
            assert np.all(err <= 1e-12 * np.maximum(sc, 1.0)), err.max()
            val, grad = p.surface_ghost(out[None])
            assert np.allclose(val[0], fld.f(*S), rtol=0, atol=1e-11 * np.abs(exact).max())
            gexact = np.stack(fld.grad(*S))
            assert np.allclose(grad[0], gexact, rtol=0, atol=1e-9 * np.abs(gexact).max())


def test_stretched_query_points_exact_and_anchor():
    inst = synth.circle_stretched(seed=3)
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    fld = synth.polynomial_field(2, [0.3, -1.2, 0.7, 2.1], DIRICHLET)
    exact = synth.sample(fld, inst.grid)
    phi = exact.copy()
    phi[p.tags != 0] = np.nan
    S = ghost_centres(p) + p.delta
    out = p.fill(phi[None], [DIRICHLET], synth.bc_values(fld, S, p.normal, DIRICHLET)[None])
    val, grad, anchor = p.surface_query(inst.queries.x, out)
    assert np.allclose(val[0], fld.f(*inst.queries.x), atol=1e-12)
    assert np.allclose(grad[0], np.stack(fld.grad(*inst.queries.x)), atol=1e-10)
    for q in range(0, inst.queries.x.shape[1], 13):
        d2 = ((S - inst.queries.x[:, q:q + 1]) ** 2).sum(0)
        assert d2[anchor[q]] <= d2.min() + 1e-15


@pytest.mark.parametrize("scheme", [CGC, HGC])
def test_stretched_levels(scheme):
    inst = synth.circle_stretched(seed=4)
    p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    pos = {int(c): k for k, c in enumerate(p.ghost_cell)}
    for k in range(p.n_ghost):
        deps = [pos[int(c)] for c in p.stencil(k) if c >= 0 and int(c) in pos]
        if p.unit[k] >= 0:
            mates = np.where(p.unit == p.unit[k])[0]
            deps = [pos[int(c)] for m in mates for c in p.stencil(m)
                    if c >= 0 and int(c) in pos and p.unit[pos[int(c)]] != p.unit[k]]
        assert p.level[k] == 1 + max((p.level[d] for d in deps), default=0)
    u = synth.sample(inst.fields[0], inst.grid)
    S = ghost_centres(p) + p.delta
    b = synth.bc_values(inst.fields[0], S, p.normal, DIRICHLET)[None]
    lev = p.fill(u[None], [DIRICHLET], b)
    jac, sweeps = p.fill_jacobi(u[None], [DIRICHLET], b)
    assert sweeps == p.n_levels
    assert np.array_equal(lev, jac)


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_ratio_one_is_the_uniform_grid(scheme):
    """Faces of a uniform grid give the uniform plan: same tags, ghosts,
    levels and multipliers, geometry equal to rounding."""
    inst = synth.circle128(seed=2)
    g = inst.grid
    faces = tuple(g.lo[a] + g.h[a] * np.arange(g.n[a] + 1) for a in range(2)) + (None,)
    gs = synth.Grid(2, g.n, g.lo, g.h, faces)
    pu = oracle.OraclePlan(g, inst.shape, scheme)
    ps = oracle.OraclePlan(gs, inst.shape, scheme)
    assert np.array_equal(pu.tags, ps.tags)
    assert np.array_equal(pu.ghost_cell, ps.ghost_cell)
    assert np.array_equal(pu.level, ps.level)
    assert np.array_equal(pu.r, ps.r)
    assert np.allclose(pu.delta, ps.delta, rtol=0, atol=1e-14)


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
@pytest.mark.parametrize("seed", [0, 1])
def test_stretched_second_layer_brute_force(scheme, seed):
    """The second layer on a stretched grid: delta n and the multipliers
    from local widths, the set by brute force over every cell."""
    inst = synth.circle_stretched(seed=seed)
    p = oracle.OraclePlan(inst.grid, inst.shape, scheme | LAYER2)
    assert p.min_margin > 1e-9
    tags, r = brute_force_circle(inst.grid, inst.shape.center, inst.shape.r0, scheme, layer2=True)
    assert np.array_equal(p.tags, tags)
    assert np.array_equal(p.r, r[:, p.ghost_cell])
    p1 = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    assert p.n_ghost > p1.n_ghost
    assert set(p1.ghost_cell.tolist()) <= set(p.ghost_cell.tolist())


def test_stretched_second_layer_alpha_and_exactness():
    """On the extended stencil |x_1,i - x_s,i| / (r_i dx_i) <= 1/2 with the
    local width dx_i (the bound below Eq. stencil_anisotropic); bilinear and
    trilinear fields reproduced to rounding; levels as longest paths."""
    rng = np.random.default_rng(53)
    for dim, inst in ((2, synth.circle_stretched(seed=2)), (3, synth.sphere_stretched(seed=1))):
        g = inst.grid
        for scheme in (CGC, HGC):
            p = oracle.OraclePlan(g, inst.shape, scheme | LAYER2)
            p1 = oracle.OraclePlan(g, inst.shape, scheme)
            first = set(p1.ghost_cell.tolist())
            ext = np.array([int(c) not in first for c in p.ghost_cell])
            assert ext.any()
            c = p.ghost_cell
            idx = [c % g.n[0], (c // g.n[0]) % g.n[1]] + ([c // (g.n[0] * g.n[1])] if dim == 3 else [])
            w = np.stack([g.widths(a)[idx[a]] for a in range(dim)])
            alpha = np.abs(p.delta) / (p.r * w)
            assert np.all(alpha[:, ext] <= 0.5 + 1e-15)
            C = rng.normal(size=4 if dim == 2 else 8)
            for bc in (DIRICHLET, NEUMANN):
                fld = synth.polynomial_field(dim, C, bc)
                exact = synth.sample(fld, g)
                phi = exact.copy()
                phi[p.tags != 0] = np.nan
                S = ghost_centres(p) + p.delta
                b = synth.bc_values(fld, S, p.normal, bc)[None]
                out = p.fill(phi[None], [bc], b)[0]
                sc = p.fill_scale(exact[None], [bc], b)[0]
                err = np.abs(out[c] - exact[c])
                assert np.all(err <= 1e-12 * np.maximum(sc, 1.0)), err.max()
            pos = {int(x): k for k, x in enumerate(c)}
            for k in range(p.n_ghost):
                if p.unit[k] >= 0:
                    continue
                deps = [pos[int(x)] for x in p.stencil(k) if x >= 0 and int(x) in pos]
                assert p.level[k] == 1 + max((p.level[d] for d in deps), default=0)
