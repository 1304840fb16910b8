"""Pins of the oracle's tolerance machinery.

Every GPU parity test accepts |y - y*| <= 1e-12 max(|y*|, s), with s the
oracle's condition-aware scale of y*.  A mistake that inflates s would
loosen every such test without turning any red, so the scales are pinned
here against independent recomputations in numpy:

  * weight bounds: wb_k = |w_k| + sum_i (|x2_i| |dw_k/dxs_i| + |dw_k/dn_i|)
    (each side projects the body on its own, so the foot point and normal
    agree to a fraction of a cell, not bit for bit), against complex-step
    derivatives of the first row of the inverted Appendix A system;
  * fill scale (propagated through the levels of Sec. 3.2): s_G = sum_k
    wb_k s_{P_k} + wsb |b_G|, s = |phi| on cells that are not ghosts, a
    coupled unit's members |A^-1| times their external sums;
  * surface scale (Sec. 6): sum over the anchor box's corners of |L_c(x)|
    (value) or |d L_c / dx_i| (gradient) times the corner scales, with the
    tensor-product Lagrange basis written out here from the box geometry;
  * adjoint scales: the reverse sweep on magnitudes, units by |A^-T|.

Besides equality with the recomputation, two properties that hold whatever
the arithmetic: a scale bounds the magnitude of its value (triangle
inequality), and, for the Dirichlet relation with every normalised distance
|alpha_i| <= 1/2 (HGC and CGC_ES, Sec. 8), each |omega_i| <= 1 and
|x2_i d omega_i / dxs_i| = 1 / (1 - alpha_i)^2 <= 4, which bounds the
weights and their bounds by constants.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import CGC, CGC_ES, HGC, DIRICHLET, NEUMANN


def _cases():
    return [("circle", synth.circle128(seed=1)),
            ("sphere", synth.sphere256(seed=2, n=40)),
            ("star", synth.stars64(seed=0, ninst=1, nmin=96, nmax=160)[0])]


def ghost_centres(p):
    g = p.grid
    c = p.ghost_cell
    idx = [c % g.n[0], (c // g.n[0]) % g.n[1]]
    if p.dim == 3:
        idx.append(c // (g.n[0] * g.n[1]))
    return np.stack([g.lo[i] + (idx[i] + 0.5) * g.h[i] for i in range(p.dim)])


def _inputs(p, inst, bc, rng):
    """Random interior values (solid and ghost slots NaN) and boundary data:
    magnitudes of both signs, so a missing |.| shows."""
    phi = rng.normal(size=p.n_cells)
    phi[p.tags != 0] = np.nan
    b = rng.normal(size=p.n_ghost)
    return phi, b


def _ghost_index(p):
    return {int(c): k for k, c in enumerate(p.ghost_cell)}


def _unit_members(p):
    units = {}
    for k in range(p.n_ghost):
        if p.unit[k] >= 0:
            units.setdefault(int(p.unit[k]), []).append(k)
    return units


def _unit_matrix(p, members, bc, pos):
    """A = I - (weights among the members) of one coupled unit."""
    k = len(members)
    A = np.eye(k)
    where = {m: i for i, m in enumerate(members)}
    for i, g in enumerate(members):
        w, _ = p.weights(g, bc)
        for wk, c in zip(w, p.stencil(g)):
            if c >= 0 and int(c) in pos and pos[int(c)] in where:
                A[i, where[pos[int(c)]]] -= wk
    return A


def numpy_fill_scale(p, phi, bc, b):
    pos = _ghost_index(p)
    units = _unit_members(p)
    s = np.full(p.n_ghost, np.nan)
    done = set()
    for g in range(p.n_ghost):
        if p.unit[g] >= 0:
            u = int(p.unit[g])
            if u in done:
                continue
            done.add(u)
            mem = units[u]
            ext = np.zeros(len(mem))
            for i, m in enumerate(mem):
                w, ws = p.weight_bounds(m, bc)
                ext[i] = ws * abs(b[m])
                for wk, c in zip(w, p.stencil(m)):
                    if c < 0:
                        continue
                    c = int(c)
                    if c in pos and pos[c] in mem:
                        continue
                    ext[i] += wk * (s[pos[c]] if c in pos else abs(phi[c]))
            s[mem] = np.abs(np.linalg.inv(_unit_matrix(p, mem, bc, pos))) @ ext
            continue
        w, ws = p.weight_bounds(g, bc)
        acc = ws * abs(b[g])
        for wk, c in zip(w, p.stencil(g)):
            if c >= 0:
                c = int(c)
                acc += wk * (s[pos[c]] if c in pos else abs(phi[c]))
        s[g] = acc
    return s


@pytest.mark.parametrize("name", ["circle", "sphere", "star"])
@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
@pytest.mark.parametrize("bc", [DIRICHLET, NEUMANN])
def test_fill_scale_recomputed(name, scheme, bc):
    inst = dict(_cases())[name]
    p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    rng = np.random.default_rng(100 + 7 * scheme + bc)
    phi, b = _inputs(p, inst, bc, rng)
    got = p.fill_scale(np.nan_to_num(phi)[None], [bc], b[None])[0]
    want = numpy_fill_scale(p, phi, bc, b)
    assert np.all(np.isfinite(want))
    assert np.allclose(got, want, rtol=1e-13, atol=0), np.abs(got - want).max()
    # the scale bounds the value it belongs to
    val = p.fill(phi[None], [bc], b[None])[0][p.ghost_cell]
    assert np.all(np.abs(val) <= got * (1 + 1e-13))
    if name == "star" and scheme == CGC:
        assert p.n_units_coupled >= 1     # the unit branch is exercised


@pytest.mark.parametrize("name", ["circle", "sphere", "star"])
@pytest.mark.parametrize("scheme", [CGC_ES, HGC])
def test_weights_and_bounds_under_the_alpha_bound(name, scheme):
    """Dirichlet with |alpha_i| <= 1/2 (Sec. 8): w_k = +-prod_{i in k}
    omega_i with |omega_i| <= 1, so sum_k |w_k| <= 2^d - 1 and |w_s| =
    prod |1 - omega_i| <= 2^d; with |x2_i d omega_i/dxs_i| <= 4 the bounds
    obey wb_k <= 1 + 4 |k| (|k| the directions of P_k) and wsb <= 2^d +
    d 4 2^(d-1), however the weights are computed."""
    inst = dict(_cases())[name]
    p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    assert np.all(p.margins["max_alpha"] <= 0.5)
    d = p.dim
    sizes = [1, 1, 2] if d == 2 else [1, 1, 1, 2, 2, 2, 3]
    for g in range(p.n_ghost):
        w, ws = p.weights(g, DIRICHLET)
        wb, wsb = p.weight_bounds(g, DIRICHLET)
        assert np.abs(w).sum() <= (2 ** d - 1) * (1 + 1e-14) and abs(ws) <= 2 ** d * (1 + 1e-14)
        assert np.all(wb >= np.abs(w)) and wsb >= abs(ws)
        assert np.all(wb <= 1 + 4 * np.array(sizes) + 1e-9), (g, wb)
        assert wsb <= 2 ** d + d * 4 * 2 ** (d - 1) + 1e-9, (g, wsb)


def _vandermonde_row(dim, bc, x2, xs, n):
    """First row of the inverse of the Appendix A system (complex allowed)."""
    def basis(x):
        if dim == 2:
            return np.array([1.0, x[0], x[1], x[0] * x[1]], dtype=complex)
        X, Y, Z = x
        return np.array([1.0, X, Y, Z, X * Y, Y * Z, X * Z, X * Y * Z], dtype=complex)

    def basis_dn(x, nn):
        if dim == 2:
            return np.array([0, nn[0], nn[1], nn[0] * x[1] + nn[1] * x[0]], dtype=complex)
        X, Y, Z = x
        return np.array([0, nn[0], nn[1], nn[2], nn[0] * Y + nn[1] * X, nn[1] * Z + nn[2] * Y,
                         nn[0] * Z + nn[2] * X,
                         nn[0] * Y * Z + nn[1] * X * Z + nn[2] * X * Y], dtype=complex)

    subsets = ([(1, 0), (0, 1), (1, 1)] if dim == 2 else
               [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (0, 1, 1), (1, 0, 1), (1, 1, 1)])
    rows = [basis(np.array(sb) * x2) for sb in subsets]
    rows.append(basis(xs) if bc == DIRICHLET else basis_dn(xs, n))
    return np.linalg.inv(np.array(rows))[0]


def _complex_step_bounds(dim, bc, x2, xs, n):
    row = _vandermonde_row(dim, bc, x2, xs.astype(complex), n.astype(complex)).real
    wb = np.abs(row)
    step = 1e-30
    for i in range(dim):
        for which in (0, 1):
            a = xs.astype(complex)
            b = n.astype(complex)
            (a if which == 0 else b)[i] += 1j * step
            der = _vandermonde_row(dim, bc, x2, a, b).imag / step
            wb += (abs(x2[i]) if which == 0 else 1.0) * np.abs(der)
    return wb[:-1], wb[-1]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("bc", [DIRICHLET, NEUMANN])
def test_weight_bounds_complex_step(dim, bc):
    rng = np.random.default_rng(40 + dim + 10 * bc)
    done = 0
    for _ in range(300):
        e = rng.choice([-1.0, 1.0], size=dim)
        r = rng.integers(1, 3, size=dim)
        h = rng.uniform(0.5, 2.0, size=dim)
        x2 = e * r * h
        n = rng.normal(size=dim)
        n /= np.linalg.norm(n)
        xs = rng.uniform(-0.5, 0.9) * h.min() * n
        want, wants = _complex_step_bounds(dim, bc, x2, xs, n)
        if not np.all(np.isfinite(want)) or max(np.abs(want).max(), abs(wants)) > 1e6:
            continue      # near a degenerate configuration
        got, gots = oracle.weight_bounds_raw(dim, bc, x2, xs, n)
        assert np.allclose(got, want, rtol=1e-6, atol=1e-9 * max(1.0, np.abs(want).max()))
        assert abs(gots - wants) <= 1e-6 * abs(wants) + 1e-9
        done += 1
    assert done > 100


def test_weight_bounds_on_plan_ghosts():
    """The bounds of actual ghosts (CGC with alpha near 1, HGC fluid side,
    Neumann) against the complex-step values from the same local
    geometry."""
    inst = synth.stars64(seed=0, ninst=1, nmin=96, nmax=160)[0]
    for scheme in (CGC, HGC):
        p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
        h = np.asarray(inst.grid.h[:2])
        for g in range(0, p.n_ghost, 3):
            e = np.where(p.normal[:, g] >= 0, 1.0, -1.0)
            x2 = e * p.r[:, g] * h
            for bc in (DIRICHLET, NEUMANN):
                want, wants = _complex_step_bounds(2, bc, x2, p.delta[:, g], p.normal[:, g])
                got, gots = p.weight_bounds(g, bc)
                assert np.allclose(got, want, rtol=1e-6, atol=1e-12 * max(1.0, np.abs(want).max()))
                assert abs(gots - wants) <= 1e-6 * abs(wants) + 1e-12


def _box(p, a):
    """Corner cells of ghost a's stencil box and its spans X_i = e_i r_i h_i
    (every corner, displaced or not, on a uniform grid)."""
    g = p.grid
    d = p.dim
    c = int(p.ghost_cell[a])
    idx = [c % g.n[0], (c // g.n[0]) % g.n[1]] + ([c // (g.n[0] * g.n[1])] if d == 3 else [])
    e = np.where(p.normal[:, a] >= 0, 1, -1)
    step = e * p.r[:, a]
    X = step * np.asarray(g.h[:d])
    corners = []
    for bits in np.ndindex(*([2] * d)):
        q = [idx[i] + bits[i] * step[i] for i in range(d)]
        lin = q[0] + g.n[0] * (q[1] + (g.n[1] * q[2] if d == 3 else 0))
        corners.append((np.array(bits), int(lin)))
    centre = np.array([g.lo[i] + (idx[i] + 0.5) * g.h[i] for i in range(d)])
    return corners, X, centre


def lagrange(bits, t, X):
    """L_c at normalised coordinates t and its Cartesian gradient."""
    f = np.where(bits == 1, t, 1 - t)
    df = np.where(bits == 1, 1.0, -1.0) / X
    val = np.prod(f)
    grad = np.array([df[i] * np.prod(np.delete(f, i)) for i in range(len(t))])
    return val, grad


@pytest.mark.parametrize("name", ["circle", "sphere", "star"])
def test_surface_scale_recomputed(name):
    inst = dict(_cases())[name]
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    rng = np.random.default_rng(9)
    # positive corner scales, as callers pass them; the basis values and
    # gradients still take both signs (fluid-side anchors extrapolate)
    fs = np.abs(rng.normal(size=(2, p.n_cells)))
    xq = inst.queries.x[:, ::7]
    val, grad, anc, sc = p.surface_query(xq, np.zeros((2, p.n_cells)), field_scale=fs)
    for q in range(xq.shape[1]):
        corners, X, centre = _box(p, int(anc[q]))
        t = (xq[:, q] - centre) / X
        want = np.zeros((2, p.dim + 1))
        for bits, cell in corners:
            v, gr = lagrange(bits, t, X)
            for f in range(2):
                want[f, 0] += abs(v) * fs[f, cell]
                want[f, 1:] += np.abs(gr) * fs[f, cell]
        assert np.allclose(sc[:, :, q], want, rtol=1e-13, atol=1e-300), (q, sc[:, :, q], want)


@pytest.mark.parametrize("name", ["circle", "sphere", "star"])
def test_surface_values_within_their_scale(name):
    inst = dict(_cases())[name]
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    rng = np.random.default_rng(10)
    phi = rng.normal(size=(1, p.n_cells))
    val, grad, anc, sc = p.surface_query(inst.queries.x, phi, field_scale=np.abs(phi))
    assert np.all(np.abs(val[0]) <= sc[0, 0] * (1 + 1e-13))
    assert np.all(np.abs(grad[0]) <= sc[0, 1:] * (1 + 1e-13))


def numpy_adjoint_scale(p, lam_s, bc):
    """Reverse canonical sweep on weight bounds (units by |A^-T| at their
    last member), as the adjoint itself is ordered."""
    pos = _ghost_index(p)
    units = _unit_members(p)
    L = lam_s.copy()
    lb = np.zeros(p.n_ghost)
    for g in range(p.n_ghost - 1, -1, -1):
        if p.unit[g] >= 0:
            mem = units[int(p.unit[g])]
            if g != mem[-1]:
                continue
            inv = np.abs(np.linalg.inv(_unit_matrix(p, mem, bc, pos)))
            mu = inv.T @ L[p.ghost_cell[mem]]
            L[p.ghost_cell[mem]] = 0.0
            for i, m in enumerate(mem):
                w, ws = p.weight_bounds(m, bc)
                lb[m] = ws * mu[i]
                for wk, c in zip(w, p.stencil(m)):
                    if c >= 0 and not (int(c) in pos and pos[int(c)] in mem):
                        L[c] += wk * mu[i]
            continue
        w, ws = p.weight_bounds(g, bc)
        Lg = L[p.ghost_cell[g]]
        lb[g] = ws * Lg
        L[p.ghost_cell[g]] = 0.0
        for wk, c in zip(w, p.stencil(g)):
            if c >= 0:
                L[c] += wk * Lg
    return L, lb


@pytest.mark.parametrize("name", ["circle", "sphere", "star"])
@pytest.mark.parametrize("scheme", [CGC, HGC])
@pytest.mark.parametrize("bc", [DIRICHLET, NEUMANN])
def test_adjoint_scale_recomputed(name, scheme, bc):
    inst = dict(_cases())[name]
    p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    rng = np.random.default_rng(200 + scheme + 3 * bc)
    lam = rng.normal(size=p.n_cells)
    got, got_bc = p.fill_adjoint_scale(np.abs(lam)[None], [bc])
    want, want_bc = numpy_adjoint_scale(p, np.abs(lam), bc)
    assert np.allclose(got[0], want, rtol=1e-13, atol=0)
    assert np.allclose(got_bc[0], want_bc, rtol=1e-13, atol=0)
    # the scales bound the adjoint's outputs
    out, out_bc = p.fill_adjoint(lam[None].copy(), [bc])
    assert np.all(np.abs(out[0]) <= got[0] * (1 + 1e-13))
    assert np.all(np.abs(out_bc[0]) <= got_bc[0] * (1 + 1e-13))
    assert np.all(got[0][p.ghost_cell] == 0)


def test_surface_adjoint_scale_recomputed():
    inst = synth.circle128(seed=5)
    p = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    rng = np.random.default_rng(12)
    xq = inst.queries.x[:, ::5]
    nq = xq.shape[1]
    gval = rng.normal(size=(1, nq))
    ggrad = rng.normal(size=(1, 2, nq))
    got = p.surface_query_adjoint_scale(xq, gval, ggrad, np.zeros((1, p.n_cells)))
    _, _, anc = p.surface_query(xq, np.zeros((1, p.n_cells)))
    want = np.zeros(p.n_cells)
    for q in range(nq):
        corners, X, centre = _box(p, int(anc[q]))
        t = (xq[:, q] - centre) / X
        for bits, cell in corners:
            v, gr = lagrange(bits, t, X)
            want[cell] += abs(v * gval[0, q]) + np.abs(gr * ggrad[0, :, q]).sum()
    assert np.allclose(got[0], want, rtol=1e-13, atol=0)
    out = p.surface_query_adjoint(xq, gval, ggrad, np.zeros((1, p.n_cells)))
    assert np.all(np.abs(out[0]) <= got[0] * (1 + 1e-13))
