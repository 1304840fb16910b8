"""Pins of the oracle's tolerance machinery.

Every GPU parity test accepts |y - y*| <= 1e-12 max(|y*|, s), with s the
oracle's condition-aware scale of y*.  A mistake that inflates s would
loosen every such test without turning any red, so the scales are pinned
here against independent recomputations in numpy:

  * fill scale (propagated through the levels of Sec. 3.2 with the weights
    of Eqs. phi_G_Dir_2d ... phi_G_Neu_3d): s_G = sum_k |w_k| s_{P_k} +
    |w_s b_G|, s = |phi| on cells that are not ghosts, a coupled unit's
    members |A^-1| times their external sums;
  * surface scale (Sec. 6): sum over the anchor box's corners of |L_c(x)|
    (value) or |d L_c / dx_i| (gradient) times the corner scales, with the
    tensor-product Lagrange basis written out here from the box geometry;
  * adjoint scales: the reverse sweep on magnitudes, units by |A^-T|.

Besides equality with the recomputation, two properties that hold whatever
the arithmetic: a scale bounds the magnitude of its value (triangle
inequality), and, for the Dirichlet relation with every normalised distance
|alpha_i| <= 1/2 (HGC and CGC_ES, Sec. 8), each |omega_i| <= 1, so
sum_k |w_k| <= 2^d - 1 and |w_s| <= 2^d bound s_G by the scales it reads.
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
                w, ws = p.weights(m, bc)
                ext[i] = abs(ws * b[m])
                for wk, c in zip(w, p.stencil(m)):
                    if c < 0:
                        continue
                    c = int(c)
                    if c in pos and pos[c] in mem:
                        continue
                    ext[i] += abs(wk) * (s[pos[c]] if c in pos else abs(phi[c]))
            s[mem] = np.abs(np.linalg.inv(_unit_matrix(p, mem, bc, pos))) @ ext
            continue
        w, ws = p.weights(g, bc)
        acc = abs(ws * b[g])
        for wk, c in zip(w, p.stencil(g)):
            if c >= 0:
                c = int(c)
                acc += abs(wk) * (s[pos[c]] if c in pos else abs(phi[c]))
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
def test_fill_scale_alpha_bound(name, scheme):
    """Dirichlet with |alpha_i| <= 1/2: |omega_i| = |alpha_i| / |1 - alpha_i|
    <= 1, so s_G <= (2^d - 1) max_k s_{P_k} + 2^d |b_G| for every ghost that
    is its own unit, however the weights are computed."""
    inst = dict(_cases())[name]
    p = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    assert np.all(p.margins["max_alpha"] <= 0.5)
    rng = np.random.default_rng(5)
    phi, b = _inputs(p, inst, DIRICHLET, rng)
    s = p.fill_scale(np.nan_to_num(phi)[None], [DIRICHLET], b[None])[0]
    pos = _ghost_index(p)
    nc = 1 << p.dim
    for g in range(p.n_ghost):
        if p.unit[g] >= 0:
            continue
        reads = [s[pos[int(c)]] if int(c) in pos else abs(phi[c]) for c in p.stencil(g) if c >= 0]
        bound = (nc - 1) * max(reads, default=0.0) + nc * abs(b[g])
        assert s[g] <= bound * (1 + 1e-14), (g, s[g], bound)


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
    """Reverse canonical sweep on magnitudes (units by |A^-T| at their last
    member), as the adjoint itself is ordered."""
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
                w, ws = p.weights(m, bc)
                lb[m] = abs(ws) * mu[i]
                for wk, c in zip(w, p.stencil(m)):
                    if c >= 0 and not (int(c) in pos and pos[int(c)] in mem):
                        L[c] += abs(wk) * mu[i]
            continue
        w, ws = p.weights(g, bc)
        Lg = L[p.ghost_cell[g]]
        lb[g] = abs(ws) * Lg
        L[p.ghost_cell[g]] = 0.0
        for wk, c in zip(w, p.stencil(g)):
            if c >= 0:
                L[c] += abs(wk) * Lg
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
