"""Pins of the oracle's second ghost layer (Sec. 7.1): solid cells with
psi <= 1.5 delta n join the ghost set, reconstructed on the extended stencil
of Eq. stencil_anisotropic.

Expected sets come from brute force over every cell with the circle's
closed-form signed distance; the other pins are properties the paper states
(alpha <= 1/2 on the extended stencil, exactness on bilinear and trilinear
fields, levels as longest dependency paths)."""
import math

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
    return np.stack([g.lo[i] + (idx[i] + 0.5) * g.h[i] for i in range(p.dim)])


def brute_force_circle(grid, centre, R, scheme):
    """Tags and per-cell multipliers of a circle by the definitions, with
    psi = R - |x - c| and n = (x - c)/|x - c| in closed form."""
    nx, ny = grid.n[0], grid.n[1]
    hx, hy = grid.h[0], grid.h[1]
    X = grid.lo[0] + (np.arange(nx) + 0.5) * hx
    Y = grid.lo[1] + (np.arange(ny) + 0.5) * hy
    x, y = np.meshgrid(X - centre[0], Y - centre[1])
    rho = np.hypot(x, y)
    psi = R - rho
    n = np.stack([x / rho, y / rho])
    dn = 1.0 / np.sqrt((n[0] / hx) ** 2 + (n[1] / hy) ** 2)       # Eq. delta_n
    solid = psi >= 0
    other = np.zeros_like(solid)                                   # a face neighbour of the other class
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
    added = solid & (tags != 2) & (psi <= 1.5 * dn)
    tags[added] = 2
    r = np.ones((2,) + psi.shape, np.int64)
    ext = added | (tags == 2) if scheme == CGC_ES else added
    for a, h in ((0, hx), (1, hy)):
        q = np.maximum(1, np.ceil(2 * np.abs(psi * n[a]) / h)).astype(np.int64)
        r[a][ext] = q[ext]
    return tags.ravel(), r.reshape(2, -1), added.ravel(), psi.ravel(), dn.ravel()


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
@pytest.mark.parametrize("seed", [0, 1])
def test_second_layer_set_brute_force(scheme, seed):
    inst = synth.circle128(seed=seed)
    p = oracle.OraclePlan(inst.grid, inst.shape, scheme | LAYER2)
    assert p.min_margin > 1e-9
    tags, r, added, psi, dn = brute_force_circle(inst.grid, inst.shape.center, inst.shape.r0,
                                                 scheme)
    assert np.array_equal(p.tags, tags)
    assert added.sum() > 0
    assert np.array_equal(p.r, r[:, p.ghost_cell])
    # the first layer is kept: every ghost of the plain scheme is a ghost here
    p1 = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    assert set(p1.ghost_cell.tolist()) <= set(p.ghost_cell.tolist())
    assert p.n_ghost == p1.n_ghost + added.sum()


def test_second_layer_alpha_bound():
    """On the extended stencil |x_1,i - x_s,i| / (r_i dx_i) <= 1/2 for every
    direction (the bound below Eq. stencil_anisotropic)."""
    for inst in (synth.circle128(seed=2), synth.sphere256(seed=1, n=40),
                 synth.stars64(seed=3, ninst=1, nmin=200, nmax=300)[0]):
        for scheme in (CGC, HGC):
            p = oracle.OraclePlan(inst.grid, inst.shape, scheme | LAYER2)
            p1 = oracle.OraclePlan(inst.grid, inst.shape, scheme)
            first = set(p1.ghost_cell.tolist())
            ext = np.array([int(c) not in first for c in p.ghost_cell])
            assert ext.any()
            h = np.asarray(inst.grid.h[:p.dim])[:, None]
            alpha = np.abs(p.delta) / (p.r * h)
            assert np.all(alpha[:, ext] <= 0.5 + 1e-15)
            # second-layer ghosts lie deeper: psi up to 1.5 cells
            assert p.psi[ext].max() > 0.5 * min(inst.grid.h[:p.dim])


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_second_layer_exact_bilinear_and_trilinear(scheme):
    rng = np.random.default_rng(31 + scheme)
    cases = [(2, synth.circle128(seed=1)), (2, synth.stars64(seed=0, ninst=1, nmin=140, nmax=200)[0]),
             (3, synth.sphere256(seed=2, n=40))]
    for dim, inst in cases:
        p = oracle.OraclePlan(inst.grid, inst.shape, scheme | LAYER2)
        C = rng.normal(size=4 if dim == 2 else 8)
        for bc in (DIRICHLET, NEUMANN):
            fld = synth.polynomial_field(dim, C, bc)
            exact = synth.sample(fld, inst.grid)
            phi = exact.copy()
            phi[p.tags != 0] = np.nan           # ghosts and solid cells poisoned
            S = ghost_centres(p) + p.delta
            b = synth.bc_values(fld, S, p.normal, bc)[None]
            out = p.fill(phi[None], [bc], b)[0]
            sc = p.fill_scale(exact[None], [bc], b)[0]
            err = np.abs(out[p.ghost_cell] - exact[p.ghost_cell])
            assert np.all(err <= 1e-12 * np.maximum(sc, 1.0)), err.max()


@pytest.mark.parametrize("scheme", [CGC, HGC])
def test_second_layer_levels(scheme):
    """Levels stay longest dependency paths and synchronous sweeps need
    exactly n_levels sweeps (Sec. 3.2)."""
    inst = synth.circle128(seed=4)
    p = oracle.OraclePlan(inst.grid, inst.shape, scheme | LAYER2)
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
