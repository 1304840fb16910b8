"""Brute-force pins of the oracle's 3D ghost tags (Sec. 3.1, Sec. 7).

The expected tags, multipliers and foot points of a sphere are computed
here over every cell of the grid from the definitions, with the sphere's
closed-form signed distance psi = R - |x - c| and normal n = (x - c)/|x - c|:

  * classification by centre, solid <=> psi >= 0;
  * the six face neighbours (reading: "adjacent" means sharing a face);
  * CGC / CGC_ES: solid cells with a fluid face neighbour;
  * HGC (Eq. HGC_criterion with Delta n of Eq. delta_n in 3D): solid cells
    with a fluid face neighbour and psi <= Delta n / 2 (+2), fluid cells
    with a solid face neighbour and -psi < Delta n / 2 (-2);
  * second layer (Sec. 7.1): every other solid cell with psi <= 1.5 Delta n;
  * multipliers r_i = max(1, ceil(2 |delta_i| / h_i)) (Eq.
    stencil_anisotropic) for CGC_ES ghosts and second-layer ghosts, 1
    otherwise;
  * foot point offset delta = psi n.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import CGC, CGC_ES, HGC, LAYER2


def brute_force_sphere(grid, centre, R, scheme, layer2):
    n = grid.n
    h = grid.h
    axes = [grid.lo[a] + (np.arange(n[a]) + 0.5) * h[a] - centre[a] for a in range(3)]
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    rho = np.sqrt(x * x + y * y + z * z)
    psi = R - rho
    nv = np.stack([x / rho, y / rho, z / rho])
    dn = 1.0 / np.sqrt(sum((nv[a] / h[a]) ** 2 for a in range(3)))     # Eq. delta_n
    solid = psi >= 0
    other = np.zeros_like(solid)
    for ax in range(3):          # array axes are (z, y, x)
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[ax], b[ax] = slice(1, None), slice(None, -1)
        diff = solid[tuple(a)] != solid[tuple(b)]
        other[tuple(a)] |= diff
        other[tuple(b)] |= diff
    tags = solid.astype(np.int8)
    if scheme == HGC:
        tags[solid & other & (psi <= dn / 2)] = 2
        tags[~solid & other & (-psi < dn / 2)] = -2
    else:
        tags[solid & other] = 2
    added = np.zeros_like(solid)
    if layer2:
        added = solid & (tags != 2) & (psi <= 1.5 * dn)
        tags[added] = 2
    ext = added | (tags == 2) if scheme == CGC_ES else added
    r = np.ones((3,) + psi.shape, np.int64)
    for a in range(3):
        q = np.maximum(1, np.ceil(2 * np.abs(psi * nv[a]) / h[a])).astype(np.int64)
        r[a][ext] = q[ext]
    delta = psi * nv
    return (tags.ravel(), r.reshape(3, -1), delta.reshape(3, -1), nv.reshape(3, -1),
            added.ravel())


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
@pytest.mark.parametrize("layer2", [False, True])
@pytest.mark.parametrize("seed", [0, 3])
def test_sphere_tags_brute_force(scheme, layer2, seed):
    inst = synth.sphere256(seed=seed, n=40)
    sch = scheme | (LAYER2 if layer2 else 0)
    p = oracle.OraclePlan(inst.grid, inst.shape, sch)
    assert p.min_margin > 1e-9
    tags, r, delta, nv, added = brute_force_sphere(inst.grid, inst.shape.center, inst.shape.r0,
                                                   scheme, layer2)
    assert np.array_equal(p.tags, tags)
    c = p.ghost_cell
    assert np.array_equal(np.sort(c), np.flatnonzero(np.abs(tags) == 2))
    assert np.array_equal(p.r, r[:, c])
    assert np.allclose(p.delta, delta[:, c], rtol=0, atol=1e-15)
    assert np.allclose(p.normal, nv[:, c], rtol=0, atol=1e-15)
    if scheme == HGC:
        assert (tags == -2).sum() > 0 and (tags == 2).sum() > 0
    if layer2:
        assert added.sum() > 0
        # the scheme's own ghosts are kept
        p1 = oracle.OraclePlan(inst.grid, inst.shape, scheme)
        assert set(p1.ghost_cell.tolist()) <= set(c.tolist())
        assert p.n_ghost == p1.n_ghost + added.sum()


def test_sphere_tags_on_an_anisotropic_grid():
    """Unequal spacings per axis make Eq. delta_n and the multipliers of Eq.
    stencil_anisotropic depend on the direction."""
    inst = synth.sphere256(seed=1, n=40)
    g = inst.grid
    grid = synth.Grid(3, (40, 36, 44), (-1.0, -0.9, -1.1), (2.0 / 40, 1.8 / 36, 2.2 / 44))
    for scheme in (CGC_ES, HGC):
        for layer2 in (False, True):
            p = oracle.OraclePlan(grid, inst.shape, scheme | (LAYER2 if layer2 else 0))
            assert p.min_margin > 1e-9
            tags, r, delta, nv, _ = brute_force_sphere(grid, inst.shape.center, inst.shape.r0,
                                                       scheme, layer2)
            assert np.array_equal(p.tags, tags)
            assert np.array_equal(p.r, r[:, p.ghost_cell])
