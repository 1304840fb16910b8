"""Pins of the oracle's fresh cells (Sec. 7.1: a moving boundary exposes
fresh fluid cells, which a second ghost layer is there to cover).

Expected sets come from the circle's closed-form signed distance over every
cell.  The coverage pin is a consequence of psi being 1-Lipschitz: moving
the body by d changes psi by at most d, so a fresh cell had psi < d before
the move, and with d <= 1.5 delta n it was a second-layer ghost."""
import numpy as np
import pytest

import oracle
import synth
from synth import CGC, HGC, LAYER2

from test_oracle_layer2 import brute_force_circle


def moved(shape, v):
    return synth.Shape(shape.kind, tuple(c + d for c, d in zip(shape.center, v)), shape.r0)


def psi_circle(grid, centre, R):
    X, Y = np.meshgrid(grid.centres(0) - centre[0], grid.centres(1) - centre[1])
    return (R - np.hypot(X, Y)).ravel()


@pytest.mark.parametrize("scheme", [CGC, HGC])
@pytest.mark.parametrize("layer2", [False, True])
def test_fresh_cells_brute_force(scheme, layer2):
    inst = synth.circle128(seed=3)
    g, h = inst.grid, inst.grid.h[0]
    flag = scheme | (LAYER2 if layer2 else 0)
    for v in ((0.7 * h, 0.2 * h, 0.0), (-1.3 * h, 0.9 * h, 0.0), (0.05 * h, -1.9 * h, 0.0)):
        a = oracle.OraclePlan(g, inst.shape, flag)
        b = oracle.OraclePlan(g, moved(inst.shape, v), flag)
        got, unc = a.fresh_cells(b)
        c0, c1 = np.asarray(inst.shape.center[:2]), np.asarray(inst.shape.center[:2]) + v[:2]
        fresh = (psi_circle(g, c0, inst.shape.r0) >= 0) & (psi_circle(g, c1, inst.shape.r0) < 0)
        assert np.array_equal(got, np.flatnonzero(fresh))
        tags, *_ = brute_force_circle(g, c0, inst.shape.r0, scheme) if layer2 else \
            (_plain_tags(g, c0, inst.shape.r0, scheme),)
        assert unc == int(np.sum(fresh & (tags == 1)))


def _plain_tags(grid, centre, R, scheme):
    """Tags of the first layer alone by the definitions (closed-form psi)."""
    psi = psi_circle(grid, centre, R).reshape(grid.n[1], grid.n[0])
    X, Y = np.meshgrid(grid.centres(0) - centre[0], grid.centres(1) - centre[1])
    rho = np.hypot(X, Y)
    n = np.stack([X / rho, Y / rho])
    hx, hy = grid.h[0], grid.h[1]
    dn = 1.0 / np.sqrt((n[0] / hx) ** 2 + (n[1] / hy) ** 2)
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
    return tags.ravel()


@pytest.mark.parametrize("scheme", [CGC, HGC])
def test_second_layer_covers_moves_up_to_its_depth(scheme):
    """delta n = h on a uniform isotropic grid: moves of up to 1.45 h leave
    no fresh cell uncovered with a second layer (2D and 3D)."""
    rng = np.random.default_rng(7 + scheme)
    for inst in (synth.circle128(seed=1), synth.sphere256(seed=2, n=40)):
        g, h, d = inst.grid, inst.grid.h[0], inst.grid.dim
        a = oracle.OraclePlan(g, inst.shape, scheme | LAYER2)
        for mag in (0.4, 0.9, 1.45):
            u = rng.normal(size=d)
            v = tuple(mag * h * u / np.linalg.norm(u)) + (0.0,) * (3 - d)
            b = oracle.OraclePlan(g, moved(inst.shape, v), scheme | LAYER2)
            fresh, unc = a.fresh_cells(b)
            assert len(fresh) > 0 and unc == 0, (mag, len(fresh), unc)


def test_first_layer_alone_leaves_fresh_cells_uncovered():
    inst = synth.circle128(seed=1)
    h = inst.grid.h[0]
    a = oracle.OraclePlan(inst.grid, inst.shape, CGC)
    b = oracle.OraclePlan(inst.grid, moved(inst.shape, (1.45 * h, 0.3 * h, 0.0)), CGC)
    fresh, unc = a.fresh_cells(b)
    assert unc > 0 and unc < len(fresh)


def test_no_move_no_fresh_cells():
    inst = synth.sphere256(seed=0, n=32)
    a = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    b = oracle.OraclePlan(inst.grid, inst.shape, HGC | LAYER2)
    fresh, unc = a.fresh_cells(b)
    assert len(fresh) == 0 and unc == 0
