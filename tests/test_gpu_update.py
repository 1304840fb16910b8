"""GPU parity of gcr_plan_update: the re-plan of a moved body (Sec. 7.1, a
moving boundary), in place, classifying again only the chunks the move can
change.

Every updated plan is compared with the oracle's full plan at the new
position (tags, ghost order, levels, stencil multipliers bit for bit; the
foot-point offsets and normals within 1e-12 of h and 1, as for a plan made
from scratch) and with the library's own full build there (every exported
array bit for bit).  Two plans updated in turn, each from two positions
back, give the fresh cells of every step (gcr_plan_fresh_cells, which skips
the chunks both plans settled alike), checked against the oracle's list.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import CGC, CGC_ES, HGC, LAYER2, DIRICHLET, NEUMANN
from tolerances import check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EXPORTS = ("tags", "cell", "level", "delta", "normal", "psi", "r", "unit")


@pytest.fixture(scope="module")
def gcr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_10165_amd as g
    g.lib()
    return g


def moved(shape, v):
    return synth.Shape(shape.kind, tuple(c + d for c, d in zip(shape.center, v)), shape.r0,
                       coef=shape.coef, ncoef=shape.ncoef)


def host(t):
    return t.detach().cpu().numpy()


def same_as_full(gcr, plan, grid, shape, scheme, what):
    """The updated plan against a plan built from scratch, bit for bit."""
    full = gcr.Plan(grid, shape, scheme)
    a, b = plan.export(EXPORTS), full.export(EXPORTS)
    torch.cuda.synchronize()
    for k in EXPORTS:
        assert np.array_equal(host(a[k]), host(b[k]), equal_nan=True), f"{what}: {k}"
    assert plan.level_offsets() == full.level_offsets(), what
    sa, sb = plan.stats(), full.stats()
    for k in ("n_ghost", "n_levels", "n_interface", "n_ghost_fluid_side", "n_units_coupled",
              "max_unit", "max_level_width", "n_band_segments"):
        assert sa[k] == sb[k], (what, k, sa[k], sb[k])
    return full


def same_as_oracle(op, plan, grid, what):
    ex = plan.export(("tags", "cell", "level", "r", "delta", "normal"))
    torch.cuda.synchronize()
    assert np.array_equal(host(ex["tags"]), op.tags), f"{what}: tags"
    assert np.array_equal(host(ex["cell"]).astype(np.int64), op.ghost_cell), f"{what}: order"
    assert np.array_equal(host(ex["level"]), op.level), f"{what}: levels"
    assert np.array_equal(host(ex["r"]), op.r), f"{what}: multipliers"
    assert plan.level_offsets() == list(op.level_off), what
    h = min(grid.h[:grid.dim])
    check(host(ex["delta"]), op.delta, np.full(op.delta.shape, h), f"{what}: delta")
    check(host(ex["normal"]), op.normal, np.ones(op.normal.shape), f"{what}: normal")


def fresh_vs_oracle(gcr, before, after, ob, oa, what):
    want, unc = ob.fresh_cells(oa)
    lst, counts = before.fresh_cells(after)
    torch.cuda.synchronize()
    c = host(counts)
    assert c[0] == len(want) and c[1] == unc, (what, c, len(want), unc)
    assert np.array_equal(host(lst[:len(want)]).astype(np.int64), want), what
    return len(want), unc


def test_update_moving_sphere256_every_step(gcr):
    """The 256^3 sphere moving 0.4 h per step, HGC with a second layer: two
    plans updated in turn over 8 steps; each step against the oracle and a
    full build, and its fresh cells against the oracle's."""
    inst = synth.sphere256(seed=0)
    g, h = inst.grid, inst.grid.h[0]
    scheme = HGC | LAYER2
    v = 0.4 * h * np.array([0.8, 0.48, 0.36])
    pos = [moved(inst.shape, k * v) for k in range(10)]
    plans = [gcr.Plan(g, pos[0], scheme), gcr.Plan(g, pos[1], scheme)]
    prev_o = oracle.OraclePlan(g, pos[1], scheme)
    for k in range(2, 10):
        p = plans[k % 2]   # at position k - 2
        p.update(pos[k])
        op = oracle.OraclePlan(g, pos[k], scheme)
        same_as_oracle(op, p, g, f"step {k}")
        full = same_as_full(gcr, p, g, pos[k], scheme, f"step {k}")
        nf, unc = fresh_vs_oracle(gcr, plans[(k - 1) % 2], p, prev_o, op, f"fresh {k}")
        assert nf > 1000 and unc == 0   # a second layer covers a move of 0.4 h
        if k == 5:
            # the dropped caches are rebuilt: fill and force agree with the full plan
            rng = np.random.default_rng(k)
            kinds = [DIRICHLET, NEUMANN]
            vals = rng.normal(size=(2, op.n_cells))
            bcs = [torch.as_tensor(rng.normal(size=op.n_ghost)).cuda() for _ in kinds]
            fa = [torch.as_tensor(x).cuda() for x in vals]
            fb = [torch.as_tensor(x).cuda() for x in vals]
            p.fill(fa, kinds, bcs)
            full.fill(fb, kinds, bcs)
            torch.cuda.synchronize()
            for x, y in zip(fa, fb):
                assert torch.equal(x, y)
        prev_o = op


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC, HGC | LAYER2])
def test_update_circle_jumps_and_shape_changes(gcr, scheme):
    """One 2D plan through small moves, a jump of many cells, a change of
    body (circle -> star -> circle of another radius): each result against
    the oracle and a full build."""
    inst = synth.circle128(seed=2)
    g, h = inst.grid, inst.grid.h[0]
    star = synth.stars64(seed=1, ninst=1, nmin=128, nmax=128)[0].shape
    seq = [moved(inst.shape, (0.3 * h, -0.2 * h, 0.0)),
           moved(inst.shape, (0.9 * h, 0.4 * h, 0.0)),
           moved(inst.shape, (17.0 * h, -11.0 * h, 0.0)),
           synth.Shape(star.kind, inst.shape.center, star.r0, coef=star.coef, ncoef=star.ncoef),
           synth.Shape(inst.shape.kind, inst.shape.center, 0.37),
           inst.shape]
    p = gcr.Plan(g, inst.shape, scheme)
    for i, s in enumerate(seq):
        p.update(s)
        op = oracle.OraclePlan(g, s, scheme)
        same_as_oracle(op, p, g, f"move {i}")
        same_as_full(gcr, p, g, s, scheme, f"move {i}")


def test_update_shstar_and_stretched(gcr):
    """A 3D spherical-harmonic star (Lipschitz-settled spans) moved in turn,
    and a circle on a stretched grid (device faces carried over)."""
    inst = synth.shstar384(seed=3, n=64, nt=8, nph=16)
    g, h = inst.grid, inst.grid.h[0]
    p = gcr.Plan(g, inst.shape, HGC)
    for k, v in enumerate(((0.5 * h, 0.1 * h, -0.3 * h), (1.4 * h, -0.7 * h, 0.2 * h))):
        s = moved(inst.shape, v)
        p.update(s)
        same_as_oracle(oracle.OraclePlan(g, s, HGC), p, g, f"shstar {k}")
        same_as_full(gcr, p, g, s, HGC, f"shstar {k}")
    inst = synth.circle_stretched(seed=1)
    p = gcr.Plan(inst.grid, inst.shape, HGC | LAYER2)
    for k, v in enumerate(((0.01, -0.02, 0.0), (-0.05, 0.03, 0.0))):
        s = moved(inst.shape, v)
        p.update(s)
        same_as_oracle(oracle.OraclePlan(inst.grid, s, HGC | LAYER2), p, inst.grid, f"str {k}")
        same_as_full(gcr, p, inst.grid, s, HGC | LAYER2, f"str {k}")


def test_update_errors_leave_the_plan_as_it_was(gcr):
    """A bad shape is refused before anything changes; a position whose
    stencils leave the grid (GCR_E_STENCIL, found after the tags were
    updated) leaves the plan rebuilt at its old position; a plan of a batch
    is refused (GCR_E_UNSUPPORTED)."""
    inst = synth.circle128(seed=0)
    g = inst.grid
    p = gcr.Plan(g, inst.shape, HGC)
    with pytest.raises(gcr.GcrError) as e:
        p.update(synth.Shape(inst.shape.kind, inst.shape.center, -1.0))
    assert e.value.code == 1
    same_as_full(gcr, p, g, inst.shape, HGC, "after a refused shape")
    edge = synth.Shape(inst.shape.kind, (1.55, 0.0, 0.0), inst.shape.r0)
    with pytest.raises(oracle.OracleError):
        oracle.OraclePlan(g, edge, HGC)
    with pytest.raises(gcr.GcrError) as e:
        p.update(edge)
    assert e.value.code == 5
    same_as_full(gcr, p, g, inst.shape, HGC, "after a failed update")
    s = moved(inst.shape, (0.02, 0.01, 0.0))
    p.update(s)   # and it still updates
    same_as_full(gcr, p, g, s, HGC, "update after a failed one")
    b = gcr.Batch([g, g], [inst.shape, s], [HGC, HGC])
    with pytest.raises(gcr.GcrError) as e:
        b.plans[0].update(s)
    assert e.value.code == 8
