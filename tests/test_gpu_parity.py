"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Integer and index outputs (tags, ghost order, levels, multipliers, coupled
units) must match bit for bit.  FP64 outputs must satisfy
|y - y*| <= 1e-12 * max(|y*|, s), where s is the oracle's condition-aware
scale (sum of |weights| times the scales of the inputs), so values that
cross zero and ill-conditioned CGC relations are judged fairly.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import CGC, CGC_ES, HGC, DIRICHLET, NEUMANN
from tolerances import force_scale

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def gcr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_10165_amd as g
    g.lib()   # fails loudly if the HIP library is missing
    return g


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def ghost_centres(p):
    g = p.grid
    c = p.ghost_cell
    idx = [c % g.n[0], (c // g.n[0]) % g.n[1]]
    if p.dim == 3:
        idx.append(c // (g.n[0] * g.n[1]))
    return np.stack([g.centres(i)[idx[i]] for i in range(p.dim)])


def check_close(got, want, scale, what):
    got, want, scale = np.asarray(got), np.asarray(want), np.asarray(scale)
    bound = TOL * np.maximum(np.abs(want), scale)
    err = np.abs(got - want)
    bad = ~(err <= bound)
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} outside 1e-12 rel; "
                           f"worst err {err[bad].max() if bad.any() else 0}")


def plan_pair(gcr, inst, scheme):
    op = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    gp = gcr.Plan(inst.grid, inst.shape, scheme)
    return op, gp


def check_plan(op, gp, strict_geometry=False):
    ex = gp.export()
    torch.cuda.synchronize()
    assert gp.n_ghost == op.n_ghost
    assert gp.n_levels == op.n_levels
    assert np.array_equal(host(ex["tags"]), op.tags), "tags"
    assert np.array_equal(host(ex["cell"]).astype(np.int64), op.ghost_cell), "ghost order"
    assert gp.level_offsets() == list(op.level_off), "level offsets"
    assert np.array_equal(host(ex["level"]), op.level), "levels"
    assert np.array_equal(host(ex["r"]), op.r), "multipliers"
    # coupled units: same partition (leader = first member in canonical order)
    unit = host(ex["unit"])
    want = np.full(op.n_ghost, -1)
    for b in np.unique(op.unit[op.unit >= 0]):
        mem = np.where(op.unit == b)[0]
        want[mem] = mem.min()
    assert np.array_equal(unit, want), "coupled units"
    h = min(op.grid.h[: op.dim])
    for key, ref, s in (("psi", op.psi, h), ("delta", op.delta, h), ("normal", op.normal, 1.0)):
        got = host(ex[key])
        if strict_geometry:
            assert np.array_equal(got, ref), key
        else:
            # geometry scale: a cell width for lengths, 1 for unit normals
            check_close(got, ref, np.full(ref.shape, s), key)
    return ex


def bc_arrays(op, flds, kinds):
    S = ghost_centres(op) + op.delta
    return np.stack([synth.bc_values(f, S, op.normal, k) for f, k in zip(flds, kinds)])


def run_fill(gcr, op, gp, inst, flds, kinds, schedule=None):
    vals = np.stack([synth.sample(f, inst.grid) for f in flds])
    vals[:, op.tags != 0] = np.nan                     # ghosts and solid cells poisoned
    b = bc_arrays(op, flds, kinds)
    bt = np.broadcast_to(np.asarray(kinds, np.int8)[:, None], b.shape) if np.ndim(kinds[0]) == 0 \
        else np.stack(kinds).astype(np.int8)
    want = op.fill(vals.copy(), bt, b)
    scale = op.fill_scale(np.nan_to_num(vals), bt, b)
    fields = [dev(v) for v in vals]
    if schedule is not None:
        gp.set_schedule(schedule)
    if np.ndim(kinds[0]) == 0:
        gp.fill(fields, list(kinds), [dev(x) for x in b])
    else:
        gp.fill(fields, [2] * len(flds), [dev(x) for x in b],
                bc_type=[dev(k, torch.uint8) for k in bt])
    torch.cuda.synchronize()
    got = np.stack([host(f) for f in fields])
    for f in range(len(flds)):
        check_close(got[f][op.ghost_cell], want[f][op.ghost_cell], scale[f], f"fill field {f}")
        nong = np.ones(op.n_cells, bool)
        nong[op.ghost_cell] = False
        assert np.array_equal(np.isnan(got[f][nong]), np.isnan(vals[f][nong]))
        assert np.array_equal(got[f][nong & ~np.isnan(vals[f])], vals[f][nong & ~np.isnan(vals[f])])
    return got, want, scale


# ---------------------------------------------------------------------------
# plans
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_plan_circle128(gcr, seed, scheme):
    inst = synth.circle128(seed=seed)
    op, gp = plan_pair(gcr, inst, scheme)
    check_plan(op, gp, strict_geometry=True)   # closed form: same operations


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_plan_sphere_small_and_ragged(gcr, scheme):
    # 3D, grid sizes that are not multiples of 16 (ragged classification tails)
    h = 2.0 / 61
    grid = synth.Grid(3, (61, 53, 47), (-1.0, -0.9, -0.8), (h, h, h))
    shape = synth.Shape(synth.SPHERE, (0.013, -0.02, 0.007), 0.41)
    inst = synth.Instance("sphere_ragged", grid, shape, scheme, synth.abc_fields())
    op, gp = plan_pair(gcr, inst, scheme)
    check_plan(op, gp, strict_geometry=True)


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_plan_sphere256_full_size(gcr, scheme):
    inst = synth.sphere256(seed=0, scheme=scheme)
    op, gp = plan_pair(gcr, inst, scheme)
    assert op.min_margin > 1e-9
    check_plan(op, gp, strict_geometry=True)


@pytest.mark.parametrize("seed", [0, 1])
def test_plan_stars_including_cycle(gcr, seed):
    insts = synth.stars64(seed=seed, ninst=3, nmin=96, nmax=400)
    for inst in insts:
        for scheme in (CGC, HGC):
            op, gp = plan_pair(gcr, inst, scheme)
            assert op.min_margin > 1e-9
            check_plan(op, gp)


def test_plan_star_with_coupled_unit(gcr):
    inst = synth.stars64(seed=0, ninst=1, nmin=96, nmax=160)[0]
    op, gp = plan_pair(gcr, inst, CGC)
    assert op.n_units_coupled >= 1
    check_plan(op, gp)
    run_fill(gcr, op, gp, inst, inst.fields[:2], [DIRICHLET, NEUMANN])


def test_plan_shstar(gcr):
    inst = synth.shstar384(seed=0, n=96, nt=4, nph=8)
    for scheme in (CGC, HGC):
        op, gp = plan_pair(gcr, inst, scheme)
        assert op.min_margin > 1e-9
        check_plan(op, gp)


def test_plan_airfoil(gcr):
    inst = synth.airfoil4096(seed=0, n=1024, m=64)
    op, gp = plan_pair(gcr, inst, HGC)
    assert op.min_margin > 1e-9
    check_plan(op, gp)


@pytest.mark.parametrize("n", [5120, 8192])
def test_plan_airfoil_fine_grids(gcr, n):
    """The airfoil on grids where a first-order (Gauss-Newton) projection
    along the contour had not converged in its iteration limit for some
    cells: the plan against the oracle's (tags, ghost order and levels bit
    for bit, foot points and normals within tolerance)."""
    inst = synth.airfoil4096(seed=0, n=n, m=64)
    op, gp = plan_pair(gcr, inst, HGC)
    assert op.min_margin > 1e-9
    check_plan(op, gp)


@pytest.fixture(params=[0, 1])
def wide(gcr, request):
    # every plan built alone is layered grid-wide; with a release buffer of
    # one slot per workgroup nearly every placed ghost takes the overflow
    gcr.set_wide_layering(1)
    gcr.set_wide_buffer(request.param)
    yield
    gcr.set_wide_layering(0)
    gcr.set_wide_buffer(0)


def _layering_case(case):
    if case == "circle128":
        return synth.circle128(seed=3), HGC
    if case == "sphere_ragged":
        h = 2.0 / 61
        grid = synth.Grid(3, (61, 53, 47), (-1.0, -0.9, -0.8), (h, h, h))
        shape = synth.Shape(synth.SPHERE, (0.013, -0.02, 0.007), 0.41)
        return synth.Instance("sphere_ragged", grid, shape, CGC, synth.abc_fields()), CGC
    if case == "sphere256":
        return synth.sphere256(seed=0, scheme=CGC_ES), CGC_ES
    if case == "star_unit":
        # a coupled unit: the grid-wide rounds stall and the one-workgroup
        # layering takes over
        return synth.stars64(seed=0, ninst=1, nmin=96, nmax=160)[0], CGC
    if case == "shstar":
        return synth.shstar384(seed=0, n=96, nt=4, nph=8), HGC
    return synth.airfoil4096(seed=0, n=1024, m=64), HGC


@pytest.mark.parametrize("case", ["circle128", "sphere_ragged", "sphere256", "star_unit",
                                  "shstar", "airfoil"])
def test_wide_layering_matches_oracle(gcr, wide, case):
    inst, scheme = _layering_case(case)
    op, gp = plan_pair(gcr, inst, scheme)
    if case == "star_unit":
        assert op.n_units_coupled >= 1
    check_plan(op, gp, strict_geometry=case in ("circle128", "sphere_ragged", "sphere256"))
    run_fill(gcr, op, gp, inst, (list(inst.fields) * 2)[:2], [DIRICHLET, NEUMANN])


def test_plan_shstar384_full_size(gcr):
    # above the default size for grid-wide layering
    inst = synth.shstar384(seed=0)
    op, gp = plan_pair(gcr, inst, HGC)
    assert op.n_interface >= 65536
    assert op.min_margin > 1e-9
    check_plan(op, gp)


def test_plan_beyond_lds_layering(gcr):
    # 74,006 ghosts: more than the one-workgroup LDS layering holds, so the
    # default takes the grid-wide layering (17 levels)
    inst = synth.sphere256(seed=0, n=512)
    op, gp = plan_pair(gcr, inst, HGC)
    assert op.n_ghost > 50000 and op.n_interface >= 65536
    check_plan(op, gp, strict_geometry=True)


# ---------------------------------------------------------------------------
# fill
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_fill_circle128(gcr, scheme):
    inst = synth.circle128(seed=1, scheme=scheme)
    op, gp = plan_pair(gcr, inst, scheme)
    f = inst.fields[0]
    run_fill(gcr, op, gp, inst, [f, f], [DIRICHLET, NEUMANN])


@pytest.mark.parametrize("schedule", [1, 2, 3, 0])
def test_fill_schedules_agree(gcr, schedule):
    inst = synth.sphere256(seed=1, n=80)
    op, gp = plan_pair(gcr, inst, HGC)
    got, _, _ = run_fill(gcr, op, gp, inst, inst.fields, [0, 0, 0, 1], schedule=schedule)
    gp2 = gcr.Plan(inst.grid, inst.shape, HGC)
    gp2.set_schedule(1)
    got2, _, _ = run_fill(gcr, op, gp2, inst, inst.fields, [0, 0, 0, 1])
    assert np.array_equal(np.nan_to_num(got, nan=7.0), np.nan_to_num(got2, nan=7.0))


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_fill_sphere256(gcr, scheme):
    inst = synth.sphere256(seed=0, scheme=scheme)
    op, gp = plan_pair(gcr, inst, scheme)
    run_fill(gcr, op, gp, inst, inst.fields, [DIRICHLET, DIRICHLET, DIRICHLET, NEUMANN])


def test_fill_mixed_stars(gcr):
    for inst in synth.stars64(seed=3, ninst=3, nmin=128, nmax=700):
        op, gp = plan_pair(gcr, inst, HGC)
        S = ghost_centres(op) + op.delta
        kinds = [synth.mixed_kinds(S, inst.shape.center, b) for b in inst.mixed_beta]
        run_fill(gcr, op, gp, inst, inst.fields, kinds)


def test_fill_shstar_and_airfoil(gcr):
    inst = synth.shstar384(seed=1, n=96, nt=4, nph=8)
    op, gp = plan_pair(gcr, inst, HGC)
    run_fill(gcr, op, gp, inst, inst.fields, [0, 0, 0, 1])
    inst = synth.airfoil4096(seed=1, n=1024, m=64)
    op, gp = plan_pair(gcr, inst, HGC)
    run_fill(gcr, op, gp, inst, inst.fields, [0, 0, 1])


def test_airfoil4096_full_size(gcr):
    """The airfoil workload at its full size (4096^2 cells, about 2,100
    ghosts in chains over 100 levels deep): plans (CGC, HGC) bit-exact, the
    HGC fill of u, v (Dirichlet) and p (Neumann), surface values at the
    2 x 1024 quadrature points and the force, all against the oracle."""
    inst = synth.airfoil4096(seed=0)
    assert inst.grid.n[:2] == (4096, 4096)
    op, gp = plan_pair(gcr, inst, CGC)
    check_plan(op, gp)
    op, gp = plan_pair(gcr, inst, HGC)
    assert op.min_margin > 1e-9 and op.n_levels > 80
    check_plan(op, gp)
    got, want, scale = run_fill(gcr, op, gp, inst, inst.fields, [DIRICHLET, DIRICHLET, NEUMANN])
    q = inst.queries
    cs = op.cell_scale(np.nan_to_num(want), scale)
    v, g, anc = gp.surface(dev(q.x), [dev(x) for x in got])
    ov, og, oanc, osc = op.surface_query(q.x, want, field_scale=cs)
    assert np.array_equal(host(anc), oanc)
    check_close(host(v), ov, osc[:, 0], "query value")
    check_close(host(g), og, osc[:, 1:], "query gradient")
    mu = 0.3
    F = gp.forces(dev(q.x), dev(q.n), dev(q.w), dev(got[2]), [dev(got[0]), dev(got[1])], mu)
    Fo = op.forces(q.x, q.n, q.w, want[2], want[:2], mu)
    check_close(host(F), Fo, force_scale(op, q, want, cs, 2, [0, 1], mu), "forces")


def test_fill_deterministic(gcr):
    inst = synth.sphere256(seed=2, n=96)
    op, gp = plan_pair(gcr, inst, HGC)
    a, _, _ = run_fill(gcr, op, gp, inst, inst.fields, [0, 0, 0, 1])
    b, _, _ = run_fill(gcr, op, gp, inst, inst.fields, [0, 0, 0, 1])
    assert np.array_equal(np.nan_to_num(a, nan=3.0), np.nan_to_num(b, nan=3.0))


# ---------------------------------------------------------------------------
# surface values, gradients, forces
# ---------------------------------------------------------------------------

def test_surface_ghost_and_query_circle(gcr):
    inst = synth.circle128(seed=2)
    op, gp = plan_pair(gcr, inst, HGC)
    got, want, scale = run_fill(gcr, op, gp, inst, inst.fields, [DIRICHLET])
    fields = [dev(got[0])]
    val, grad = gp.surface_ghost(fields)
    wv, wg = op.surface_ghost(want)
    cs = op.cell_scale(np.nan_to_num(want), scale)
    # foot-point outputs: scale = sum |coefficients| * corner scales, bounded by
    # (sum over the box of scales) * max |coefficient|
    _, _, _, qs = op.surface_query(ghost_centres(op) + op.delta, want, field_scale=cs)
    check_close(host(val), wv, qs[:, 0], "surface value")
    check_close(host(grad), wg, qs[:, 1:], "surface gradient")
    xq = dev(inst.queries.x)
    v2, g2, anc = gp.surface(xq, fields)
    ov, og, oanc, osc = op.surface_query(inst.queries.x, want, field_scale=cs)
    assert np.array_equal(host(anc), oanc), "anchors"
    check_close(host(v2), ov, osc[:, 0], "query value")
    check_close(host(g2), og, osc[:, 1:], "query gradient")


def test_surface_query_sphere256(gcr):
    inst = synth.sphere256(seed=1)
    op, gp = plan_pair(gcr, inst, HGC)
    got, want, scale = run_fill(gcr, op, gp, inst, inst.fields, [0, 0, 0, 1])
    cs = op.cell_scale(np.nan_to_num(want), scale)
    v, g, anc = gp.surface(dev(inst.queries.x), [dev(x) for x in got])
    ov, og, oanc, osc = op.surface_query(inst.queries.x, want, field_scale=cs)
    assert np.array_equal(host(anc), oanc)
    check_close(host(v), ov, osc[:, 0], "query value")
    check_close(host(g), og, osc[:, 1:], "query gradient")


@pytest.mark.parametrize("which", ["circle128", "sphere256"])
def test_forces(gcr, which):
    inst = synth.circle128(seed=0) if which == "circle128" else synth.sphere256(seed=0)
    d = inst.grid.dim
    op, gp = plan_pair(gcr, inst, HGC)
    if d == 2:
        flds = [inst.fields[0], synth.polynomial_field(2, [0.1, 0.2, -0.3, 0.4], DIRICHLET),
                synth.polynomial_field(2, [1.0, -0.5, 0.25, 0.3], NEUMANN)]
        kinds = [DIRICHLET, DIRICHLET, NEUMANN]
    else:
        flds, kinds = inst.fields, [0, 0, 0, 1]
    got, want, scale = run_fill(gcr, op, gp, inst, flds, kinds)
    q = inst.queries
    u_idx = list(range(d))
    p_idx = d
    mu = 0.7
    F = gp.forces(dev(q.x), dev(q.n), dev(q.w), dev(got[p_idx]), [dev(got[i]) for i in u_idx], mu)
    Fo = op.forces(q.x, q.n, q.w, want[p_idx], np.stack([want[i] for i in u_idx]), mu)
    cs = op.cell_scale(np.nan_to_num(want), scale)
    check_close(host(F), Fo, force_scale(op, q, want, cs, p_idx, u_idx, mu), "forces")


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_no_ghosts(gcr):
    # body far outside the grid: every cell fluid, zero ghosts, fill is a no-op
    grid = synth.Grid(2, (40, 33, 1), (0.0, 0.0, 0.0), (0.1, 0.1, 1.0))
    shape = synth.Shape(synth.SPHERE, (50.0, 50.0, 0.0), 1.0)
    gp = gcr.Plan(grid, shape, HGC)
    assert gp.n_ghost == 0 and gp.n_levels == 0
    ex = gp.export()
    assert int(ex["tags"].abs().sum()) == 0
    u = torch.ones(grid.n_cells, dtype=torch.float64, device="cuda")
    gp.fill([u], [0], [torch.zeros(1, dtype=torch.float64, device="cuda")])
    torch.cuda.synchronize()
    assert float(u.sum()) == grid.n_cells


def test_body_touching_the_edge_is_reported(gcr):
    # the circle's left edge lies inside the first column, so the ghost there
    # needs a stencil point in column -1
    grid = synth.Grid(2, (32, 32, 1), (0.0, 0.0, 0.0), (1.0 / 32, 1.0 / 32, 1.0))
    shape = synth.Shape(synth.SPHERE, (0.305, 0.5, 0.0), 0.3)
    with pytest.raises(gcr.GcrError) as e:
        gcr.Plan(grid, shape, CGC)
    assert e.value.code == 5
    with pytest.raises(oracle.OracleError) as e2:
        oracle.OraclePlan(grid, shape, CGC)
    assert e2.value.code == 5


def test_zero_normal_components(gcr):
    h = 1.0 / 32
    grid = synth.Grid(2, (128, 128, 1), (-2.0, -2.0, 0.0), (h, h, 1.0))
    c = (-2.0 + 64.5 * h, -2.0 + 64.5 * h, 0.0)
    inst = synth.Instance("axis", grid, synth.Shape(synth.SPHERE, c, 0.5), HGC,
                          synth.circle128().fields)
    op, gp = plan_pair(gcr, inst, HGC)
    assert (op.normal == 0).any()
    check_plan(op, gp, strict_geometry=True)
    run_fill(gcr, op, gp, inst, inst.fields * 2, [DIRICHLET, NEUMANN])


@pytest.mark.parametrize("which", ["circle128", "sphere64"])
def test_foot_points(gcr, which):
    """gcr_plan_foot_points: S = x_c + delta and the normals, against the
    oracle's foot points (1e-12 of a cell width) and the exported arrays."""
    inst = synth.circle128(seed=3) if which == "circle128" else synth.sphere256(seed=1, n=64)
    op, gp = plan_pair(gcr, inst, HGC)
    S, n = gp.foot_points()
    ex = gp.export(which=("normal",))
    torch.cuda.synchronize()
    h = min(op.grid.h[: op.dim])
    want = ghost_centres(op) + op.delta
    check_close(host(S), want, np.full(want.shape, h), "foot points")
    assert np.array_equal(host(n), host(ex["normal"]))
    assert S.shape == (op.dim, op.n_ghost)


def test_plan_long_chunk_scan(gcr):
    # 8320^2 = 69.2M cells: 16,900 classification chunks, more than two scan
    # tiles, so the chunk scan takes its three-pass form
    n = 8320
    h = 4.0 / n
    grid = synth.Grid(2, (n, n, 1), (-2.0, -2.0, 0.0), (h, h, 1.0))
    shape = synth.Shape(synth.SPHERE, (0.3 * h, 0.7 * h, 0.0), 0.5)
    op, gp = plan_pair(gcr, synth.Instance("circle8320", grid, shape, HGC, []), HGC)
    assert op.min_margin > 1e-9
    check_plan(op, gp, strict_geometry=True)


# ---------------------------------------------------------------------------
# second ghost layer (Sec. 7.1)
# ---------------------------------------------------------------------------

def _layer2_case(case):
    if case == "circle128":
        return synth.circle128(seed=5)
    if case == "sphere_ragged":
        h = 2.0 / 61
        grid = synth.Grid(3, (61, 53, 47), (-1.0, -0.9, -0.8), (h, h, h))
        shape = synth.Shape(synth.SPHERE, (0.013, -0.02, 0.007), 0.41)
        return synth.Instance("sphere_ragged", grid, shape, HGC, synth.abc_fields())
    if case == "star":
        return synth.stars64(seed=3, ninst=1, nmin=200, nmax=300)[0]
    return synth.shstar384(seed=2, n=96, nt=4, nph=8)


@pytest.mark.parametrize("case", ["circle128", "sphere_ragged", "star", "shstar"])
@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_second_layer_plan_and_fill(gcr, case, scheme):
    inst = _layer2_case(case)
    sch = scheme | synth.LAYER2
    op, gp = plan_pair(gcr, inst, sch)
    assert op.min_margin > 1e-9
    op1 = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    assert op.n_ghost > op1.n_ghost
    assert gp.n_interface == op.n_interface
    check_plan(op, gp, strict_geometry=case in ("circle128", "sphere_ragged"))
    flds = (list(inst.fields) * 2)[:2]
    run_fill(gcr, op, gp, inst, flds, [DIRICHLET, NEUMANN])


def test_second_layer_batch_mixed_flags(gcr):
    # one batch: instances with and without the second layer
    insts = synth.stars64(seed=5, ninst=4, nmin=96, nmax=400)
    schemes = [HGC | synth.LAYER2, HGC, CGC | synth.LAYER2, CGC_ES]
    B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], schemes)
    for inst, sch, bp in zip(insts, schemes, B.plans):
        op = oracle.OraclePlan(inst.grid, inst.shape, sch)
        check_plan(op, bp)


# ---------------------------------------------------------------------------
# stretched grids (cell faces per axis; local widths in Eq. delta_n and
# Eq. stencil_anisotropic, centre differences as stencil spans)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["circle0", "circle1", "sphere"])
@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
def test_stretched_plan_fill_surface(gcr, which, scheme):
    inst = synth.sphere_stretched(seed=0) if which == "sphere" else \
        synth.circle_stretched(seed=int(which[-1]))
    op, gp = plan_pair(gcr, inst, scheme)
    assert op.min_margin > 1e-9
    check_plan(op, gp, strict_geometry=True)
    flds = (list(inst.fields) * 2)[:2]
    got, want, scale = run_fill(gcr, op, gp, inst, flds, [DIRICHLET, NEUMANN])
    cs = op.cell_scale(np.nan_to_num(want), scale)
    v, g, anc = gp.surface(dev(inst.queries.x), [dev(x) for x in got])
    ov, og, oanc, osc = op.surface_query(inst.queries.x, want, field_scale=cs)
    assert np.array_equal(host(anc), oanc)
    check_close(host(v), ov, osc[:, 0], "query value")
    check_close(host(g), og, osc[:, 1:], "query gradient")


def test_stretched_batch_forward(gcr):
    insts = [synth.circle_stretched(seed=s) for s in range(3)]
    B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], [HGC] * 3)
    fields, bcv, refs = [], [], []
    for inst, bp in zip(insts, B.plans):
        op = oracle.OraclePlan(inst.grid, inst.shape, HGC)
        check_plan(op, bp, strict_geometry=True)
        f = inst.fields[0]
        vals = synth.sample(f, inst.grid)
        vals[op.tags != 0] = np.nan
        S = np.stack([inst.grid.centres(a)[[op.ghost_cell % inst.grid.n[0],
                                           op.ghost_cell // inst.grid.n[0]][a]]
                      for a in range(2)]) + op.delta
        b = synth.bc_values(f, S, op.normal, DIRICHLET)
        want = op.fill(vals[None].copy(), [DIRICHLET], b[None])[0]
        sc = op.fill_scale(np.nan_to_num(vals)[None], [DIRICHLET], b[None])[0]
        refs.append((op, want, sc))
        fields.append(dev(vals))
        bcv.append(dev(b))
    B.forward(1, fields, [DIRICHLET], bcv)
    torch.cuda.synchronize()
    for (op, want, sc), fld in zip(refs, fields):
        c = op.ghost_cell
        check_close(host(fld)[c], want[c], sc, "batched fill on a stretched grid")


@pytest.mark.parametrize("scheme", [CGC, CGC_ES, HGC])
@pytest.mark.parametrize("which", ["circle", "sphere"])
def test_stretched_second_layer(gcr, which, scheme):
    """Second ghost layer on a stretched grid (candidate box from the
    largest and smallest cell widths): plan, fill and surface against the
    oracle."""
    inst = synth.sphere_stretched(seed=2) if which == "sphere" else synth.circle_stretched(seed=0)
    op, gp = plan_pair(gcr, inst, scheme | synth.LAYER2)
    assert op.min_margin > 1e-9
    check_plan(op, gp, strict_geometry=True)
    flds = (list(inst.fields) * 2)[:2]
    got, want, scale = run_fill(gcr, op, gp, inst, flds, [DIRICHLET, NEUMANN])
    cs = op.cell_scale(np.nan_to_num(want), scale)
    v, g, anc = gp.surface(dev(inst.queries.x), [dev(x) for x in got])
    ov, og, oanc, osc = op.surface_query(inst.queries.x, want, field_scale=cs)
    assert np.array_equal(host(anc), oanc)
    check_close(host(v), ov, osc[:, 0], "query value")
    check_close(host(g), og, osc[:, 1:], "query gradient")


def test_stretched_second_layer_refused_beyond_box_limit(gcr):
    # widths growing 20 % per cell: the candidate box would exceed 64 cells
    n = 64
    f = synth.stretched_faces(n, -2.0, 2.0, 1.2)
    grid = synth.Grid(2, (n, n, 1), (-2.0, -2.0, 0.0), (4.0 / n, 4.0 / n, 1.0), (f, f, None))
    shape = synth.Shape(synth.SPHERE, (0.01, 0.02, 0.0), 0.5)
    with pytest.raises(gcr.GcrError):
        gcr.Plan(grid, shape, HGC | synth.LAYER2)
    gcr.Plan(grid, shape, HGC)   # the first layer alone is fine


# ---------------------------------------------------------------------------
# cycles: the remainder of a stalled Kahn layering resolved by one wave or
# by the workgroup (Sec. 3.2: coupled units, levels by longest path)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which", [0, 32, 33, 63, "small"])
def test_cycle_remainder_wave_and_workgroup_agree(gcr, which):
    """Instances whose layering stalls on cycles (four of the 64-star
    workload, and a small star): built with the one-wave remainder solver
    and with the workgroup path, every exported array bit for bit the same,
    and both equal to the oracle (levels, order, units)."""
    if which == "small":
        inst, scheme = synth.stars64(seed=0, ninst=1, nmin=96, nmax=160)[0], CGC
    else:
        inst, scheme = synth.stars64(seed=0)[which], HGC
    op = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    exports = []
    try:
        for limit in (64, 0):
            gcr.set_wave_residual(limit)
            gp = gcr.Plan(inst.grid, inst.shape, scheme)
            exports.append((check_plan(op, gp), gp.stats()))
    finally:
        gcr.set_wave_residual(64)
    (a, sa), (b, sb) = exports
    for k in a:
        assert np.array_equal(host(a[k]), host(b[k]), equal_nan=True), k
    for k in ("n_units_coupled", "max_unit", "n_levels", "max_level_width"):
        assert sa[k] == sb[k], k
    assert sa["n_units_coupled"] >= 1 or op.n_units_coupled == 0
    with pytest.raises(gcr.GcrError):
        gcr.set_wave_residual(65)


def test_canonical_order_of_a_deep_plan(gcr):
    """The canonical ghost order, level then linear index, on a plan deeper
    than 128 levels (the airfoil on a 7168^2 grid: 141 levels, the thin
    trailing edge being a long dependency chain), so that a ghost's rank
    among those of its level uses every bit of the level index: levels
    ascend, cells ascend within a level, and the level offsets count them."""
    inst = synth.airfoil4096(seed=0, n=7168)
    p = gcr.Plan(inst.grid, inst.shape, HGC)
    ex = p.export(("cell", "level"))
    torch.cuda.synchronize()
    lev = ex["level"].cpu().numpy().astype(np.int64)
    cell = ex["cell"].cpu().numpy().astype(np.int64)
    off = np.asarray(p.level_offsets())
    nl = len(off) - 1
    print(f"airfoil n=7168: {cell.size} ghosts, {nl} levels", flush=True)
    assert 128 < nl <= 256
    assert lev[0] == 1 and np.all(np.diff(lev) >= 0)
    same = np.diff(lev) == 0
    assert np.all(np.diff(cell)[same] > 0)
    assert np.array_equal(np.searchsorted(lev, np.arange(1, nl + 2)), off)


def test_fill_of_a_plan_without_ghosts(gcr):
    """A body far outside its grid: no ghosts, no levels.  Its fill reads no
    boundary data (zero-size tensors, null pointers, are accepted) and
    leaves the field as it was."""
    grid = synth.Grid(2, (40, 33, 1), (0.0, 0.0, 0.0), (0.1, 0.1, 1.0))
    shape = synth.Shape(synth.SPHERE, (50.0, 50.0, 0.0), 1.0)
    p = gcr.Plan(grid, shape, HGC)
    assert p.n_ghost == 0 and p.level_offsets() == [0]
    u = torch.as_tensor(np.random.default_rng(3).standard_normal(40 * 33), device="cuda")
    before = u.clone()
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    p.fill([u], [DIRICHLET], [empty])
    p.fill([u], [2], [empty], bc_type=[torch.empty(0, dtype=torch.uint8, device="cuda")])
    torch.cuda.synchronize()
    assert torch.equal(u, before)
