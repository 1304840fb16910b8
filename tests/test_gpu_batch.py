"""GPU parity of the batched path: plans of many uneven instances built by
shared launches, and the persistent batched forward (fill of several fields
with mixed Dirichlet/Neumann data + force), against the oracle per instance
and against the single-instance path."""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
import synth
from synth import HGC
from tolerances import check, force_scale

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gcr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_10165_amd as g
    g.lib()
    return g


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def ghost_centres(op):
    g = op.grid
    c = op.ghost_cell
    return np.stack([g.lo[0] + (c % g.n[0] + 0.5) * g.h[0],
                     g.lo[1] + (c // g.n[0] + 0.5) * g.h[1]])


def run_batch(gcr, insts, with_forces=True, fwd_kw=None):
    B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], [HGC] * len(insts))
    nf = 3
    ops, fields, bcv, bct, host_in, wants = [], [], [], [], [], []
    for inst, plan in zip(insts, B.plans):
        op = oracle.OraclePlan(inst.grid, inst.shape, HGC)
        ops.append(op)
        S = ghost_centres(op) + op.delta
        kinds = [synth.mixed_kinds(S, inst.shape.center, b) for b in inst.mixed_beta]
        vals = np.stack([synth.sample(f, inst.grid) for f in inst.fields])
        vals[:, op.tags != 0] = np.nan
        b = np.stack([synth.bc_values(f, S, op.normal, k) for f, k in zip(inst.fields, kinds)])
        want = op.fill(vals.copy(), np.stack(kinds), b)
        sc = op.fill_scale(np.nan_to_num(vals), np.stack(kinds), b)
        wants.append((want, sc))
        host_in.append(vals)
        for f in range(nf):
            fields.append(dev(vals[f]))
            bcv.append(dev(b[f]))
            bct.append(dev(kinds[f], torch.uint8))
    kw = {}
    F = None
    if with_forces:
        nq = [i.queries.x.shape[1] for i in insts]
        xq = [dev(i.queries.x) for i in insts]
        nr = [dev(i.queries.n) for i in insts]
        wq = [dev(i.queries.w) for i in insts]
        F = torch.zeros((len(insts), 3), dtype=torch.float64, device="cuda")
        kw = dict(nq=nq, xq=xq, nrm=nr, wq=wq, p_field=2, u_first=0, mu=0.9, F=F)
    B.forward(nf, fields, [2, 2, 2], bcv, bc_type=bct, **kw, **(fwd_kw or {}))
    torch.cuda.synchronize()
    return B, ops, fields, wants, F


def test_batch_plans_match_single_plans(gcr):
    insts = synth.stars64(seed=5, ninst=6, nmin=96, nmax=600)
    B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], [HGC] * len(insts))
    for inst, bp in zip(insts, B.plans):
        sp = gcr.Plan(inst.grid, inst.shape, HGC)
        a, b = bp.export(), sp.export()
        torch.cuda.synchronize()
        for k in ("tags", "cell", "level", "r", "unit"):
            assert torch.equal(a[k], b[k]), k
        for k in ("delta", "normal", "psi"):
            assert torch.equal(a[k], b[k]), k
        assert bp.level_offsets() == sp.level_offsets()


@pytest.mark.parametrize("seed,ninst", [(6, 8), (9, 11)])
def test_batch_forward_matches_oracle(gcr, seed, ninst):
    """Fills and forces of every instance against the oracle.  With 11
    instances the launch's item order places eight instances' field items
    8 workgroups apart and leaves the last three in place."""
    insts = synth.stars64(seed=seed, ninst=ninst, nmin=96, nmax=500)
    B, ops, fields, wants, F = run_batch(gcr, insts)
    nf = 3
    for i, (op, (want, sc)) in enumerate(zip(ops, wants)):
        for f in range(nf):
            got = host(fields[i * nf + f])
            err = np.abs(got[op.ghost_cell] - want[f][op.ghost_cell])
            assert np.all(err <= 1e-12 * np.maximum(np.abs(want[f][op.ghost_cell]), sc[f])), (i, f)
        inst = insts[i]
        q = inst.queries
        Fo = op.forces(q.x, q.n, q.w, want[2], want[:2], 0.9)
        cs = op.cell_scale(np.nan_to_num(want), sc)
        check(host(F[i])[:2], Fo, force_scale(op, q, want, cs, 2, [0, 1], 0.9), f"force {i}")


def test_batch_forward_plan_beyond_lds_records(gcr):
    """A 2D batch whose largest plan (a star on 4096^2, about 4,300 ghosts)
    has more ghosts than a workgroup's LDS holds records for: its items
    sweep their levels from HBM, one ghost per thread.  Fills and forces of
    every instance against the oracle."""
    insts = synth.stars64(seed=0, ninst=1, nmin=4096, nmax=4096) + \
        synth.stars64(seed=2, ninst=2, nmin=96, nmax=300)
    B, ops, fields, wants, F = run_batch(gcr, insts)
    assert ops[0].n_ghost > 3968
    nf = 3
    for i, (op, (want, sc)) in enumerate(zip(ops, wants)):
        for f in range(nf):
            got = host(fields[i * nf + f])
            err = np.abs(got[op.ghost_cell] - want[f][op.ghost_cell])
            assert np.all(err <= 1e-12 * np.maximum(np.abs(want[f][op.ghost_cell]), sc[f])), (i, f)
        q = insts[i].queries
        Fo = op.forces(q.x, q.n, q.w, want[2], want[:2], 0.9)
        cs = op.cell_scale(np.nan_to_num(want), sc)
        check(host(F[i])[:2], Fo, force_scale(op, q, want, cs, 2, [0, 1], 0.9), f"force {i}")


def test_batch_forward_eight_fields(gcr):
    """The most fields a call takes (8) over 9 instances: the launch's item
    order places eight instances' 8 field items 8 workgroups apart and
    leaves the ninth instance's in place.  Dirichlet and Neumann fields in
    turn, no force; every fill against the oracle."""
    insts = synth.stars64(seed=11, ninst=9, nmin=96, nmax=260)
    B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], [HGC] * len(insts))
    nf = 8
    kinds = [f % 2 for f in range(nf)]
    rng = np.random.default_rng(8)
    ops, fields, bcv, wants = [], [], [], []
    for inst in insts:
        op = oracle.OraclePlan(inst.grid, inst.shape, HGC)
        ops.append(op)
        vals = rng.standard_normal((nf, op.n_cells))
        vals[:, op.tags != 0] = np.nan
        b = rng.standard_normal((nf, op.n_ghost))
        kk = np.repeat(np.asarray(kinds, np.int8)[:, None], op.n_ghost, axis=1)
        wants.append((op.fill(vals.copy(), kk, b), op.fill_scale(np.nan_to_num(vals), kk, b)))
        for f in range(nf):
            fields.append(dev(vals[f]))
            bcv.append(dev(b[f]))
    B.forward(nf, fields, kinds, bcv)
    torch.cuda.synchronize()
    for i, (op, (want, sc)) in enumerate(zip(ops, wants)):
        c = op.ghost_cell
        for f in range(nf):
            got = host(fields[i * nf + f])
            check(got[c], want[f][c], sc[f], f"instance {i} field {f}")


def test_batch_forward_uneven_points(gcr):
    """Surface points spread unevenly over the instances (256, 8, 0, 24, 8,
    8: the anchor search runs as one row of workgroups, each point finding
    its instance) and evenly (24 each: a row of workgroups per instance).
    Surface values, gradients and forces against the oracle's at 1e-12 of
    its propagated scales, both times."""
    insts = synth.stars64(seed=3, ninst=6, nmin=96, nmax=400)
    B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], [HGC] * len(insts))
    nf, mu = 3, 0.8
    ops, fields, bcv, bct, wants = [], [], [], [], []
    for inst in insts:
        op = oracle.OraclePlan(inst.grid, inst.shape, HGC)
        ops.append(op)
        S = ghost_centres(op) + op.delta
        kinds = np.stack([synth.mixed_kinds(S, inst.shape.center, b) for b in inst.mixed_beta])
        vals = np.stack([synth.sample(f, inst.grid) for f in inst.fields])
        vals[:, op.tags != 0] = np.nan
        b = np.stack([synth.bc_values(f, S, op.normal, k) for f, k in zip(inst.fields, kinds)])
        want = op.fill(vals.copy(), kinds, b)
        sc = op.fill_scale(np.nan_to_num(vals), kinds, b)
        wants.append((want, op.cell_scale(np.nan_to_num(want), sc)))
        for f in range(nf):
            fields.append(dev(vals[f]))
            bcv.append(dev(b[f]))
            bct.append(dev(kinds[f], torch.uint8))
    for counts in ([256, 8, 0, 24, 8, 8], [24] * 6):
        qs = [(i.queries.x[:, :k], i.queries.n[:, :k], i.queries.w[:k]) for i, k in zip(insts, counts)]
        F = torch.zeros((len(insts), 3), dtype=torch.float64, device="cuda")
        sv = [torch.empty(k, dtype=torch.float64, device="cuda") for k in counts for _ in range(nf)]
        sg = [torch.empty((2, k), dtype=torch.float64, device="cuda") for k in counts for _ in range(nf)]
        B.forward(nf, fields, [2, 2, 2], bcv, bc_type=bct, nq=counts,
                  xq=[dev(x) for x, _, _ in qs], nrm=[dev(n) for _, n, _ in qs],
                  wq=[dev(w) for _, _, w in qs], p_field=2, u_first=0, mu=mu, F=F,
                  sval=sv, sgrad=sg)
        torch.cuda.synchronize()
        for i, (op, (want, cs)) in enumerate(zip(ops, wants)):
            x, n, w = qs[i]
            if counts[i] == 0:
                assert np.all(host(F[i]) == 0), (counts, i)
                continue
            ov, og, oanc, osc = op.surface_query(x, want, field_scale=cs)
            bv = np.stack([host(sv[i * nf + f]) for f in range(nf)])
            bg = np.stack([host(sg[i * nf + f]) for f in range(nf)])
            check(bv, ov, osc[:, 0], f"{counts} surface values {i}")
            check(bg, og, osc[:, 1:], f"{counts} surface gradients {i}")
            Fo = op.forces(x, n, w, want[2], want[:2], mu)
            q = SimpleNamespace(x=x, n=n, w=w)
            check(host(F[i])[:2], Fo, force_scale(op, q, want, cs, 2, [0, 1], mu),
                  f"{counts} force {i}")


def test_batch_forward_full_size(gcr):
    """The batched workload at its full size: 64 instances, n ~ U{128..2048}
    (107M cells, about 105K ghosts), three fields with mixed
    Dirichlet/Neumann data, one persistent launch.  Every instance against
    the oracle: tags, ghost order and levels bit for bit; fills, surface
    values and gradients at its 256 points and its force at 1e-12 of the
    oracle's propagated scales; cells that are not ghosts untouched."""
    insts = synth.stars64(seed=0)
    assert len(insts) == 64
    B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], [HGC] * len(insts))
    nf = 3
    mu = 1.0
    ops, fields, bcv, bct, ref = [], [], [], [], []
    for inst, plan in zip(insts, B.plans):
        op = oracle.OraclePlan(inst.grid, inst.shape, HGC)
        assert op.min_margin > 1e-9
        ex = plan.export(("tags", "cell", "level"))
        torch.cuda.synchronize()
        assert np.array_equal(host(ex["tags"]), op.tags), inst.name
        assert np.array_equal(host(ex["cell"]).astype(np.int64), op.ghost_cell), inst.name
        assert np.array_equal(host(ex["level"]), op.level), inst.name
        assert plan.level_offsets() == list(op.level_off), inst.name
        del ex
        ops.append(op)
        S = ghost_centres(op) + op.delta
        kinds = np.stack([synth.mixed_kinds(S, inst.shape.center, b) for b in inst.mixed_beta])
        vals = np.stack([synth.sample(f, inst.grid) for f in inst.fields])
        vals[:, op.tags != 0] = np.nan
        b = np.stack([synth.bc_values(f, S, op.normal, k) for f, k in zip(inst.fields, kinds)])
        for f in range(nf):
            fields.append(dev(vals[f]))
            bcv.append(dev(b[f]))
            bct.append(dev(kinds[f], torch.uint8))
        ref.append((b, kinds))
    nq = [i.queries.x.shape[1] for i in insts]
    F = torch.zeros((len(insts), 3), dtype=torch.float64, device="cuda")
    sv = [torch.empty(n, dtype=torch.float64, device="cuda") for n in nq for _ in range(nf)]
    sg = [torch.empty((2, n), dtype=torch.float64, device="cuda") for n in nq for _ in range(nf)]
    B.forward(nf, fields, [2, 2, 2], bcv, bc_type=bct, nq=nq,
              xq=[dev(i.queries.x) for i in insts], nrm=[dev(i.queries.n) for i in insts],
              wq=[dev(i.queries.w) for i in insts], p_field=2, u_first=0, mu=mu, F=F,
              sval=sv, sgrad=sg)
    torch.cuda.synchronize()
    Fh = host(F)
    assert np.all(Fh[:, 2] == 0)
    for k, (inst, op) in enumerate(zip(insts, ops)):
        b, kinds = ref[k]
        vals = np.stack([synth.sample(f, inst.grid) for f in inst.fields])
        vals[:, op.tags != 0] = np.nan
        want = op.fill(vals, kinds, b)
        sc = op.fill_scale(np.nan_to_num(vals), kinds, b)
        c = op.ghost_cell
        nong = np.ones(op.n_cells, bool)
        nong[c] = False
        for f in range(nf):
            got = host(fields[k * nf + f])
            check(got[c], want[f][c], sc[f], f"{inst.name} fill field {f}")
            assert np.array_equal(np.isnan(got[nong]), np.isnan(vals[f][nong])), inst.name
            keep = nong & ~np.isnan(vals[f])
            assert np.array_equal(got[keep], vals[f][keep]), inst.name
        cs = op.cell_scale(np.nan_to_num(want), sc)
        q = inst.queries
        ov, og, oanc, osc = op.surface_query(q.x, want, field_scale=cs)
        bv = np.stack([host(sv[k * nf + f]) for f in range(nf)])
        bg = np.stack([host(sg[k * nf + f]) for f in range(nf)])
        check(bv, ov, osc[:, 0], f"{inst.name} surface values")
        check(bg, og, osc[:, 1:], f"{inst.name} surface gradients")
        Fo = op.forces(q.x, q.n, q.w, want[2], want[:2], mu)
        check(Fh[k, :2], Fo, force_scale(op, q, want, cs, 2, [0, 1], mu), f"{inst.name} force")


def test_batch_three_schemes_sphere256_full_size(gcr):
    """The benchmark step's configuration: the 256^3 sphere with CGC, CGC_ES
    and HGC built as one batch, u, v, w (Dirichlet) and p (Neumann) filled
    with the force in one persistent launch, then surface values and
    gradients per plan; every scheme against the oracle at full size."""
    from synth import CGC, CGC_ES
    inst = synth.sphere256(seed=0)
    g = inst.grid
    schemes = [CGC, CGC_ES, HGC]
    kinds = [f.bc for f in inst.fields]
    B = gcr.Batch([g] * 3, [inst.shape] * 3, schemes)
    ops, fields, bcv, wants, vals_in = [], [], [], [], []
    for sch, plan in zip(schemes, B.plans):
        op = oracle.OraclePlan(g, inst.shape, sch)
        ops.append(op)
        ex = plan.export(("tags", "cell", "level"))
        torch.cuda.synchronize()
        assert np.array_equal(host(ex["tags"]), op.tags), sch
        assert np.array_equal(host(ex["cell"]).astype(np.int64), op.ghost_cell), sch
        assert np.array_equal(host(ex["level"]), op.level), sch
        assert plan.level_offsets() == list(op.level_off), sch
        c = op.ghost_cell
        xc = np.stack([g.lo[0] + (c % g.n[0] + 0.5) * g.h[0],
                       g.lo[1] + ((c // g.n[0]) % g.n[1] + 0.5) * g.h[1],
                       g.lo[2] + (c // (g.n[0] * g.n[1]) + 0.5) * g.h[2]])
        S = xc + op.delta
        vals = np.stack([synth.sample(f, g) for f in inst.fields])
        vals[:, op.tags != 0] = np.nan
        bt = np.broadcast_to(np.asarray(kinds, np.int8)[:, None], (4, op.n_ghost))
        b = np.stack([synth.bc_values(f, S, op.normal, k) for f, k in zip(inst.fields, kinds)])
        wants.append((op.fill(vals.copy(), bt, b), op.fill_scale(np.nan_to_num(vals), bt, b)))
        vals_in.append(vals)
        fields += [dev(v) for v in vals]
        bcv += [dev(x) for x in b]
    q = inst.queries
    nq = q.x.shape[1]
    xq, nr, wq = dev(q.x), dev(q.n), dev(q.w)
    mu = 0.7
    F = torch.zeros((3, 3), dtype=torch.float64, device="cuda")
    sv = [torch.empty(nq, dtype=torch.float64, device="cuda") for _ in range(12)]
    sg = [torch.empty((3, nq), dtype=torch.float64, device="cuda") for _ in range(12)]
    B.forward(4, fields, kinds, bcv, nq=[nq] * 3, xq=[xq] * 3, nrm=[nr] * 3, wq=[wq] * 3,
              p_field=3, u_first=0, mu=mu, F=F, sval=sv, sgrad=sg)
    torch.cuda.synchronize()
    for i, (op, plan) in enumerate(zip(ops, B.plans)):
        want, sc = wants[i]
        got = np.stack([host(fields[4 * i + f]) for f in range(4)])
        c = op.ghost_cell
        for f in range(4):
            err = np.abs(got[f][c] - want[f][c])
            assert np.all(err <= 1e-12 * np.maximum(np.abs(want[f][c]), sc[f])), (i, f)
            nong = np.ones(op.n_cells, bool)
            nong[c] = False
            keep = nong & ~np.isnan(vals_in[i][f])
            assert np.array_equal(got[f][keep], vals_in[i][f][keep]), (i, f)
        cs = op.cell_scale(np.nan_to_num(want), sc)
        Fo = op.forces(q.x, q.n, q.w, want[3], want[:3], mu)
        check(host(F[i]), Fo, force_scale(op, q, want, cs, 3, [0, 1, 2], mu), f"force {i}")
        v, gr, anc = plan.surface(xq, fields[4 * i:4 * i + 4])
        ov, og, oanc, osc = op.surface_query(q.x, want, field_scale=cs)
        assert np.array_equal(host(anc), oanc), i
        assert np.all(np.abs(host(v) - ov) <= 1e-12 * np.maximum(np.abs(ov), osc[:, 0])), i
        assert np.all(np.abs(host(gr) - og) <= 1e-12 * np.maximum(np.abs(og), osc[:, 1:])), i
        # the same values and gradients written by the forward launch itself
        bv = np.stack([host(sv[4 * i + f]) for f in range(4)])
        bg = np.stack([host(sg[4 * i + f]) for f in range(4)])
        assert np.all(np.abs(bv - ov) <= 1e-12 * np.maximum(np.abs(ov), osc[:, 0])), i
        assert np.all(np.abs(bg - og) <= 1e-12 * np.maximum(np.abs(og), osc[:, 1:])), i


def test_batch_forward_with_coupled_units(gcr):
    """CGC on concave stars: instances with coupled units (solved by a unit
    tile of their level) beside instances without, against the oracle."""
    from synth import CGC
    insts = synth.stars64(seed=0, ninst=1, nmin=96, nmax=160) + \
        synth.stars64(seed=7, ninst=3, nmin=96, nmax=300)
    B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], [CGC] * len(insts))
    nf = 3
    ops, fields, bcv, bct, wants = [], [], [], [], []
    for inst in insts:
        op = oracle.OraclePlan(inst.grid, inst.shape, CGC)
        ops.append(op)
        S = ghost_centres(op) + op.delta
        kinds = [synth.mixed_kinds(S, inst.shape.center, b) for b in inst.mixed_beta]
        vals = np.stack([synth.sample(f, inst.grid) for f in inst.fields])
        vals[:, op.tags != 0] = np.nan
        b = np.stack([synth.bc_values(f, S, op.normal, k) for f, k in zip(inst.fields, kinds)])
        wants.append((op.fill(vals.copy(), np.stack(kinds), b),
                      op.fill_scale(np.nan_to_num(vals), np.stack(kinds), b)))
        for f in range(nf):
            fields.append(dev(vals[f]))
            bcv.append(dev(b[f]))
            bct.append(dev(kinds[f], torch.uint8))
    assert ops[0].n_units_coupled >= 1
    B.forward(nf, fields, [2, 2, 2], bcv, bc_type=bct)
    torch.cuda.synchronize()
    for i, (op, (want, sc)) in enumerate(zip(ops, wants)):
        for f in range(nf):
            got = host(fields[i * nf + f])
            c = op.ghost_cell
            err = np.abs(got[c] - want[f][c])
            assert np.all(err <= 1e-12 * np.maximum(np.abs(want[f][c]), sc[f])), (i, f)


def test_batch_forward_with_an_empty_plan(gcr):
    """The batched forward over instances of which one has no ghosts (its
    body far outside its grid) and one sits on a stretched grid: the other
    instances' fills and forces against the oracle, the empty one's field
    untouched and its force zero."""
    insts = synth.stars64(seed=4, ninst=2, nmin=96, nmax=300) + [synth.circle_stretched(seed=1)]
    grids = [i.grid for i in insts]
    shapes = [i.shape for i in insts]
    grids.insert(1, synth.Grid(2, (40, 33, 1), (0.0, 0.0, 0.0), (0.1, 0.1, 1.0)))
    shapes.insert(1, synth.Shape(synth.SPHERE, (50.0, 50.0, 0.0), 1.0))
    B = gcr.Batch(grids, shapes, [HGC] * len(grids))
    assert B.plans[1].n_ghost == 0
    nf, mu = 3, 0.6
    rng = np.random.default_rng(5)
    ops, fields, bcv, wants, qs, before = [], [], [], [], [], []
    for k, (grid, shape) in enumerate(zip(grids, shapes)):
        op = oracle.OraclePlan(grid, shape, HGC)
        ops.append(op)
        vals = rng.standard_normal((nf, op.n_cells))
        vals[:, op.tags != 0] = np.nan
        b = rng.standard_normal((nf, op.n_ghost))
        kinds = np.zeros((nf, op.n_ghost), np.int8)
        kinds[1] = 1
        if op.n_ghost:
            want = op.fill(vals.copy(), kinds, b)
            sc = op.fill_scale(np.nan_to_num(vals), kinds, b)
            wants.append((want, op.cell_scale(np.nan_to_num(want), sc), sc))
        else:
            wants.append(None)
        before.append(vals)
        for f in range(nf):
            fields.append(dev(vals[f]))
            bcv.append(dev(b[f]))
        # (the empty instance gets no surface points)
        q = insts[k if k < 1 else k - 1].queries
        qs.append(q if op.n_ghost else SimpleNamespace(x=q.x[:, :0], n=q.n[:, :0], w=q.w[:0]))
    F = torch.full((len(grids), 3), 7.0, dtype=torch.float64, device="cuda")
    B.forward(nf, fields, [0, 1, 0], bcv, nq=[q.x.shape[1] for q in qs],
              xq=[dev(q.x) for q in qs], nrm=[dev(q.n) for q in qs], wq=[dev(q.w) for q in qs],
              p_field=2, u_first=0, mu=mu, F=F)
    torch.cuda.synchronize()
    for k, op in enumerate(ops):
        got = np.stack([host(fields[k * nf + f]) for f in range(nf)])
        if wants[k] is None:
            assert np.array_equal(np.isnan(got), np.isnan(before[k]))
            assert np.array_equal(np.nan_to_num(got), np.nan_to_num(before[k]))
            assert np.all(host(F[k]) == 0), k
            continue
        want, cs, sc = wants[k]
        c = op.ghost_cell
        for f in range(nf):
            check(got[f][c], want[f][c], sc[f], f"fill {k} field {f}")
        q = qs[k]
        Fo = op.forces(q.x, q.n, q.w, want[2], want[:2], mu)
        check(host(F[k])[:2], Fo, force_scale(op, q, want, cs, 2, [0, 1], mu), f"force {k}")


def test_batch_foot_points(gcr):
    """gcr_batch_foot_points: the instances' foot points and normals one
    after another, bitwise equal to each plan's own gcr_plan_foot_points and
    within 1e-12 of a cell width of the oracle's S = x_c + delta; instances on
    different grids (one stretched), one of them without ghosts."""
    insts = synth.stars64(seed=7, ninst=3, nmin=96, nmax=400) + [synth.circle_stretched(seed=1)]
    grids = [i.grid for i in insts]
    shapes = [i.shape for i in insts]
    # body far outside its grid: no ghosts
    grids.insert(2, synth.Grid(2, (40, 33, 1), (0.0, 0.0, 0.0), (0.1, 0.1, 1.0)))
    shapes.insert(2, synth.Shape(synth.SPHERE, (50.0, 50.0, 0.0), 1.0))
    B = gcr.Batch(grids, shapes, [HGC] * len(grids))
    S, n = B.foot_points()
    assert B.plans[2].n_ghost == 0
    off = 0
    for grid, shape, plan in zip(grids, shapes, B.plans):
        Sp, n_p = plan.foot_points()
        ng = plan.n_ghost
        assert torch.equal(S[:, off:off + ng], Sp) and torch.equal(n[:, off:off + ng], n_p)
        op = oracle.OraclePlan(grid, shape, HGC)
        assert op.n_ghost == ng
        c = op.ghost_cell
        want = np.stack([grid.centres(0)[c % grid.n[0]], grid.centres(1)[c // grid.n[0]]])
        want = want + op.delta
        h = min(grid.widths(0).min(), grid.widths(1).min())
        assert np.all(np.abs(host(S[:, off:off + ng]) - want) <= 1e-12 * h)
        off += ng
    assert S.shape == (2, off)


def test_batch_released_without_cycle_collection(gcr):
    """A dropped Batch is destroyed at once (its device memory goes back to
    the pool for the next build), while a plan still held keeps the batch's
    arrays alive."""
    import gc
    import weakref
    insts = synth.stars64(seed=8, ninst=2, nmin=96, nmax=200)
    gc.disable()
    try:
        B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], [HGC] * 2)
        owner = weakref.ref(B._owner)
        S0, _ = B.plans[1].foot_points()
        keep = B.plans[1]
        del B
        assert owner() is not None          # the held plan keeps it
        S1, _ = keep.foot_points()
        torch.cuda.synchronize()
        assert torch.equal(S0, S1)
        del keep
        assert owner() is None              # released without the cycle collector
    finally:
        gc.enable()


def test_batch_forward_surface_outputs(gcr):
    """Values and gradients of every filled field at the instances' points,
    written by the batched forward, against the oracle's surface query (and
    gcr_surface on the same filled fields); outputs left out (None entries)
    leave the others intact."""
    insts = synth.stars64(seed=9, ninst=5, nmin=96, nmax=400)
    nf = 3
    nqs = [i.queries.x.shape[1] for i in insts]
    sv = [torch.full((nq,), 7.0, dtype=torch.float64, device="cuda") for nq in nqs for _ in range(nf)]
    sg = [torch.full((2, nq), 7.0, dtype=torch.float64, device="cuda") for nq in nqs for _ in range(nf)]
    sv[1] = None                       # instance 0, field 1: value not wanted
    sg[2 * nf] = None                  # instance 2, field 0: gradient not wanted
    B, ops, fields, wants, F = run_batch(gcr, insts, fwd_kw=dict(sval=sv, sgrad=sg))
    for i, (inst, op, plan) in enumerate(zip(insts, ops, B.plans)):
        want, sc = wants[i]
        cs = op.cell_scale(np.nan_to_num(want), sc)
        ov, og, _, osc = op.surface_query(inst.queries.x, want, field_scale=cs)
        v2, g2, _ = plan.surface(dev(inst.queries.x), fields[i * nf:(i + 1) * nf])
        torch.cuda.synchronize()
        for f in range(nf):
            w = i * nf + f
            if sv[w] is not None:
                got = host(sv[w])
                assert np.all(np.abs(got - ov[f]) <= 1e-12 * np.maximum(np.abs(ov[f]), osc[f, 0])), w
                assert np.all(np.abs(got - host(v2[f])) <= 1e-14 * np.maximum(np.abs(ov[f]), osc[f, 0])), w
            if sg[w] is not None:
                got = host(sg[w])
                assert np.all(np.abs(got - og[f]) <= 1e-12 * np.maximum(np.abs(og[f]), osc[f, 1:])), w
                assert np.all(np.abs(got - host(g2[f])) <= 1e-14 * np.maximum(np.abs(og[f]), osc[f, 1:])), w


def test_batch_forward_packed_args(gcr):
    """ForwardArgs packed once and reused on two fresh batches in a row: the
    same fill, surface values and forces as the unpacked call, bitwise; a
    pack for another number of instances is refused before any launch."""
    insts = synth.stars64(seed=10, ninst=3, nmin=96, nmax=300)
    nf = 3
    base = []
    for inst in insts:
        op = oracle.OraclePlan(inst.grid, inst.shape, HGC)
        vals = np.stack([synth.sample(f, inst.grid) for f in inst.fields])
        vals[:, op.tags != 0] = np.nan
        base += [dev(v) for v in vals]
    grids, shapes = [i.grid for i in insts], [i.shape for i in insts]
    B0 = gcr.Batch(grids, shapes, [HGC] * 3)
    bcv = [dev(np.linspace(0.1, 0.9, p.n_ghost) + f) for p in B0.plans for f in range(nf)]
    nqs = [i.queries.x.shape[1] for i in insts]
    kw = dict(nq=nqs, xq=[dev(i.queries.x) for i in insts], nrm=[dev(i.queries.n) for i in insts],
              wq=[dev(i.queries.w) for i in insts], p_field=2, u_first=0, mu=0.9)
    F = torch.zeros((3, 3), dtype=torch.float64, device="cuda")
    sv = [torch.empty(n, dtype=torch.float64, device="cuda") for n in nqs for _ in range(nf)]
    fk = [b.clone() for b in base]
    B0.forward(nf, fk, [0] * nf, bcv, F=F, sval=sv, **kw)
    torch.cuda.synchronize()
    ref = ([f.clone() for f in fk], F.clone(), [v.clone() for v in sv])

    def same(a, b):
        return torch.equal(a.isnan(), b.isnan()) and torch.equal(a.nan_to_num(), b.nan_to_num())

    work = [b.clone() for b in base]
    args = gcr.ForwardArgs(nf, work, [0] * nf, bcv, F=F, sval=sv, **kw)
    for _ in range(2):
        for w, b in zip(work, base):
            w.copy_(b)
        F.zero_()
        for v in sv:
            v.fill_(7.0)
        Bk = gcr.Batch(grids, shapes, [HGC] * 3)
        Bk.forward(args=args)
        torch.cuda.synchronize()
        assert all(same(a, b) for a, b in zip(work, ref[0]))
        assert torch.equal(F, ref[1])
        assert all(same(a, b) for a, b in zip(sv, ref[2]))
    B2 = gcr.Batch([insts[0].grid], [insts[0].shape], [HGC])
    with pytest.raises(ValueError):
        B2.forward(args=args)


@pytest.mark.parametrize("case", ["stars", "spheres"])
def test_batch_tiled_fill_equals_level_sweep(gcr, case):
    """The tiled fill (closures of tiles in LDS) gives the level-by-level
    sweep's fields, surface values and forces bit for bit."""
    if case == "stars":
        insts = synth.stars64(seed=11, ninst=6, nmin=128, nmax=900)
        schemes, nf, kinds = [HGC] * 6, 3, [0, 0, 1]
    else:
        from synth import CGC, CGC_ES
        insts = [synth.sphere256(seed=1, n=96)] * 3
        schemes, nf, kinds = [CGC, CGC_ES, HGC], 4, [0, 0, 0, 1]
    base = []
    for inst, sch in zip(insts, schemes):
        op = oracle.OraclePlan(inst.grid, inst.shape, sch)
        vals = np.stack([synth.sample(f, inst.grid) for f in inst.fields[:nf]])
        vals[:, op.tags != 0] = np.nan
        base += [dev(v) for v in vals]
    nqs = [i.queries.x.shape[1] for i in insts]
    kw = dict(nq=nqs, xq=[dev(i.queries.x) for i in insts], nrm=[dev(i.queries.n) for i in insts],
              wq=[dev(i.queries.w) for i in insts], p_field=nf - 1, u_first=0, mu=0.8)
    out = []
    for tiled in (True, False):
        gcr.set_batch_tiling(2 if tiled else 0)
        try:
            B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], schemes)
            bcv = [dev(np.cos(np.arange(p.n_ghost) * 0.37 + f)) for p in B.plans for f in range(nf)]
            fk = [b.clone() for b in base]
            F = torch.zeros((len(insts), 3), dtype=torch.float64, device="cuda")
            sv = [torch.empty(n, dtype=torch.float64, device="cuda") for n in nqs for _ in range(nf)]
            B.forward(nf, fk, kinds, bcv, F=F, sval=sv, **kw)
            torch.cuda.synchronize()
            assert B.tiled() == (1 if tiled else -1)
            out.append((fk, F, sv))
        finally:
            gcr.set_batch_tiling(1)

    def same(a, b):
        return torch.equal(a.isnan(), b.isnan()) and torch.equal(a.nan_to_num(), b.nan_to_num())

    (fa, Fa, sa), (fb, Fb, sb) = out
    assert all(same(a, b) for a, b in zip(fa, fb))
    assert torch.equal(Fa, Fb)
    assert all(same(a, b) for a, b in zip(sa, sb))


def test_batch_tiling_from_second_call(gcr):
    """Default mode: the first forward call sweeps the levels, the second
    sets the tiles up and uses them; both give the same fields."""
    insts = synth.stars64(seed=12, ninst=3, nmin=128, nmax=400)
    base = []
    for inst in insts:
        op = oracle.OraclePlan(inst.grid, inst.shape, HGC)
        vals = np.stack([synth.sample(f, inst.grid) for f in inst.fields])
        vals[:, op.tags != 0] = np.nan
        base += [dev(v) for v in vals]
    B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], [HGC] * 3)
    bcv = [dev(np.sin(np.arange(p.n_ghost) * 0.21 + f)) for p in B.plans for f in range(3)]
    outs = []
    for call in range(2):
        fk = [b.clone() for b in base]
        B.forward(3, fk, [0, 0, 1], bcv)
        torch.cuda.synchronize()
        outs.append(fk)
        assert B.tiled() == (0 if call == 0 else 1)
    for a, b in zip(*outs):
        assert torch.equal(a.isnan(), b.isnan()) and torch.equal(a.nan_to_num(), b.nan_to_num())


def test_batch_concurrent_builds_on_two_threads(gcr):
    """Builds from two host threads at once, each on a stream of its own
    (the library's pools, tables and launch attributes shared between them):
    every plan equals, bit for bit, the plan of the same batch built alone,
    and a forward run from one thread while the other builds equals the
    forward run alone."""
    import threading
    from synth import CGC, CGC_ES
    sph = synth.sphere256(seed=0)
    stars = synth.stars64(seed=11, ninst=6, nmin=96, nmax=600)
    cfgs = [([sph.grid] * 3, [sph.shape] * 3, [CGC, CGC_ES, HGC]),
            ([i.grid for i in stars], [i.shape for i in stars], [HGC] * len(stars))]
    keys = ("tags", "cell", "level", "r", "unit", "delta", "normal", "psi")

    def snap(B):
        return [(p.export(keys), p.level_offsets()) for p in B.plans]

    ref = [snap(gcr.Batch(*c)) for c in cfgs]
    # a forward on the star batch alone, then the same from a thread
    rng = np.random.default_rng(3)
    Bs = gcr.Batch(*cfgs[1])
    vals = [rng.standard_normal(i.grid.n[0] * i.grid.n[1]) for i in stars]

    def forward(B, st):
        fields = [dev(v) for v in vals]
        bcv = [torch.full((p.n_ghost,), 0.25, dtype=torch.float64, device="cuda")
               for p in B.plans]
        with torch.cuda.stream(st):
            B.forward(1, fields, [0], bcv, stream=st)
        st.synchronize()
        return [host(f) for f in fields]

    want_fwd = forward(Bs, torch.cuda.current_stream())
    torch.cuda.synchronize()
    got = [[], []]
    fwd_got = []
    err = []

    def work(t):
        st = torch.cuda.Stream()
        try:
            for r in range(6):
                k = (t + r) % 2
                with torch.cuda.stream(st):
                    B = gcr.Batch(*cfgs[k], stream=st)
                    s = snap(B)
                st.synchronize()
                got[t].append((k, s))
                if t == 1 and r % 2 == 0:
                    fwd_got.append(forward(Bs, st))
        except Exception as e:   # noqa: BLE001 - reported below
            err.append(e)

    ths = [threading.Thread(target=work, args=(t,)) for t in range(2)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    assert not err, err
    torch.cuda.synchronize()
    for t in range(2):
        assert len(got[t]) == 6
        for k, s in got[t]:
            for (a, la), (b, lb) in zip(s, ref[k]):
                assert la == lb, (t, k)
                for key in keys:
                    assert torch.equal(a[key], b[key]), (t, k, key)
    assert len(fwd_got) == 3
    for fg in fwd_got:
        for a, b in zip(fg, want_fwd):
            assert np.array_equal(a, b, equal_nan=True)


def _bits(t):
    return t.contiguous().view(torch.int64)


@pytest.mark.parametrize("case", ["spheres", "units", "single", "deep"])
def test_batch_split_sweep_equals_per_item(gcr, case):
    """The split level sweep (several workgroups per instance meeting at a
    device-scope counter between levels) against the per-item sweep: the
    same field values bit for bit, and the same force, surface values and
    gradients bit for bit at the same workgroup size; over several
    workgroups per instance, up to the largest grid allowed, with coupled
    units in the 'units' case.  In the 'deep' case (a 2D airfoil of more
    than 64 levels) the per-item sweep runs from LDS records and reloads its
    level offsets past level 64.  Each launch shape is run twice in a row,
    so both sets of level counters are used."""
    from synth import CGC, CGC_ES
    if case == "deep":
        inst = synth.airfoil4096(seed=0)
        grids, shapes, schemes = [inst.grid], [inst.shape], [HGC]
        kinds = [0, 0, 1]
        qs = [inst.queries]
    elif case == "single":
        inst = synth.sphere256(seed=0)
        grids, shapes, schemes = [inst.grid], [inst.shape], [HGC]
        kinds = [f.bc for f in inst.fields]
        qs = [inst.queries]
    elif case == "spheres":
        inst = synth.sphere256(seed=0)
        grids, shapes, schemes = [inst.grid] * 3, [inst.shape] * 3, [CGC, CGC_ES, HGC]
        kinds = [f.bc for f in inst.fields]
        qs = [inst.queries] * 3
    else:
        insts = synth.stars64(seed=0, ninst=1, nmin=96, nmax=160) + \
            synth.stars64(seed=7, ninst=3, nmin=96, nmax=300)
        grids, shapes = [i.grid for i in insts], [i.shape for i in insts]
        schemes = [CGC] * len(insts)
        kinds = [0, 1, 0]
        qs = [i.queries for i in insts]
    nf = len(kinds)
    gcr.set_batch_tiling(0)
    try:
        B = gcr.Batch(grids, shapes, schemes)
        if case == "units":
            assert any(p.stats()["n_units_coupled"] > 0 for p in B.plans)
        if case == "deep":
            assert len(B.plans[0].level_offsets()) - 1 > 64 and B.plans[0].n_ghost < 3968
        rng = np.random.default_rng(17)
        clean, bcv = [], []
        for g, p in zip(grids, B.plans):
            ncell = int(np.prod(g.n))
            for f in range(nf):
                clean.append(torch.as_tensor(rng.standard_normal(ncell), device="cuda"))
                bcv.append(torch.as_tensor(rng.standard_normal(p.n_ghost), device="cuda"))
        nq = [q.x.shape[1] for q in qs]
        xq, nr, wq = [dev(q.x) for q in qs], [dev(q.n) for q in qs], [dev(q.w) for q in qs]

        def run(threads, grid):
            gcr.set_batch_shape(threads, grid)   # every call on the batch after the first
            fields = [c.clone() for c in clean]
            F = torch.zeros((len(grids), 3), dtype=torch.float64, device="cuda")
            sv = [torch.empty(n, dtype=torch.float64, device="cuda")
                  for n in nq for _ in range(nf)]
            sg = [torch.empty((grids[0].dim, n), dtype=torch.float64, device="cuda")
                  for n in nq for _ in range(nf)]
            B.forward(nf, fields, kinds, bcv, nq=nq, xq=xq, nrm=nr, wq=wq, p_field=nf - 1,
                      u_first=0, mu=0.8, F=F, sval=[s for s in sv], sgrad=[s for s in sg])
            torch.cuda.synchronize()
            return fields, F, sv, sg

        maxg = 256 // len(grids)
        for threads in (1024, 256):
            ref = run(threads, 1)
            for G in sorted({2, 4, 16, min(32, maxg), min(128, maxg)}):
                for _ in range(2):
                    got = run(threads, -G)
                    for a, b in zip(got[0], ref[0]):
                        assert torch.equal(_bits(a), _bits(b)), (threads, G, "field")
                    assert torch.equal(_bits(got[1]), _bits(ref[1])), (threads, G, "force")
                    for a, b in zip(got[2] + got[3], ref[2] + ref[3]):
                        assert torch.equal(_bits(a), _bits(b)), (threads, G, "surface")
    finally:
        gcr.set_batch_shape(0, 0)
        gcr.set_batch_tiling(1)


def test_batch_split_sweep_refuses_oversized_grid(gcr):
    """A forced split shape whose grid would exceed one workgroup per compute
    unit is refused before any launch; bad shapes are refused at once."""
    insts = synth.stars64(seed=12, ninst=20, nmin=96, nmax=128)
    gcr.set_batch_tiling(0)
    try:
        B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], [HGC] * len(insts))
        fields = [torch.zeros(int(np.prod(i.grid.n)), dtype=torch.float64, device="cuda")
                  for i in insts]
        bcv = [torch.zeros(p.n_ghost, dtype=torch.float64, device="cuda") for p in B.plans]
        gcr.set_batch_shape(256, -16)   # 20 x 16 = 320 workgroups
        with pytest.raises(gcr.GcrError):
            B.forward(1, fields, [0], bcv)
        gcr.set_batch_shape(256, -8)    # 160: allowed
        B.forward(1, fields, [0], bcv)
        torch.cuda.synchronize()
        for bad in ((100, 1), (256, 0), (256, 5), (256, -129), (2048, 1)):
            with pytest.raises(gcr.GcrError):
                gcr.set_batch_shape(*bad)
    finally:
        gcr.set_batch_shape(0, 0)
        gcr.set_batch_tiling(1)


def test_batch_split_wait_that_gives_up_is_reported(gcr):
    """The host makes every wait of the split sweep give up after one poll
    (gcr_set_batch_spin(1)): every kernel still ends, and gcr_batch_status
    reports GCR_E_TIMEOUT for the call instead of letting its possibly wrong
    values pass as valid.  With the default limit, the next calls are clean
    again and equal the per-item sweep bit for bit."""
    inst = synth.sphere256(seed=0, n=160)
    kinds = [f.bc for f in inst.fields]
    nf = len(kinds)
    gcr.set_batch_tiling(0)
    try:
        B = gcr.Batch([inst.grid], [inst.shape], [HGC])
        assert B.plans[0].n_levels >= 5
        rng = np.random.default_rng(5)
        clean = [torch.as_tensor(rng.standard_normal(inst.grid.n_cells), device="cuda")
                 for _ in range(nf)]
        bcv = [torch.as_tensor(rng.standard_normal(B.plans[0].n_ghost), device="cuda")
               for _ in range(nf)]

        def run(threads, grid):
            gcr.set_batch_shape(threads, grid)
            fields = [c.clone() for c in clean]
            B.forward(nf, fields, kinds, bcv)
            return fields

        ref = run(256, 1)
        B.status()                                   # clean so far
        gcr.set_batch_spin(1)
        try:
            for _ in range(3):
                run(256, -64)
            with pytest.raises(gcr.GcrError) as e:
                B.status()
            assert e.value.code == 9                 # GCR_E_TIMEOUT
        finally:
            gcr.set_batch_spin(0)
        B.status()                                   # the query cleared the word
        got = run(256, -64)
        B.status()
        for a, b in zip(got, ref):
            assert torch.equal(_bits(a), _bits(b))
        with pytest.raises(gcr.GcrError):
            gcr.set_batch_spin(-1)
    finally:
        gcr.set_batch_shape(0, 0)
        gcr.set_batch_tiling(1)
