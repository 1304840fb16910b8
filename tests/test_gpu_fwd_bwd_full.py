"""The forward + adjoint workload at its full size: a spherical-harmonic star
(l = 2..4) on 384^3 cells, u, v, w (Dirichlet) and p (Neumann), HGC.

Against the oracle on the same inputs: the plan bit for bit (tags, ghost
order, levels, multipliers); the filled ghost values; surface values and
gradients at the 64 x 128 quadrature points (Sec. 6); the drag F_x; and the
gradient of the drag with respect to every interior field value and every
boundary datum (the force adjoint followed by the reverse-level fill
adjoint), element by element at 1e-12 of the oracle's per-entry scales.
Then central differences (step 1e-6) on 32 entries drawn from the
gradient's support, 16 interior cells and 16 boundary data: the drag is
affine in both, so the differences carry rounding only.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import HGC, DIRICHLET, NEUMANN
from tolerances import check, force_gradient, force_scale

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


def test_shstar384_forward_and_adjoint_full_size(gcr):
    inst = synth.shstar384(seed=0)
    g = inst.grid
    assert tuple(g.n) == (384, 384, 384)
    d = 3
    kinds = [f.bc for f in inst.fields]
    assert kinds == [DIRICHLET, DIRICHLET, DIRICHLET, NEUMANN]
    nf = len(kinds)
    mu = 1.0
    q = inst.queries
    assert q.x.shape[1] == 64 * 128

    op = oracle.OraclePlan(g, inst.shape, HGC)
    assert op.min_margin > 1e-9
    gp = gcr.Plan(g, inst.shape, HGC)
    ex = gp.export(("tags", "cell", "level", "r", "delta", "normal"))
    torch.cuda.synchronize()
    assert np.array_equal(host(ex["tags"]), op.tags), "tags"
    assert np.array_equal(host(ex["cell"]).astype(np.int64), op.ghost_cell), "ghost order"
    assert np.array_equal(host(ex["level"]), op.level), "levels"
    assert np.array_equal(host(ex["r"]), op.r), "multipliers"
    assert gp.level_offsets() == list(op.level_off)
    h = g.h[0]
    check(host(ex["delta"]), op.delta, np.full(op.delta.shape, h), "delta")
    check(host(ex["normal"]), op.normal, np.ones(op.normal.shape), "normal")
    del ex

    # ---- forward: fill, surface values and gradients, drag
    c = op.ghost_cell
    idx = [c % g.n[0], (c // g.n[0]) % g.n[1], c // (g.n[0] * g.n[1])]
    S = np.stack([g.lo[i] + (idx[i] + 0.5) * g.h[i] for i in range(d)]) + op.delta
    b0 = np.stack([synth.bc_values(f, S, op.normal, k) for f, k in zip(inst.fields, kinds)])
    vals = np.stack([synth.sample(f, g) for f in inst.fields])
    vals[:, op.tags != 0] = np.nan                   # ghosts and solid cells poisoned
    want = op.fill(vals, kinds, b0)                  # a filled copy
    fscale = op.fill_scale(np.nan_to_num(vals), kinds, b0)
    fields = [dev(v) for v in vals]
    bcs = [dev(x) for x in b0]
    gp.fill(fields, kinds, bcs)
    torch.cuda.synchronize()
    for f in range(nf):
        check(host(fields[f][torch.as_tensor(c, device="cuda")]), want[f][c], fscale[f],
              f"fill field {f}")
    cs = op.cell_scale(np.nan_to_num(want), fscale)
    xq, nq_, wq = dev(q.x), dev(q.n), dev(q.w)
    v, gr, anc = gp.surface(xq, fields)
    ov, og, oanc, osc = op.surface_query(q.x, want, field_scale=cs)
    assert np.array_equal(host(anc), oanc), "anchors"
    check(host(v), ov, osc[:, 0], "surface values")
    check(host(gr), og, osc[:, 1:], "surface gradients")
    F = host(gp.forces(xq, nq_, wq, fields[3], fields[:3], mu))
    Fo = op.forces(q.x, q.n, q.w, want[3], want[:3], mu)
    check(F, Fo, force_scale(op, q, want, cs, 3, [0, 1, 2], mu), "force")
    del cs, osc, want

    # ---- adjoint of the drag J = F_x
    gF = np.array([1.0, 0.0, 0.0])
    lam = [torch.zeros(op.n_cells, dtype=torch.float64, device="cuda") for _ in range(nf)]
    gp.forces_adjoint(xq, nq_, wq, mu, dev(gF), lam[3], lam[:3])
    lam_bc = [torch.empty(op.n_ghost, dtype=torch.float64, device="cuda") for _ in range(nf)]
    gp.fill_adjoint(lam, kinds, lam_bc)
    torch.cuda.synchronize()
    Go, Gbo, So, Sbo = force_gradient(op, q, mu, gF, kinds, 3, [0, 1, 2])
    for f in range(nf):
        G = host(lam[f])
        sup = (Go[f] != 0) | (So[f] != 0)
        assert np.all(G[~sup] == 0), f"gradient off the support, field {f}"
        check(G[sup], Go[f][sup], So[f][sup], f"interior gradient field {f}")
    Gb = np.stack([host(x) for x in lam_bc])
    check(Gb, Gbo, Sbo, "boundary-data gradient")

    # ---- central differences, perturbing device copies in place
    rng = np.random.default_rng(384)
    eps = 1e-6
    work = [dev(np.nan_to_num(v, nan=0.0)) for v in vals]   # interior inputs (solid slots 0)
    del vals

    def J():
        gp.fill(work, kinds, bcs)
        return float(gp.forces(xq, nq_, wq, work[3], work[:3], mu)[0])

    picks = []
    for f in range(nf):
        nz = np.flatnonzero(Go[f])
        picks += [(f, int(x)) for x in nz]
    chosen = rng.choice(len(picks), 16, replace=False)
    for k in chosen:
        f, cell = picks[k]
        x0 = work[f][cell].item()
        work[f][cell] = x0 + eps
        jp = J()
        work[f][cell] = x0 - eps
        jm = J()
        work[f][cell] = x0
        fd = (jp - jm) / (2 * eps)
        want_g = Go[f][cell]
        assert abs(fd - want_g) <= 1e-7 * max(1.0, abs(want_g)), (f, cell, fd, want_g)
    for k in rng.choice(nf * op.n_ghost, 16, replace=False):
        f, gi = divmod(int(k), op.n_ghost)
        x0 = bcs[f][gi].item()
        bcs[f][gi] = x0 + eps
        jp = J()
        bcs[f][gi] = x0 - eps
        jm = J()
        bcs[f][gi] = x0
        fd = (jp - jm) / (2 * eps)
        assert abs(fd - Gbo[f, gi]) <= 1e-7 * max(1.0, abs(Gbo[f, gi])), (f, gi, fd, Gbo[f, gi])
