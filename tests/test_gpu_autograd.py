"""torch.autograd front end: gradients of a drag functional through
ghost_fill -> forces, and of surface outputs through surface(), checked
bitwise against the direct C-ABI adjoint chain, against the oracle's
transposes (1e-12 of the oracle's per-entry adjoint scale) and by central
differences through the autograd forward."""
import numpy as np
import pytest

import oracle
import synth
from synth import HGC, DIRICHLET, NEUMANN
from tolerances import check, force_gradient

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


def foot_bc(inst, op, flds, kinds):
    g, d, c = inst.grid, inst.grid.dim, op.ghost_cell
    idx = [c % g.n[0], (c // g.n[0]) % g.n[1]] + ([c // (g.n[0] * g.n[1])] if d == 3 else [])
    S = np.stack([g.lo[i] + (idx[i] + 0.5) * g.h[i] for i in range(d)]) + op.delta
    return np.stack([synth.bc_values(f, S, op.normal, k) for f, k in zip(flds, kinds)])


def test_drag_gradient_through_autograd(gcr):
    from paper_2609_10165_amd import autograd as ga
    inst = synth.shstar384(seed=5, n=48, nt=8, nph=16)
    d = inst.grid.dim
    flds = inst.fields
    kinds = [f.bc for f in flds]
    nf = len(flds)
    op = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    gp = gcr.Plan(inst.grid, inst.shape, HGC)
    b0 = foot_bc(inst, op, flds, kinds)
    phi0 = np.stack([synth.sample(f, inst.grid) for f in flds])
    q = inst.queries
    xq, nq_, wq = dev(q.x), dev(q.n), dev(q.w)
    mu = 0.7

    fields = [dev(x).requires_grad_() for x in phi0]
    bcs = [dev(x).requires_grad_() for x in b0]
    out = ga.ghost_fill(gp, fields, kinds, bcs)
    F = ga.forces(gp, xq, nq_, wq, out[d], out[:d], mu)
    F[0].backward()
    torch.cuda.synchronize()
    # inputs untouched by the out-of-place fill
    assert np.array_equal(host(fields[0]), phi0[0])
    G = np.stack([host(f.grad) for f in fields])
    Gb = np.stack([host(b.grad) for b in bcs])

    # the direct C-ABI chain gives the same bits
    lam = [torch.zeros(op.n_cells, dtype=torch.float64, device="cuda") for _ in range(nf)]
    gp.forces_adjoint(xq, nq_, wq, mu, dev(np.eye(d)[0]), lam[d], lam[:d])
    lam_bc = [torch.empty(op.n_ghost, dtype=torch.float64, device="cuda") for _ in range(nf)]
    gp.fill_adjoint(lam, kinds, lam_bc)
    torch.cuda.synchronize()
    assert np.array_equal(G, np.stack([host(x) for x in lam]))
    assert np.array_equal(Gb, np.stack([host(x) for x in lam_bc]))

    # the oracle's transposes, per-entry scales
    Go, Gbo, So, Sbo = force_gradient(op, q, mu, np.eye(d)[0], kinds, d, list(range(d)))
    check(G, Go, So, "gradient vs oracle")
    check(Gb, Gbo, Sbo, "bc gradient vs oracle")

    # central differences (J is affine: rounding only) on 8 + 8 entries
    def J(phi, b):
        with torch.no_grad():
            o = ga.ghost_fill(gp, [dev(x) for x in phi], kinds, [dev(x) for x in b])
            return float(ga.forces(gp, xq, nq_, wq, o[d], o[:d], mu)[0])

    rng = np.random.default_rng(11)
    sup = np.argwhere(G != 0)
    eps = 1e-6
    for f, c in sup[rng.choice(len(sup), 8, replace=False)]:
        a, m = phi0.copy(), phi0.copy()
        a[f, c] += eps
        m[f, c] -= eps
        fd = (J(a, b0) - J(m, b0)) / (2 * eps)
        assert abs(fd - G[f, c]) <= 1e-7 * max(1.0, abs(G[f, c])), (f, c, fd, G[f, c])
    for k in rng.choice(nf * op.n_ghost, 8, replace=False):
        f, gi = divmod(int(k), op.n_ghost)
        a, m = b0.copy(), b0.copy()
        a[f, gi] += eps
        m[f, gi] -= eps
        fd = (J(phi0, a) - J(phi0, m)) / (2 * eps)
        assert abs(fd - Gb[f, gi]) <= 1e-7 * max(1.0, abs(Gb[f, gi])), (f, gi, fd, Gb[f, gi])


def test_surface_gradient_through_autograd(gcr):
    from paper_2609_10165_amd import autograd as ga
    inst = synth.circle128(seed=9)
    op = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    gp = gcr.Plan(inst.grid, inst.shape, HGC)
    rng = np.random.default_rng(2)
    nq = inst.queries.x.shape[1]
    phi = [dev(x).requires_grad_() for x in rng.normal(size=(2, op.n_cells))]
    gval = rng.normal(size=(2, nq))
    ggrad = rng.normal(size=(2, 2, nq))
    xq = dev(inst.queries.x)
    val, grad = ga.surface(gp, xq, phi)
    ((val * dev(gval)).sum() + (grad * dev(ggrad)).sum()).backward()
    torch.cuda.synchronize()
    got = np.stack([host(p.grad) for p in phi])
    want = op.surface_query_adjoint(inst.queries.x, gval, ggrad, np.zeros((2, op.n_cells)))
    scale = op.surface_query_adjoint_scale(inst.queries.x, np.abs(gval), np.abs(ggrad),
                                           np.zeros((2, op.n_cells)))
    check(got, want, scale, "surface gradient vs oracle")


def test_fill_rejects_non_f64(gcr):
    from paper_2609_10165_amd import autograd as ga
    inst = synth.circle128(seed=1)
    gp = gcr.Plan(inst.grid, inst.shape, HGC)
    f = torch.zeros(gp.n_cells, dtype=torch.float32, device="cuda")
    b = torch.zeros(gp.n_ghost, dtype=torch.float64, device="cuda")
    with pytest.raises(TypeError):
        ga.ghost_fill(gp, [f], [DIRICHLET], [b])
