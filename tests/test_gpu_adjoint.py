"""GPU parity of the adjoints (fill, surface, forces) through the C-ABI.

Checks: element-wise against the oracle's explicit transposes at 1e-12 of
the oracle's per-entry adjoint scale (the reverse sweeps on magnitudes,
coupled units by |A^-T|), the dot-product identity <A x, y> = <x, A^T y>
with the GPU's own forward, bitwise determinism, and central differences of
the drag functional (affine, so differences carry rounding only).
"""
import numpy as np
import pytest

import oracle
import synth
from synth import HGC, CGC, DIRICHLET, NEUMANN
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


@pytest.mark.parametrize("which", ["circle128", "sphere64", "star_cycle"])
def test_fill_adjoint_matches_oracle(gcr, which):
    if which == "circle128":
        inst, scheme = synth.circle128(seed=4), HGC
    elif which == "sphere64":
        inst, scheme = synth.sphere256(seed=2, n=64), HGC
    else:
        inst, scheme = synth.stars64(seed=0, ninst=1, nmin=96, nmax=160)[0], CGC
    op = oracle.OraclePlan(inst.grid, inst.shape, scheme)
    gp = gcr.Plan(inst.grid, inst.shape, scheme)
    rng = np.random.default_rng(3)
    kinds = [DIRICHLET, NEUMANN]
    lam0 = rng.normal(size=(2, op.n_cells))
    want, want_bc = op.fill_adjoint(lam0.copy(), kinds)
    scale, scale_bc = op.fill_adjoint_scale(np.abs(lam0), kinds)
    if which == "star_cycle":
        assert op.n_units_coupled >= 1
    lam = [dev(l) for l in lam0]
    lam_bc = [torch.empty(op.n_ghost, dtype=torch.float64, device="cuda") for _ in kinds]
    gp.fill_adjoint(lam, kinds, lam_bc)
    torch.cuda.synchronize()
    got = np.stack([host(l) for l in lam])
    got_bc = np.stack([host(l) for l in lam_bc])
    check(got, want, scale, "lam")
    check(got_bc, want_bc, scale_bc, "lam_bc")
    assert np.all(got[:, op.ghost_cell] == 0)
    # determinism
    lam2 = [dev(l) for l in lam0]
    lam_bc2 = [torch.empty_like(x) for x in lam_bc]
    gp.fill_adjoint(lam2, kinds, lam_bc2)
    torch.cuda.synchronize()
    assert np.array_equal(np.stack([host(l) for l in lam2]), got)
    assert np.array_equal(np.stack([host(l) for l in lam_bc2]), got_bc)


@pytest.mark.parametrize("which", ["circle128", "sphere64"])
def test_surface_adjoint_matches_oracle_and_dot_product(gcr, which):
    inst = synth.circle128(seed=5) if which == "circle128" else synth.sphere256(seed=3, n=64)
    op = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    gp = gcr.Plan(inst.grid, inst.shape, HGC)
    rng = np.random.default_rng(8)
    d = op.dim
    nq = inst.queries.x.shape[1]
    gval = rng.normal(size=(2, nq))
    ggrad = rng.normal(size=(2, d, nq))
    want = op.surface_query_adjoint(inst.queries.x, gval, ggrad, np.zeros((2, op.n_cells)))
    xq = dev(inst.queries.x)
    lam = [torch.zeros(op.n_cells, dtype=torch.float64, device="cuda") for _ in range(2)]
    gp.surface_adjoint(xq, dev(gval), dev(ggrad), lam)
    torch.cuda.synchronize()
    got = np.stack([host(l) for l in lam])
    scale = op.surface_query_adjoint_scale(inst.queries.x, np.abs(gval), np.abs(ggrad),
                                           np.zeros((2, op.n_cells)))
    check(got, want, scale, "surface adjoint")
    # <S phi, g> == <phi, S^T g> with the GPU forward
    phi = rng.normal(size=(2, op.n_cells))
    v, gr, _ = gp.surface(xq, [dev(x) for x in phi])
    lhs = (host(v) * gval).sum() + (host(gr) * ggrad).sum()
    rhs = (got * phi).sum()
    assert abs(lhs - rhs) <= 1e-10 * (np.abs(got * phi).sum() + abs(lhs))


@pytest.mark.parametrize("which", ["circle128", "shstar_small"])
def test_drag_gradient_fd_and_oracle(gcr, which):
    """J = drag F_x; gradient w.r.t. interior field values and boundary data
    from gcr_forces_adjoint + gcr_fill_adjoint; central differences (step
    1e-6) on 32 seed-drawn entries, and the oracle's gradient."""
    if which == "circle128":
        inst = synth.circle128(seed=6)
        flds = [synth.Field("u", *synth.workloads._trig2d(), DIRICHLET),
                synth.Field("v", lambda x, y: np.cos(x + 2 * y),
                            lambda x, y: [-np.sin(x + 2 * y), -2 * np.sin(x + 2 * y)], DIRICHLET),
                synth.Field("p", lambda x, y: np.exp(0.5 * x) * np.sin(y),
                            lambda x, y: [0.5 * np.exp(0.5 * x) * np.sin(y),
                                          np.exp(0.5 * x) * np.cos(y)], NEUMANN)]
    else:
        inst = synth.shstar384(seed=3, n=64, nt=8, nph=16)
        flds = inst.fields
    d = inst.grid.dim
    kinds = [f.bc for f in flds]
    op = oracle.OraclePlan(inst.grid, inst.shape, HGC)
    gp = gcr.Plan(inst.grid, inst.shape, HGC)
    c = op.ghost_cell
    g = inst.grid
    idx = [c % g.n[0], (c // g.n[0]) % g.n[1]] + ([c // (g.n[0] * g.n[1])] if d == 3 else [])
    S = np.stack([g.lo[i] + (idx[i] + 0.5) * g.h[i] for i in range(d)]) + op.delta
    b0 = np.stack([synth.bc_values(f, S, op.normal, k) for f, k in zip(flds, kinds)])
    phi0 = np.stack([synth.sample(f, g) for f in flds])
    q = inst.queries
    xq, nq_, wq = dev(q.x), dev(q.n), dev(q.w)
    mu = 0.8
    nf = d + 1

    def J(phi, b):
        fs = [dev(x) for x in phi]
        gp.fill(fs, kinds, [dev(x) for x in b])
        F = gp.forces(xq, nq_, wq, fs[d], fs[:d], mu)
        return float(F[0])

    # adjoint: dJ/d(filled) via forces adjoint, then the fill adjoint
    gF = dev(np.eye(d)[0])
    lam = [torch.zeros(op.n_cells, dtype=torch.float64, device="cuda") for _ in range(nf)]
    gp.forces_adjoint(xq, nq_, wq, mu, gF, lam[d], lam[:d])
    lam_bc = [torch.empty(op.n_ghost, dtype=torch.float64, device="cuda") for _ in range(nf)]
    gp.fill_adjoint(lam, kinds, lam_bc)
    torch.cuda.synchronize()
    G = np.stack([host(l) for l in lam])
    Gb = np.stack([host(l) for l in lam_bc])
    # oracle gradient: same chain with the oracle's transposes, per-entry scales
    Go, Gbo, So, Sbo = force_gradient(op, q, mu, np.eye(d)[0], kinds, d, list(range(d)))
    check(G, Go, So, "gradient vs oracle")
    check(Gb, Gbo, Sbo, "bc gradient vs oracle")
    # central differences on 16 interior and 16 boundary entries
    rng = np.random.default_rng(32)
    sup = np.argwhere(G != 0)
    eps = 1e-6
    for f, cidx in sup[rng.choice(len(sup), 16, replace=False)]:
        a, m = phi0.copy(), phi0.copy()
        a[f, cidx] += eps
        m[f, cidx] -= eps
        fd = (J(a, b0) - J(m, b0)) / (2 * eps)
        assert abs(fd - G[f, cidx]) <= 1e-7 * max(1.0, abs(G[f, cidx])), (f, cidx, fd, G[f, cidx])
    for k in rng.choice(nf * op.n_ghost, 16, replace=False):
        f, gi = divmod(int(k), op.n_ghost)
        a, m = b0.copy(), b0.copy()
        a[f, gi] += eps
        m[f, gi] -= eps
        fd = (J(phi0, a) - J(phi0, m)) / (2 * eps)
        assert abs(fd - Gb[f, gi]) <= 1e-7 * max(1.0, abs(Gb[f, gi])), (f, gi, fd, Gb[f, gi])
