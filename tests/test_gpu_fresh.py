"""GPU parity of gcr_plan_fresh_cells: the cells a moved body exposes (Sec.
7.1), bit-exact against the oracle's list and counts."""
import numpy as np
import pytest

import oracle
import synth
from synth import CGC, HGC, LAYER2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gcr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_10165_amd as g
    g.lib()
    return g


def moved(shape, v):
    return synth.Shape(shape.kind, tuple(c + d for c, d in zip(shape.center, v)), shape.r0)


def check(gcr, inst, flag, v, cap=None):
    a_o = oracle.OraclePlan(inst.grid, inst.shape, flag)
    b_o = oracle.OraclePlan(inst.grid, moved(inst.shape, v), flag)
    want, unc = a_o.fresh_cells(b_o)
    a = gcr.Plan(inst.grid, inst.shape, flag)
    b = gcr.Plan(inst.grid, moved(inst.shape, v), flag)
    lst, counts = a.fresh_cells(b, cap=cap)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    assert c[0] == len(want) and c[1] == unc, (c, len(want), unc)
    k = min(len(want), lst.numel())
    assert np.array_equal(lst[:k].cpu().numpy().astype(np.int64), want[:k])
    return len(want), unc


@pytest.mark.parametrize("scheme", [CGC, HGC])
@pytest.mark.parametrize("layer2", [False, True])
def test_fresh_cells_circle(gcr, scheme, layer2):
    inst = synth.circle128(seed=3)
    h = inst.grid.h[0]
    for v in ((0.7 * h, 0.2 * h, 0.0), (-1.3 * h, 0.9 * h, 0.0), (0.05 * h, -1.9 * h, 0.0)):
        nf, unc = check(gcr, inst, scheme | (LAYER2 if layer2 else 0), v)
        assert nf > 0
        if layer2 and np.hypot(v[0], v[1]) < 1.5 * h:
            assert unc == 0


def test_fresh_cells_sphere256_full_size(gcr):
    inst = synth.sphere256(seed=0)
    h = inst.grid.h[0]
    nf, unc = check(gcr, inst, HGC | LAYER2, (0.6 * h, -0.5 * h, 0.8 * h))
    assert nf > 1000 and unc == 0
    nf, unc = check(gcr, inst, CGC, (1.2 * h, 0.3 * h, -0.4 * h))
    assert unc > 0


def test_fresh_cells_stretched_and_truncated(gcr):
    inst = synth.circle_stretched(seed=1)
    check(gcr, inst, HGC | LAYER2, (0.01, -0.02, 0.0))
    nf, _ = check(gcr, inst, CGC, (0.03, 0.01, 0.0), cap=7)   # list cut at 7, counts whole
    assert nf > 7


def test_fresh_cells_refuses_other_grids(gcr):
    a_inst = synth.circle128(seed=0)
    big = synth.Grid(2, (130, 128, 1), a_inst.grid.lo, a_inst.grid.h)
    a = gcr.Plan(a_inst.grid, a_inst.shape, HGC)
    b = gcr.Plan(big, a_inst.shape, HGC)
    with pytest.raises(gcr.GcrError):
        a.fresh_cells(b)
