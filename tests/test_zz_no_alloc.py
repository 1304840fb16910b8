"""gcr_forces_noalloc (the allocation-free variant of gcr_forces, partial sums
in a static device array of the library) against gcr_forces, through the
C-ABI: the same force bit for bit, on two calls in a row, the second with
fewer points, in 3D and 2D; a point count beyond the array's capacity is
refused before any launch."""
import ctypes

import numpy as np
import pytest

import synth
from synth import HGC

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gcr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_10165_amd as g
    g.lib()
    return g


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _call(gcr, name, plan, xq, nr, wq, p, u, mu, F):
    L = gcr.lib()
    ua = (ctypes.c_void_p * len(u))(*[t.data_ptr() for t in u])
    return getattr(L, name)(plan._h, xq.shape[1], _ptr(xq), _ptr(nr), _ptr(wq), _ptr(p), ua,
                            ctypes.c_double(mu), _ptr(F), None)


@pytest.mark.parametrize("which", ["sphere", "circle"])
def test_forces_noalloc_matches_forces(gcr, which):
    inst = synth.sphere256(seed=1, n=96) if which == "sphere" else synth.circle128(seed=2)
    d = inst.grid.dim
    plan = gcr.Plan(inst.grid, inst.shape, HGC)
    rng = np.random.default_rng(4)
    fields = [torch.as_tensor(rng.standard_normal(inst.grid.n_cells), device="cuda")
              for _ in range(d + 1)]
    q = inst.queries
    nq = q.x.shape[1]
    for count in (nq, nq // 3):           # the second call with fewer points
        xq, nr, wq = dev(q.x[:, :count]), dev(q.n[:, :count]), dev(q.w[:count])
        F_ref = torch.full((d,), np.nan, dtype=torch.float64, device="cuda")
        F_new = torch.full((d,), np.nan, dtype=torch.float64, device="cuda")
        assert _call(gcr, "gcr_forces", plan, xq, nr, wq, fields[d], fields[:d], 0.6, F_ref) == 0
        assert _call(gcr, "gcr_forces_noalloc", plan, xq, nr, wq, fields[d], fields[:d], 0.6,
                     F_new) == 0
        torch.cuda.synchronize()
        assert torch.isfinite(F_ref).all()
        assert torch.equal(F_new.view(torch.int64), F_ref.view(torch.int64)), (count, F_new, F_ref)


def test_forces_noalloc_refuses_beyond_capacity(gcr):
    inst = synth.sphere256(seed=1, n=64)
    plan = gcr.Plan(inst.grid, inst.shape, HGC)
    small = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
    w = torch.zeros(4, dtype=torch.float64, device="cuda")
    f = [torch.zeros(inst.grid.n_cells, dtype=torch.float64, device="cuda") for _ in range(4)]
    F = torch.zeros(3, dtype=torch.float64, device="cuda")
    L = gcr.lib()
    ua = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in f[:3]])
    # 3D: four points per block, 65,536 blocks; refused before anything is read
    st = L.gcr_forces_noalloc(plan._h, 4 * 65536 + 1, _ptr(small), _ptr(small), _ptr(w),
                              _ptr(f[3]), ua, ctypes.c_double(1.0), _ptr(F), None)
    assert st == 8    # GCR_E_UNSUPPORTED
    st = L.gcr_forces_noalloc(plan._h, -1, _ptr(small), _ptr(small), _ptr(w), _ptr(f[3]), ua,
                              ctypes.c_double(1.0), _ptr(F), None)
    assert st == 1    # GCR_E_ARG
