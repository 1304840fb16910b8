"""Benchmark of the ghost-cell hot path on one MI355X.

Headline (`value`): the batched workload end to end.  64 2D star-shaped
bodies, r(t) = r0 (1 + sum_{k=2..5} a_k cos(k t + phi_k)), on square grids
of n ~ U{128..2048} cells per side (107M cells, 104,936 HGC ghosts), three
FP64 fields with mixed Dirichlet/Neumann data per ghost.  One step is the
whole path for all 64 instances:
  plans (classification, tags, geometry, dependency levels, canonical order)
  -> foot points and the caller's boundary data there (kinds and values of
     the three fields, torch)
  -> one persistent launch: level-by-level fill of the three fields, their
     values and gradients at each instance's 256 surface points and the
     pressure + viscous force on each body.
Metric: ghost cells per second (ghosts of the 64 plans per step / step
time).  The timed steps run pipelined: host threads build batches on
streams of their own while another enqueues each built batch's boundary
data and forward on a forward stream (every step still builds its own
batch and runs the whole path).  The same steps one after another on one
stream (serial_step), with a 1 GiB write between steps (cold_llc), and one
plan at a time with per-level fill launches (plain_step) are timed beside it.

`roofline`: the step's longest kernel among the batched forward, the
classification store pass and the layering, timed by HIP events the library
records around it on the stream it runs on, against its algorithmic bytes.

Side keys (same GPU, never `value`):
  sphere256  the 256^3 sphere with CGC, CGC_ES and HGC as one batch, four
             fields, 2048 surface points, pipelined the same way;
  fwd_bwd    384^3 grid, spherical-harmonic star, u, v, w, p, HGC: fill +
             drag forward, then the reverse-level adjoint, against the plain
             per-level forward; its own roofline and CPU baseline;
  latency    single calls of the 128^2 circle (three schemes) and the
             4096^2 airfoil (plan + fill + surface values + force);
  hbm_copy   the box's device-to-device copy bandwidth;
  static_forward, layer2, moving, large (as documented in each function).

Prints one JSON line.  Only N=1 is supported (one GPU).
"""
from __future__ import annotations

import argparse
import collections
import gc
import hashlib
import json
import os
import queue
import subprocess
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
DIRICHLET, NEUMANN, MIXED = 0, 1, 2
HGC = 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--build-threads", type=int, default=2, choices=(1, 2, 3),
                    help="host threads building batches in the timed steps (each on "
                         "a stream of its own; the forwards are enqueued by another)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="oracle time budget of each CPU baseline sample")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side measurements")
    ap.add_argument("--only-headline", action="store_true",
                    help="headline, roofline and nothing else (for profiling runs)")
    ap.add_argument("--extra-reps", type=int, default=10)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first "
                         "(reference kernel for byte counters)")
    return ap.parse_args()


def _dev(torch, a, dtype=None):
    """Contiguous device copy of a host array (inputs resident in HBM)."""
    a = np.ascontiguousarray(a)
    return torch.tensor(a, dtype=dtype, device="cuda")


def kernel_traffic(name, workload):
    """HBM bytes per launch of kernel `name` on `workload` from the committed
    byte-counter summary, or None when it is absent or the kernel's sources
    changed since."""
    key = name.split("<")[0].replace(" + ", "+")
    path = os.path.join(ROOT, "profiles", f"{key}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for rel in rec.get("sources", []):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# boundary data on the caller's side (torch), evaluated at the foot points
# ---------------------------------------------------------------------------

def bc_sphere_fields(S, n, out=None):
    """Boundary data of the u, v, w, p fields at the foot points: values of
    u = sin z + cos y, v = sin x + cos z, w = sin y + cos x and the normal
    derivative of p = cos x cos y cos z, written dp/dn = -(c_x c_y c_z)
    sum_i tan(S_i) n_i (cos > 0.5 on the domain) to keep the caller's
    launches few (into `out` [4][n] if given)."""
    import torch
    s, c = torch.sin(S), torch.cos(S)
    if out is None:
        out = torch.empty((4, S.shape[1]), dtype=torch.float64, device=S.device)
    # rows (sin z, sin x, sin y) + (cos y, cos z, cos x): rolls, no index lists
    # (an index list is a host-to-device copy that waits for the stream)
    torch.add(torch.roll(s, 1, 0), torch.roll(c, -1, 0), out=out[:3])
    t = s / c
    t.mul_(n)
    torch.sum(t, dim=0, out=out[3])
    out[3].mul_(c.prod(dim=0)).neg_()
    return out


def bc_star_fields(S, n, cen, beta, out, kinds):
    """Mixed boundary data of the star workload's three fields (u = sin 2x
    cos 3y, v = cos(x + 2y), p = exp(x/2) sin y) at the foot points S with
    normals n: field f is Dirichlet where cos(theta_S - beta_f) >= 0 (theta_S
    the angle of S about its body's centre, cen [2][ng]), else Neumann; out
    [3][ng] the values, kinds [3][ng] uint8 the kinds.  The three fields go
    as [3][ng] stacks, so each step is one launch for all of them."""
    import torch
    x, y = S[0], S[1]
    th = torch.atan2(y - cen[1], x - cen[0])
    # arguments 2x, 3y, x + 2y, y: their sines and cosines in one launch each
    arg = torch.stack((x, y, x, y))
    arg[0].mul_(2.0)
    arg[1].mul_(3.0)
    arg[2].add_(y, alpha=2.0)
    sn, cs = torch.sin(arg), torch.cos(arg)
    e = torch.exp(0.5 * x)
    n0, n1 = n[0], n[1]
    vals = torch.stack((sn[0] * cs[1], cs[2], e * sn[3]))
    dns = torch.stack((2 * cs[0] * cs[1] * n0 - 3 * sn[0] * sn[1] * n1,
                       -sn[2] * (n0 + 2 * n1),
                       e * (0.5 * sn[3] * n0 + cs[3] * n1)))
    dirichlet = torch.cos(th.unsqueeze(0) - beta) >= 0
    torch.logical_not(dirichlet, out=kinds)
    torch.where(dirichlet, vals, dns, out=out)


# ---------------------------------------------------------------------------
# a batched step: build, foot points, boundary data, one forward launch
# ---------------------------------------------------------------------------

class BatchStep:
    """One workload of the batched path, with the buffers and pointer
    tables its steps reuse (two buffer sets used in turn)."""

    def __init__(self, gcr, torch, name, grids, shapes, schemes, fields, kinds, mixed, queries,
                 p_field, u_first, bc_fn):
        self.gcr, self.torch, self.name = gcr, torch, name
        self.grids, self.shapes, self.schemes = grids, shapes, schemes
        self.ninst = len(grids)
        self.dim = grids[0].dim
        self.fields = fields                 # [ninst * nf] device tensors
        self.nf = len(kinds)
        self.kinds = kinds
        self.mixed = mixed
        dev = "cuda"
        self.xq = [_dev(torch, q.x) for q in queries]
        self.nr = [_dev(torch, q.n) for q in queries]
        self.wq = [_dev(torch, q.w) for q in queries]
        self.nq = [q.x.shape[1] for q in queries]
        self.F = torch.zeros((self.ninst, 3), dtype=torch.float64, device=dev)
        self.sval = [torch.empty(n, dtype=torch.float64, device=dev)
                     for n in self.nq for _ in range(self.nf)]
        self.sgrad = [torch.empty((self.dim, n), dtype=torch.float64, device=dev)
                      for n in self.nq for _ in range(self.nf)]
        self.p_field, self.u_first = p_field, u_first
        self.spec = gcr.BatchSpec(grids, shapes, schemes)   # packed once
        self.bc_fn = bc_fn                   # (pk) -> writes pk["bc"] (and pk["bt"])
        self.packs = [{}, {}]
        self.bc_graph_ok = None
        self.ghosts = 0
        self.band_segments = 0
        self.shape = (0, 0)   # the forward's launch shape (threads, grid)

    def batch(self, stream=None):
        return self.gcr.Batch(spec=self.spec, stream=stream)

    def pack(self, k, counts):
        pk = self.packs[k]
        if pk.get("counts") == counts:
            return pk
        torch, dev = self.torch, "cuda"
        ng = sum(counts)
        bc = torch.empty((self.nf, ng), dtype=torch.float64, device=dev)
        bt = torch.empty((self.nf, ng), dtype=torch.uint8, device=dev) if self.mixed else None
        bcv, bct, off = [], [], 0
        for c in counts:
            bcv += [bc[f, off:off + c] for f in range(self.nf)]
            if bt is not None:
                bct += [bt[f, off:off + c] for f in range(self.nf)]
            off += c
        pk.clear()
        pk.update(counts=counts, bc=bc, bt=bt,
                  S=torch.empty((self.dim, ng), dtype=torch.float64, device=dev),
                  n=torch.empty((self.dim, ng), dtype=torch.float64, device=dev))
        pk["args"] = self.gcr.ForwardArgs(
            self.nf, self.fields, [MIXED] * self.nf if self.mixed else self.kinds, bcv,
            bc_type=bct if self.mixed else None, nq=self.nq, xq=self.xq, nrm=self.nr, wq=self.wq,
            p_field=self.p_field, u_first=self.u_first, mu=1.0, F=self.F, sval=self.sval,
            sgrad=self.sgrad)
        self.bc_fn(pk, init=True)
        return pk

    def boundary_data(self, pk):
        if pk.get("graph") is not None:
            pk["graph"].replay()
        else:
            self.bc_fn(pk)

    def capture(self):
        """The boundary-data evaluation of each buffer set captured as one HIP
        graph, used only if its replays reproduce the eager result bitwise
        (several inputs, eager work and synchronisations between replays)."""
        torch = self.torch
        ok = True
        for pk in self.packs:
            if "S" not in pk:
                ok = False
                continue
            pk["graph"] = None
            S0 = pk["S"].clone()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                self.bc_fn(pk)          # warm-up before capture
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            try:
                with torch.cuda.graph(g):
                    self.bc_fn(pk)
                torch.cuda.synchronize()
            except RuntimeError:
                ok = False
                continue
            good = True
            for r in range(4):
                pk["S"].copy_(S0 * (1.0 + 1e-3 * r))
                self.bc_fn(pk)
                torch.cuda.synchronize()
                want = (pk["bc"].clone(), None if pk["bt"] is None else pk["bt"].clone())
                pk["bc"].fill_(float("nan"))
                g.replay()
                torch.cuda.synchronize()
                if not torch.equal(pk["bc"], want[0]) or (
                        want[1] is not None and not torch.equal(pk["bt"], want[1])):
                    good = False
                    break
            pk["S"].copy_(S0)
            self.bc_fn(pk)
            torch.cuda.synchronize()
            if good:
                pk["graph"] = g
            else:
                ok = False
        if not ok:
            for pk in self.packs:
                pk["graph"] = None
        self.bc_graph_ok = ok
        return ok

    def step(self, k=0, record=None):
        """One step on the current stream."""
        B = self.batch()
        if record is not None:
            record.append(self.gcr.last_build_times())
        pk = self.pack(k, B.counts())
        B.foot_points(out=(pk["S"], pk["n"]))
        self.boundary_data(pk)
        B.forward(args=pk["args"])
        self.shape = B.shape()
        self.ghosts = sum(pk["counts"])
        return B

    def run_threads(self, nsteps, s_fwd, s_builds, nbuild):
        """Pipelined steps: `nbuild` threads build batches (each on a build
        stream of its own); another takes each built batch and enqueues its
        foot points, boundary data and forward on the forward stream.  A
        batch is handed over once built (an event after the build, waited on
        by the forward stream); everything after that is in order on the
        forward stream, and a batch is dropped only after its forward's
        event, so no pooled memory is reused while still read."""
        torch = self.torch
        q = queue.Queue(maxsize=2)
        tickets = queue.Queue()
        for _ in range(nsteps):
            tickets.put(True)
        for _ in range(nbuild):
            tickets.put(None)
        err = []

        def forwarder():
            held = collections.deque()
            t = 0
            try:
                while True:
                    item = q.get()
                    if item is None:
                        break
                    B, built = item
                    with torch.cuda.stream(s_fwd):
                        s_fwd.wait_event(built)
                        pk = self.pack(t & 1, B.counts())
                        B.foot_points(stream=s_fwd, out=(pk["S"], pk["n"]))
                        self.boundary_data(pk)
                        B.forward(args=pk["args"], stream=s_fwd)
                        done = torch.cuda.Event()
                        done.record(s_fwd)
                    held.append((B, done))
                    if len(held) > 2:
                        _, e0 = held.popleft()
                        e0.synchronize()
                    t += 1
                for _, e in held:
                    e.synchronize()
            except Exception as e:   # reported by the main thread
                err.append(e)
                while q.get() is not None:   # keep the builders from blocking
                    pass

        def builder(st):
            try:
                while tickets.get() is not None:
                    with torch.cuda.stream(st):
                        B = self.batch(stream=st)
                        built = torch.cuda.Event()
                        built.record(st)
                    q.put((B, built))
                    del B
            except Exception as e:
                err.append(e)
                while tickets.get() is not None:   # let the other builders finish
                    pass

        fw = threading.Thread(target=forwarder)
        fw.start()
        bs = [threading.Thread(target=builder, args=(st,)) for st in s_builds[:nbuild]]
        try:
            for b in bs:
                b.start()
        finally:
            for b in bs:
                b.join()
            q.put(None)
            fw.join()
        if err:
            raise err[0]

    def grow_pools(self, s_build, count=12):
        """As many batches built and forwarded at once as the deepest pipeline
        holds, then released: the library's device and pinned pools then
        hold enough blocks that no timed step calls hipMalloc."""
        torch = self.torch
        with torch.cuda.stream(s_build):
            held = [self.batch(stream=s_build) for _ in range(count)]
            pk = self.pack(0, held[0].counts())
            for B in held:
                B.forward(args=pk["args"], stream=s_build)
        torch.cuda.synchronize()
        del held


def forward_bytes(dim, nf, ng, npts):
    """Algorithmic bytes of one batched forward launch: per ghost and field,
    the 2^d - 1 stencil values and the boundary datum read and the result
    written (8 B each), and its kind (1 B, mixed data only counted when
    given); per ghost, its cell, code, foot-point offset and normal once
    (4 + 4 + 16d B); per surface point, position, normal, weight and anchor
    (16d + 12 B), and per field the 2^d corner values read and the value
    and gradient written (8 (2^d + 1 + d) B)."""
    per_gf = 8 * ((1 << dim) - 1) + 8 + 8
    return ng * (nf * per_gf + 8 + 16 * dim) + npts * (16 * dim + 12 + nf * 8 * ((1 << dim) + 1 + dim))


def levels_bytes(dim, ng):
    """Algorithmic bytes of the layering: per ghost its 2^d - 1 dependency
    ids read, as many reverse edges read and its reverse-edge offset, and
    its level and canonical position written (4 B each)."""
    return ng * (8 * ((1 << dim) - 1) + 12)


def timed_steps(torch, fn, reps, between=None):
    """Median, p10 and p90 ms of fn() over reps calls (HIP events on the
    current stream, a synchronisation before each); between() runs outside
    the timed region."""
    ts = []
    for _ in range(reps):
        if between is not None:
            between()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts)), float(np.percentile(ts, 10)), float(np.percentile(ts, 90))


def measure_batched(gcr, torch, W, args, s_fwd, s_builds, extra=True):
    """Serial steps, then the pipelined steps (the headline form), then stage
    events, on workload W.  Returns a dict of figures."""
    stream = torch.cuda.current_stream()
    gcr.set_profiling(gcr.PROFILE_FORWARD)
    for _ in range(args.warmup):
        W.step()
    torch.cuda.synchronize()
    gc.collect()
    gcr.forward_times()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(args.steps):
        W.step()
    t1.record(stream)
    torch.cuda.synchronize()
    ms_serial = t0.elapsed_time(t1) / args.steps
    # both buffer sets exist after two pipelined steps; capture the boundary
    # data then
    W.run_threads(4, s_fwd, s_builds, 1)
    torch.cuda.synchronize()
    W.capture()
    nbuild = args.build_threads
    W.grow_pools(s_builds[0])
    # pipelined warm-up steps, for at least 0.3 s: the first process on a
    # fresh machine runs its host code slowly at first (pages of the
    # libraries still coming in), which a few steps do not cover
    w0 = time.perf_counter()
    W.run_threads(4 + 2 * nbuild, s_fwd, s_builds, nbuild)
    torch.cuda.synchronize()
    while time.perf_counter() - w0 < 0.3:
        W.run_threads(16, s_fwd, s_builds, nbuild)
        torch.cuda.synchronize()
    # the warm-ups have grown the pools to the pipeline's depth; objects made
    # so far are frozen out of the cycle collector's scans (a full scan of
    # torch's objects costs milliseconds), as a long-running solver would
    gc.collect()
    gc.freeze()
    gcr.forward_times()   # drop the events of the runs before the timed one
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    W.run_threads(args.steps, s_fwd, s_builds, nbuild)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = wall * 1e3 / args.steps
    fwd_times = gcr.forward_times()   # around the forward kernels in the timed steps
    # build-stage times: as many serial steps again with stage events on
    gcr.set_profiling(gcr.PROFILE_BUILD)
    rec = []
    for _ in range(max(5, args.steps // 2)):
        W.step(record=rec)
    torch.cuda.synchronize()
    gcr.set_profiling(False)
    stage_ms = {k: float(np.mean([r[k] for r in rec])) for k in rec[0]}
    W.band_segments = W.batch().plans[0].stats()["n_band_segments"]
    out = {"ms_per_step": ms_step, "ms_serial": ms_serial, "wall_s": wall,
           "ghosts": W.ghosts, "fwd_ms": fwd_times["forward"], "anchor_ms": fwd_times["anchor"],
           "stage_ms": stage_ms, "band_segments": W.band_segments, "nbuild": nbuild}
    if extra:
        # the same steps one after another with the last-level cache flushed
        # by a 1 GiB write between steps (outside the timed region)
        flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        med, p10, p90 = timed_steps(torch, W.step, max(5, args.steps // 2),
                                    between=lambda: flush.fill_(1.0))
        hot = timed_steps(torch, W.step, max(5, args.steps // 2))
        del flush
        out["cold_llc"] = {"ms_median": med, "ms_p10": p10, "ms_p90": p90,
                           "hot_ms_median": hot[0], "hot_ms_p10": hot[1], "hot_ms_p90": hot[2]}
    return out


def roofline_of(W, m, cells):
    """The step's longest kernel among the batched forward (library events
    around the launch in the timed steps), the classification (the span
    pass, which stores settled spans, and the store pass over the chunks it
    leaves: 1 byte per cell written) and the layering (stage events around
    each launch), against its algorithmic bytes."""
    d = W.dim
    npts = sum(W.nq)
    # the forward's kernel: the split sweep for a negative grid, else the
    # per-item kernel
    fwd = f"k_batch_split<{d}>" if W.shape[1] < 0 else f"k_batch_forward<{d}>"
    cands = {
        fwd: (m["fwd_ms"], forward_bytes(d, W.nf, m["ghosts"], npts)),
        "k_spans + k_classify": (m["stage_ms"]["classify_prepass"] + m["stage_ms"]["classify_store"],
                                 cells),
        "k_levels": (m["stage_ms"]["levels_order"], levels_bytes(d, m["ghosts"])),
    }
    out = {}
    for name, (ms, nbytes) in cands.items():
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"bound": "hbm", "kernel": name, "achieved": round(gbs, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
                     "traffic": kernel_traffic(name, W.name), "algorithmic_bytes": int(nbytes),
                     "avg_ms": round(ms, 5)}
    top = max(out, key=lambda k: out[k]["avg_ms"])
    return out[top], out


def stars_workload(gcr, torch, synth):
    insts = synth.stars64(seed=0)
    fields = []
    for inst in insts:
        for f in inst.fields:
            fields.append(_dev(torch, synth.sample(f, inst.grid), torch.float64))
    centre_of, beta_of = [], []

    def bc(pk, init=False):
        if init:
            # per ghost: its body's centre and the fields' angles (a static
            # body: the counts per instance are those of every step)
            cen, beta = [], []
            for inst, c in zip(insts, pk["counts"]):
                cen.append(np.repeat(np.asarray(inst.shape.center[:2])[:, None], c, axis=1))
                beta.append(np.repeat(np.asarray(inst.mixed_beta)[:, None], c, axis=1))
            pk["cen"] = _dev(torch, np.concatenate(cen, axis=1), torch.float64)
            pk["beta"] = _dev(torch, np.concatenate(beta, axis=1), torch.float64)
            return
        bc_star_fields(pk["S"], pk["n"], pk["cen"], pk["beta"], pk["bc"], pk["bt"])

    W = BatchStep(gcr, torch, "stars64", [i.grid for i in insts], [i.shape for i in insts],
                  [HGC] * len(insts), fields, [MIXED] * 3, True, [i.queries for i in insts],
                  p_field=2, u_first=0, bc_fn=bc)
    W.insts = insts
    W.cells = sum(i.grid.n_cells for i in insts)
    return W


def sphere_workload(gcr, torch, synth):
    inst = synth.sphere256(seed=0)
    base = [_dev(torch, synth.sample(f, inst.grid), torch.float64) for f in inst.fields]
    # one copy of the 4 fields per scheme: each scheme overwrites its own
    # ghost cells, and HGC's include fluid cells the other schemes read
    fields = [f.clone() for _ in range(3) for f in base]

    def bc(pk, init=False):
        if not init:
            bc_sphere_fields(pk["S"], pk["n"], out=pk["bc"])

    W = BatchStep(gcr, torch, "sphere256x3", [inst.grid] * 3, [inst.shape] * 3, [0, 1, 2], fields,
                  [DIRICHLET, DIRICHLET, DIRICHLET, NEUMANN], False, [inst.queries] * 3,
                  p_field=3, u_first=0, bc_fn=bc)
    W.inst = inst
    W.cells = 3 * inst.grid.n_cells
    return W


def plain_stars(gcr, torch, W, reps):
    """The headline step one instance at a time: a plan per instance,
    boundary data, the fill with one launch per level, the force."""

    def step():
        for i, inst in enumerate(W.insts):
            p = gcr.Plan(inst.grid, inst.shape, HGC)
            p.set_schedule(1)
            S, n = p.foot_points()
            cen = torch.tensor(inst.shape.center[:2], dtype=torch.float64, device="cuda")
            ng = p.n_ghost
            bc = torch.empty((3, ng), dtype=torch.float64, device="cuda")
            bt = torch.empty((3, ng), dtype=torch.uint8, device="cuda")
            beta = torch.tensor(np.repeat(np.asarray(inst.mixed_beta)[:, None], ng, axis=1),
                                device="cuda")
            bc_star_fields(S, n, cen[:, None].expand(2, ng), beta, bc, bt)
            fs = W.fields[3 * i:3 * i + 3]
            p.fill(fs, [MIXED] * 3, list(bc), bc_type=list(bt))
            p.forces(W.xq[i], W.nr[i], W.wq[i], fs[2], fs[:2], 1.0, out=W.F[i])
        return None

    step()
    torch.cuda.synchronize()
    med, _, _ = timed_steps(torch, step, reps)
    return med


def bench_fwd_bwd(gcr, torch, synth, reps):
    """384^3 spherical-harmonic star, HGC, u, v, w, p: the plain forward (fill
    with one launch per level, then the drag), the tuned forward, and forward
    + reverse-level adjoint (d drag / d interior field and boundary data).
    The dense zero-fill of the gradient buffers is timed on its own and kept
    out of the adjoint figure.  Roofline: the adjoint's level sweep
    (gcr_fill_adjoint), 128 B per (ghost, field) in 3D."""
    inst = synth.shstar384(seed=0)
    plan = gcr.Plan(inst.grid, inst.shape, HGC)
    kinds = [f.bc for f in inst.fields]
    nf = len(kinds)
    S, n = plan.foot_points()
    Sh, nh = S.cpu().numpy(), n.cpu().numpy()
    fields = [_dev(torch, synth.sample(f, inst.grid), torch.float64) for f in inst.fields]
    bcv = [_dev(torch, synth.bc_values(f, Sh, nh, k), torch.float64)
           for f, k in zip(inst.fields, kinds)]
    q = inst.queries
    xq, nr, wq = (_dev(torch, a) for a in (q.x, q.n, q.w))
    F = torch.empty(3, dtype=torch.float64, device="cuda")
    gF = torch.tensor([1.0, 0.0, 0.0], dtype=torch.float64, device="cuda")
    lam = [torch.zeros(plan.n_cells, dtype=torch.float64, device="cuda") for _ in range(nf)]
    lam_bc = [torch.empty(plan.n_ghost, dtype=torch.float64, device="cuda") for _ in range(nf)]

    def fwd():
        plan.fill(fields, kinds, bcv)
        plan.forces(xq, nr, wq, fields[3], fields[:3], 1.0, out=F)

    def seed():
        plan.forces_adjoint(xq, nr, wq, 1.0, gF, lam[3], lam[:3])

    def sweep():
        plan.fill_adjoint(lam, kinds, lam_bc)

    def zero():
        for t in lam:
            t.zero_()

    def fwd_bwd():
        fwd()
        seed()
        sweep()

    tf, _, _ = timed_steps(torch, fwd, reps)
    # the adjoint accumulates into lam: zeroed between timed calls, outside
    # the timed region
    tfb, p10, p90 = timed_steps(torch, fwd_bwd, reps, between=zero)
    tsw, _, _ = timed_steps(torch, sweep, reps, between=lambda: (zero(), seed()))
    tz, _, _ = timed_steps(torch, zero, reps)
    plan.set_schedule(1)
    tplain, _, _ = timed_steps(torch, fwd, reps)
    plan.set_schedule(0)
    ng = plan.n_ghost
    sweep_bytes = ng * nf * 128
    gbs = sweep_bytes / (tsw * 1e-3) / 1e9
    return {"workload": "shstar384: 384^3 grid on [-1,1]^3, SH star (l=2..4), u,v,w Dirichlet + "
                        "p Neumann, HGC, fill + drag, then adjoint of drag",
            "cells": plan.n_cells, "ghosts": ng, "fields": nf, "levels": plan.n_levels,
            "plain_fwd_ms": round(tplain, 4), "fwd_ms": round(tf, 4),
            "fwd_bwd_ms": round(tfb, 4), "fwd_bwd_p10_ms": round(p10, 4),
            "fwd_bwd_p90_ms": round(p90, 4),
            "fwd_bwd_over_plain_fwd": round(tfb / tplain, 3),
            "fwd_bwd_over_fwd": round(tfb / tf, 3),
            "fwd_ghost_cells_per_s": round(ng / (tf * 1e-3), 1),
            "fwd_bwd_ghost_cells_per_s": round(ng / (tfb * 1e-3), 1),
            "dense_grad_zero_ms": round(tz, 4),
            "roofline": {"bound": "hbm", "kernel": "gcr_fill_adjoint (level sweep)",
                         "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None,
                         "algorithmic_bytes": int(sweep_bytes), "avg_ms": round(tsw, 5)}}


def bench_latency(gcr, torch, synth, reps):
    """Single calls, one plan at a time: the 128^2 circle (CGC, CGC_ES and
    HGC; plan + fill of u + values and gradients at 256 boundary points) and
    the 4096^2 airfoil (HGC; plan + fill of u, v, p + values at 2 x 1024
    points + force).  The boundary data at the foot points are resident
    (a static body: the same foot points every call)."""
    out = {}
    circ = synth.circle128(seed=0)
    xq = _dev(torch, circ.queries.x)
    u = _dev(torch, synth.sample(circ.fields[0], circ.grid), torch.float64)
    bcs = {}
    for sch in (0, 1, 2):
        p = gcr.Plan(circ.grid, circ.shape, sch)
        S, n = p.foot_points()
        bcs[sch] = _dev(torch, synth.bc_values(circ.fields[0], S.cpu().numpy(), n.cpu().numpy(),
                                               DIRICHLET), torch.float64)
    per = {}
    for sch, name in ((0, "cgc"), (1, "cgc_es"), (2, "hgc")):
        def call(sch=sch):
            p = gcr.Plan(circ.grid, circ.shape, sch)
            p.fill([u], [DIRICHLET], [bcs[sch]])
            p.surface(xq, [u])
        med, p10, p90 = timed_steps(torch, call, reps)
        per[name] = {"ms_median": round(med, 4), "ms_p10": round(p10, 4), "ms_p90": round(p90, 4)}
    out["circle128"] = {"workload": "128^2 circle R=0.5: plan + fill of u + surface values and "
                                    "gradients at 256 points, one scheme per call", **per}
    air = synth.airfoil4096(seed=0)
    g = air.grid
    p = gcr.Plan(g, air.shape, HGC)
    S, n = p.foot_points()
    Sh, nh = S.cpu().numpy(), n.cpu().numpy()
    kinds = [DIRICHLET, DIRICHLET, NEUMANN]
    fields = [_dev(torch, synth.sample(f, g), torch.float64) for f in air.fields]
    bcv = [_dev(torch, synth.bc_values(f, Sh, nh, k), torch.float64)
           for f, k in zip(air.fields, kinds)]
    q = air.queries
    aq, an, aw = (_dev(torch, a) for a in (q.x, q.n, q.w))
    F = torch.empty(2, dtype=torch.float64, device="cuda")
    levels = p.n_levels
    ng = p.n_ghost
    del p

    def call():
        pl = gcr.Plan(g, air.shape, HGC)
        pl.fill(fields, kinds, bcv)
        pl.surface(aq, fields)
        pl.forces(aq, an, aw, fields[2], fields[:2], 1.0, out=F)

    med, p10, p90 = timed_steps(torch, call, reps)
    out["airfoil4096"] = {"workload": "4096^2 airfoil, HGC: plan + fill of u, v, p + surface "
                                      "values at 2048 points + force",
                          "ghosts": ng, "levels": levels, "ms_median": round(med, 4),
                          "ms_p10": round(p10, 4), "ms_p90": round(p90, 4)}
    return out


def hbm_copy(torch):
    """Device-to-device copy of 1 GiB: GB/s counted as bytes read + written."""
    nb = 1 << 30
    a = torch.ones(nb, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    med, _, _ = timed_steps(torch, lambda: b.copy_(a), 10)
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * nb, "ms_median": round(med, 4),
            "gbs": round(2 * nb / (med * 1e-3) / 1e9, 1)}


def bench_static(gcr, torch, W, steps):
    """The headline batch built once and forwarded repeatedly (a static body
    filled every time step): level-by-level sweep against the tiled fill."""
    static = {}
    stream = torch.cuda.current_stream()
    gcr.set_profiling(gcr.PROFILE_FORWARD)
    for mode, name in ((0, "sweep"), (2, "tiled")):
        gcr.set_batch_tiling(mode)
        B = W.batch()
        pk = W.pack(0, B.counts())
        B.foot_points(out=(pk["S"], pk["n"]))
        W.bc_fn(pk)
        for _ in range(3):
            B.forward(args=pk["args"])
        torch.cuda.synchronize()
        gcr.forward_times()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(steps):
            B.forward(args=pk["args"])
        t1.record(stream)
        torch.cuda.synchronize()
        ft = gcr.forward_times()
        static[name] = {"ms_per_forward": round(t0.elapsed_time(t1) / steps, 4),
                        "kernel_ms": round(ft["forward"], 5), "path": B.tiled()}
        del B
    gcr.set_batch_tiling(1)
    gcr.set_profiling(False)
    return static


def bench_layer2(gcr, torch, synth, reps):
    """The 256^3 sphere with a second ghost layer (HGC | LAYER2): plan,
    boundary data, fill of u, v, w, p and force, one plan at a time, beside
    the same step with HGC alone."""
    inst = synth.sphere256(seed=0)
    g = inst.grid
    fields = [_dev(torch, synth.sample(f, g), torch.float64) for f in inst.fields]
    kinds = [DIRICHLET, DIRICHLET, DIRICHLET, NEUMANN]
    q = inst.queries
    xq, nq, wq = (_dev(torch, a) for a in (q.x, q.n, q.w))
    F = torch.empty(3, dtype=torch.float64, device="cuda")
    out = {"workload": "sphere256, HGC with a second ghost layer (solid cells with "
                       "psi <= 1.5 delta n, extended stencils): plan + fill of u,v,w,p + force"}
    for name, sch in (("layer2", 2 | 4), ("hgc", 2)):
        info = {}

        def step():
            plan = gcr.Plan(g, inst.shape, sch)
            S, nrm = plan.foot_points()
            plan.fill(fields, kinds, list(bc_sphere_fields(S, nrm)))
            plan.forces(xq, nq, wq, fields[3], fields[:3], 1.0, out=F)
            info["ghosts"], info["levels"] = plan.n_ghost, plan.n_levels

        t, _, _ = timed_steps(torch, step, reps)
        out[name] = {"ghosts": info["ghosts"], "levels": info["levels"], "step_ms": round(t, 4),
                     "ghost_cells_per_s": round(info["ghosts"] / (t * 1e-3), 1)}
    return out


def bench_moving(gcr, torch, synth, reps):
    """The 256^3 sphere moving by 0.4 h per step (HGC with a second ghost
    layer, so that the cells the move exposes were ghosts before), two ways:
    full, a new plan at each position; incremental, two plans updated in
    turn (gcr_plan_update, each from two positions back), which classify
    again only the chunks the move can change.  Per step: the plan, its
    fresh cells against the previous position's plan, boundary data, fill
    of u, v, w, p and force.  Every step's fresh cells must be covered.
    Then the re-plan alone (plan + fresh cells) on the 1024^3 grid, where
    the classification of every cell is bandwidth-scale."""
    inst = synth.sphere256(seed=0)
    g, h = inst.grid, inst.grid.h[0]
    fields = [_dev(torch, synth.sample(f, g), torch.float64) for f in inst.fields]
    kinds = [DIRICHLET, DIRICHLET, DIRICHLET, NEUMANN]
    q = inst.queries
    xq, nq, wq = (_dev(torch, a) for a in (q.x, q.n, q.w))
    F = torch.empty(3, dtype=torch.float64, device="cuda")
    step_v = 0.4 * h * np.array([0.8, 0.48, 0.36])   # |v| = 0.4 h
    scheme = 2 | 4

    def shape_at(sh, k, v):
        c = tuple(float(x) for x in np.asarray(sh.center) + k * v)
        return synth.Shape(sh.kind, c, sh.r0)

    def run(mode, grid, sh, v, physics, nsteps):
        state = {"k": 0, "plans": [], "counts": []}
        replan = []

        def step():
            k = state["k"]
            state["k"] += 1
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            if mode == "full" or len(state["plans"]) < 2:
                plan = gcr.Plan(grid, shape_at(sh, k, v), scheme)
                state["plans"].append(plan)
            else:
                plan = state["plans"][-2].update(shape_at(sh, k, v))
                state["plans"].append(plan)
            prev = state["plans"][-2] if len(state["plans"]) > 1 else None
            if prev is not None:
                _, counts = prev.fresh_cells(plan)
                state["counts"].append(counts)
            t1.record()
            del state["plans"][:-2]
            if physics:
                S, nrm = plan.foot_points()
                plan.fill(fields, kinds, list(bc_sphere_fields(S, nrm)))
                plan.forces(xq, nq, wq, fields[3], fields[:3], 1.0, out=F)
            replan.append((t0, t1))

        for _ in range(2):   # both plans of the turn exist before timing
            step()
        replan.clear()
        t, p10, p90 = timed_steps(torch, step, nsteps)
        torch.cuda.synchronize()
        rp = float(np.median([a.elapsed_time(b) for a, b in replan]))
        counts = torch.stack(state["counts"][1:]).cpu().numpy()
        return {"step_ms": round(t, 4), "step_p10_ms": round(p10, 4),
                "step_p90_ms": round(p90, 4), "replan_ms": round(rp, 4),
                "fresh_per_step": int(counts[:, 0].mean()),
                "uncovered_total": int(counts[:, 1].sum()), "steps": int(len(counts))}

    out = {"workload": "sphere256 moving 0.4 h per step, HGC with a second ghost layer: "
                       "plan at the new position (full build, or an update of the plan two "
                       "positions back) + fresh cells against the previous position's plan + "
                       "boundary data + fill of u,v,w,p + force; replan_ms: plan + fresh "
                       "cells alone"}
    for mode in ("full", "incremental"):
        out[mode] = run(mode, g, inst.shape, step_v, True, reps)
    out["incremental_over_full"] = round(out["full"]["step_ms"] / out["incremental"]["step_ms"], 3)
    del fields
    big = synth.sphere256(seed=0, n=1024)
    hb = big.grid.h[0]
    vb = 0.4 * hb * np.array([0.8, 0.48, 0.36])
    out["sphere1024"] = {"workload": "sphere1024 (1.07e9 cells) moving 0.4 h per step, HGC with "
                                     "a second ghost layer: plan + fresh cells"}
    for mode in ("full", "incremental"):
        r = run(mode, big.grid, big.shape, vb, False, max(4, reps // 2))
        out["sphere1024"][mode] = {k: r[k] for k in ("replan_ms", "fresh_per_step",
                                                      "uncovered_total", "steps")}
    out["sphere1024"]["incremental_over_full"] = round(
        out["sphere1024"]["full"]["replan_ms"] / out["sphere1024"]["incremental"]["replan_ms"], 3)
    return out


def bench_large(gcr, torch, synth, reps):
    """The 256^3 workload's sphere on a 1024^3 grid (1.07e9 cells): the size
    at which the classification pass (1 byte per cell written) is
    bandwidth-scale.  HGC plan, fill of u, v, w, p, force; fields generated
    on the device."""
    inst = synth.sphere256(seed=0, n=1024)
    g = inst.grid
    dev = "cuda"
    ax = [g.lo[a] + (torch.arange(g.n[a], dtype=torch.float64, device=dev) + 0.5) * g.h[a]
          for a in range(3)]
    x, y, z = ax[0][None, None, :], ax[1][None, :, None], ax[2][:, None, None]
    shape = (g.n[2], g.n[1], g.n[0])
    fields = [(torch.sin(z) + torch.cos(y)).expand(shape).contiguous().view(-1),
              (torch.sin(x) + torch.cos(z)).expand(shape).contiguous().view(-1),
              (torch.sin(y) + torch.cos(x)).expand(shape).contiguous().view(-1),
              (torch.cos(x) * torch.cos(y) * torch.cos(z)).contiguous().view(-1)]
    kinds = [DIRICHLET, DIRICHLET, DIRICHLET, NEUMANN]
    q = inst.queries
    xq, nq, wq = (_dev(torch, a) for a in (q.x, q.n, q.w))
    F = torch.empty(3, dtype=torch.float64, device=dev)
    info = {}

    def step():
        plan = gcr.Plan(g, inst.shape, 2)
        info["times"] = gcr.last_build_times()
        info["seg"] = plan.stats()["n_band_segments"]
        info["ng"] = plan.n_ghost
        S, nrm = plan.foot_points()
        plan.fill(fields, kinds, list(bc_sphere_fields(S, nrm)))
        plan.forces(xq, nq, wq, fields[3], fields[:3], 1.0, out=F)

    gcr.set_profiling(True)
    step()
    cls = []
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        step()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
        cls.append(info["times"]["classify_prepass"] + info["times"]["classify_store"])
    gcr.set_profiling(False)
    t = float(np.median(ts))
    c = float(np.median(cls))
    ncell = g.n[0] * g.n[1] * g.n[2]
    cbytes = ncell   # the span and store passes write every cell's tag
    del fields
    torch.cuda.empty_cache()
    return {"workload": "sphere1024: 1024^3 grid on [-1,1]^3, the 256^3 workload's sphere, HGC, "
                        "plan + fill of u,v,w,p + force",
            "cells": ncell, "ghosts": info["ng"], "step_ms": round(t, 4),
            "ghost_cells_per_s": round(info["ng"] / (t * 1e-3), 1),
            "classify_store_ms": round(c, 5),
            "classify_roofline": {"bound": "hbm", "kernel": "k_spans + k_classify",
                                  "achieved": round(cbytes / (c * 1e-3) / 1e9, 2),
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(cbytes / (c * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "algorithmic_bytes": cbytes}}


# ---------------------------------------------------------------------------
# CPU baselines: the oracle as it stands, on the host of the GPU
# ---------------------------------------------------------------------------

def _oracle_stars(indices, budget):
    """Oracle time of the headline workload's path (plan, boundary data,
    mixed fill, surface values, force) on the given instances: (ghosts, s)."""
    import oracle
    import synth
    insts = synth.stars64(seed=0)
    ng, t = 0, 0.0
    for k in indices:
        inst = insts[k]
        g = inst.grid
        vals = np.stack([synth.sample(f, g) for f in inst.fields])
        t0 = time.perf_counter()
        p = oracle.OraclePlan(g, inst.shape, HGC)
        c = p.ghost_cell
        S = np.stack([g.lo[0] + (c % g.n[0] + 0.5) * g.h[0],
                      g.lo[1] + (c // g.n[0] + 0.5) * g.h[1]]) + p.delta
        kinds = np.stack([synth.mixed_kinds(S, inst.shape.center, b) for b in inst.mixed_beta])
        b = np.stack([synth.bc_values(f, S, p.normal, kk) for f, kk in zip(inst.fields, kinds)])
        out = p.fill(vals, kinds, b)
        q = inst.queries
        p.surface_query(q.x, out)
        p.forces(q.x, q.n, q.w, out[2], out[:2], 1.0)
        t += time.perf_counter() - t0
        ng += p.n_ghost
        if t > budget:
            break
    return ng, t


def _child_single_thread(budget):
    """The single-thread oracle sample in a child process (OpenMP threads are
    fixed when the oracle library loads)."""
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import sys, json; sys.path.insert(0, %r); import bench; "
            "print(json.dumps(bench._oracle_stars(list(range(0, 64, 4)), %f)))" % (ROOT, budget))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        return None
    ng, t = json.loads(r.stdout.strip().splitlines()[-1])
    return ng, t


def cpu_baseline_stars(seconds):
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    ng, t = _oracle_stars(range(64), 3 * seconds)
    one = _child_single_thread(seconds)
    out = {"value": round(ng / t, 1), "unit": "ghost cells/s", "cores": threads,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"the headline workload's path per instance (plan, boundary data, mixed "
                     f"fill, surface values, force), {ng} ghosts in {t:.1f} s of oracle time; "
                     f"cores = OpenMP threads of its one parallel loop (classification)"}
    if one is not None:
        out["single_thread"] = {"value": round(one[0] / one[1], 1), "unit": "ghost cells/s",
                                "sample": f"every 4th instance, {one[0]} ghosts in "
                                          f"{one[1]:.1f} s"}
    return out


def cpu_baseline_fwd_bwd():
    """The oracle's forward (plan, fill, drag) and forward + adjoint on the
    384^3 star."""
    import oracle
    import synth
    inst = synth.shstar384(seed=0)
    g = inst.grid
    kinds = [f.bc for f in inst.fields]
    vals = np.stack([synth.sample(f, g) for f in inst.fields])
    q = inst.queries
    t0 = time.perf_counter()
    p = oracle.OraclePlan(g, inst.shape, HGC)
    c = p.ghost_cell
    idx = [c % g.n[0], (c // g.n[0]) % g.n[1], c // (g.n[0] * g.n[1])]
    S = np.stack([g.lo[i] + (idx[i] + 0.5) * g.h[i] for i in range(3)]) + p.delta
    b = np.stack([synth.bc_values(f, S, p.normal, k) for f, k in zip(inst.fields, kinds)])
    out = p.fill(vals, kinds, b)
    p.forces(q.x, q.n, q.w, out[3], out[:3], 1.0)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    nq = q.x.shape[1]
    gval = np.zeros((4, nq))
    ggrad = np.zeros((4, 3, nq))
    gval[3] = -q.w * q.n[0]
    for i in range(3):
        for j in range(3):
            ggrad[i, j] = q.w * ((1.0 if i == 0 else 0.0) * q.n[j] + (1.0 if j == 0 else 0.0) * q.n[i])
    L0 = p.surface_query_adjoint(q.x, gval, ggrad, np.zeros((4, p.n_cells)))
    p.fill_adjoint(L0, kinds)
    t_bwd = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(p.n_ghost / (t_fwd + t_bwd), 1), "unit": "ghost cells/s",
            "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"one forward (plan, fill, drag: {t_fwd:.2f} s) and adjoint "
                      f"({t_bwd:.2f} s) of the 384^3 star; cores = OpenMP threads of the "
                      f"classification loop",
            "fwd_s": round(t_fwd, 3), "bwd_s": round(t_bwd, 3)}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: measures one GPU; --gpus must be 1 (the multi-GPU layout is a design, "
              "not code)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2609_10165_amd as gcr
    import synth

    dev = torch.device("cuda:0")
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        a = torch.ones(nb, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    s_fwd = torch.cuda.Stream(device=dev)
    s_builds = [torch.cuda.Stream(device=dev) for _ in range(3)]

    W = stars_workload(gcr, torch, synth)
    m = measure_batched(gcr, torch, W, args, s_fwd, s_builds, extra=not args.only_headline)
    value = m["ghosts"] / (m["ms_per_step"] * 1e-3)
    roofline, rooflines = roofline_of(W, m, W.cells)
    out = {
        "metric": "ghost cells/s (plan + fill + surface + forces, 64 batched instances)",
        "value": round(value, 1),
        "unit": "ghost cells/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "stars64: 64 2D star bodies (Fourier modes k=2..5), square grids "
                               "n ~ U{128..2048} on [-1,1]^2, HGC, 3 FP64 fields with mixed "
                               "Dirichlet/Neumann data per ghost, 256 surface points each; per "
                               "step a batch built and forwarded (fill + surface values + force "
                               "in one persistent launch); steps pipelined: batches built by "
                               "host threads on streams of their own, forwards on another",
                   "ghosts_per_step": m["ghosts"], "cells": W.cells, "instances": W.ninst,
                   "build_threads": m["nbuild"]},
        "roofline": roofline,
    }
    if args.only_headline:
        print(json.dumps(out), flush=True)
        return
    out["rooflines"] = rooflines
    out["stage_ms"] = {k: round(v, 5) for k, v in m["stage_ms"].items()}
    out["forward_kernel_ms"] = round(m["fwd_ms"], 5)
    out["bc_graph"] = W.bc_graph_ok
    out["serial_step"] = {"ms_per_step": round(m["ms_serial"], 4),
                          "ghost_cells_per_s": round(m["ghosts"] / (m["ms_serial"] * 1e-3), 1),
                          "pipelined_speedup": round(m["ms_serial"] / m["ms_per_step"], 3)}
    cl = m["cold_llc"]
    out["cold_llc"] = {"what": "the same steps one after another, each timed alone; cold: a "
                               "1 GiB write between steps flushes the 256 MB last-level cache",
                       **{k: round(v, 4) for k, v in cl.items()},
                       "ghost_cells_per_s_cold": round(m["ghosts"] / (cl["ms_median"] * 1e-3), 1)}
    ms_plain = plain_stars(gcr, torch, W, max(3, args.extra_reps // 2))
    out["plain_step"] = {"what": "one instance at a time: plan, boundary data, fill with one "
                                 "launch per level, force",
                         "ms_per_step": round(ms_plain, 4),
                         "ghost_cells_per_s": round(m["ghosts"] / (ms_plain * 1e-3), 1),
                         "speedup_of_serial_batched": round(ms_plain / m["ms_serial"], 3),
                         "speedup_of_pipelined": round(ms_plain / m["ms_per_step"], 3)}
    out["static_forward"] = bench_static(gcr, torch, W, args.steps)
    out["hbm_copy"] = hbm_copy(torch)
    out["wall_s"] = round(m["wall_s"], 3)
    del W
    gc.unfreeze()
    gc.collect()
    torch.cuda.synchronize()

    if not args.no_extras:
        Ws = sphere_workload(gcr, torch, synth)
        ms = measure_batched(gcr, torch, Ws, args, s_fwd, s_builds, extra=False)
        r_s, _ = roofline_of(Ws, ms, Ws.cells)
        out["sphere256"] = {"workload": "256^3 sphere R=0.3, CGC + CGC_ES + HGC as one batch, "
                                        "u,v,w Dirichlet + p Neumann, 2048 surface points, "
                                        "pipelined like the headline",
                            "ghosts_per_step": ms["ghosts"],
                            "ms_per_step": round(ms["ms_per_step"], 4),
                            "ghost_cells_per_s": round(ms["ghosts"] / (ms["ms_per_step"] * 1e-3), 1),
                            "ms_serial": round(ms["ms_serial"], 4),
                            "forward_kernel_ms": round(ms["fwd_ms"], 5),
                            "stage_ms": {k: round(v, 5) for k, v in ms["stage_ms"].items()},
                            "roofline": r_s}
        del Ws
        gc.unfreeze()
        gc.collect()
        out["fwd_bwd"] = bench_fwd_bwd(gcr, torch, synth, args.extra_reps)
        out["latency"] = bench_latency(gcr, torch, synth, args.extra_reps)
        out["layer2"] = bench_layer2(gcr, torch, synth, args.extra_reps)
        out["moving"] = bench_moving(gcr, torch, synth, args.extra_reps)
        out["large"] = bench_large(gcr, torch, synth, max(3, args.extra_reps // 2))

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_stars(args.cpu_seconds)
        if "fwd_bwd" in out:
            out["fwd_bwd"]["cpu_baseline"] = cpu_baseline_fwd_bwd()
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
