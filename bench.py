"""Benchmark of the ghost-cell hot path on one MI355X.

One step = the whole path on a 256^3 grid cut by a sphere (R = 0.3,
sub-cell offset) with four FP64 fields (u, v, w Dirichlet; p Neumann), for
each of the three ghost schemes (CGC, CGC_ES, HGC), the three built and
applied as one batch:
  plans (classification, tags, geometry, dependency levels, canonical order)
  -> foot points and boundary data there (caller side, torch)
  -> level-by-level fill of the 4 fields, their values and gradients at
     2048 surface points and the pressure + viscous force there (one
     persistent launch for all schemes and fields).
Metric: ghost cells per second (sum of the three plans' ghosts per step).
The timed steps run pipelined over two HIP streams: each step builds its
own batch and computes its boundary data on one stream while the previous
step's forward runs on the other (every step still does the whole path).
The same steps one after another on one stream (serial_step) and one plan
at a time (plain_step) are timed beside it.

Side measurements on the same GPU (reported beside the headline, never as
`value`):
  batched  64 2D star instances, n ~ U{128..2048}, 3 fields with mixed
           Dirichlet/Neumann data, HGC: one persistent launch (fill + force)
           against the plain per-instance forward (per-level launches);
  fwd_bwd  384^3 grid, spherical-harmonic star, u, v, w, p, HGC: fill + drag
           forward, then the reverse-level adjoint, against the forward alone;
  layer2   the headline sphere with a second ghost layer, against HGC alone;
  moving   that sphere moving 0.4 h per step: a plan per step, the fresh
           cells against the previous plan (all covered by the second
           layer), fill and force;
  large    the headline sphere on 1024^3 (classification at 1.07 GB).

Prints one JSON line.  Only N=1 is supported (one GPU).
"""
from __future__ import annotations

import argparse
import collections
import gc
import queue
import threading
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
SCHEMES = (0, 1, 2)
DIRICHLET, NEUMANN, MIXED = 0, 1, 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--build-threads", type=int, default=2, choices=(1, 2, 3),
                    help="host threads building batches in the timed steps (each on "
                         "a stream of its own; the forwards are enqueued by another)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="oracle time budget of the CPU baseline sample")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and forward+adjoint side measurements")
    ap.add_argument("--extra-reps", type=int, default=10)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first "
                         "(reference kernel for byte counters)")
    return ap.parse_args()


def bc_sphere_fields(S, n, out=None):
    """Boundary data of the u, v, w, p fields at the foot points: values of
    u = sin z + cos y, v = sin x + cos z, w = sin y + cos x and the normal
    derivative of p = cos x cos y cos z, written dp/dn = -(c_x c_y c_z)
    sum_i tan(S_i) n_i (cos > 0.5 on the domain) to keep the caller's
    launches few (caller side, torch; into `out` [4][n] if given)."""
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


def _dev(torch, a, dtype=None):
    """Contiguous device copy of a host array (inputs resident in HBM)."""
    a = np.ascontiguousarray(a)
    return torch.tensor(a, dtype=dtype, device="cuda")


def kernel_traffic(name, workload):
    """HBM bytes per launch of kernel `name` on `workload` from the committed
    byte-counter summary, or None when it is absent or the kernel's sources
    changed since."""
    path = os.path.join(ROOT, "profiles", f"{name}_{workload}_traffic.json")
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


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: measures one GPU; --gpus must be 1 (the multi-GPU layout is a design, not code)", file=sys.stderr)
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

    inst = synth.sphere256(seed=0)
    grid, shape = inst.grid, inst.shape
    kinds = [DIRICHLET, DIRICHLET, DIRICHLET, NEUMANN]
    # inputs resident in HBM before timing: one copy of the 4 fields per
    # scheme (each scheme overwrites its own ghost cells, and HGC's include
    # fluid cells that the other schemes read)
    base = [_dev(torch, synth.sample(f, grid), torch.float64) for f in inst.fields]
    fieldsets = [[f.clone() for f in base] for _ in SCHEMES]
    q = inst.queries
    xq, nq, wq = (_dev(torch, a) for a in (q.x, q.n, q.w))
    nqp = xq.shape[1]
    F3 = torch.zeros((len(SCHEMES), 3), dtype=torch.float64, device=dev)
    # surface values and gradients of the 4 fields at the points, per scheme
    sval = [torch.empty(nqp, dtype=torch.float64, device=dev) for _ in range(4 * len(SCHEMES))]
    sgrad = [torch.empty((3, nqp), dtype=torch.float64, device=dev)
             for _ in range(4 * len(SCHEMES))]
    F = torch.empty(3, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    seg = []

    # foot points and boundary data go to buffers kept across steps, and the
    # forward's pointer tables are packed once for them (repacked only if
    # the ghost counts change, which they do not for a fixed body)
    pack = {}

    def buffers(counts):
        if pack.get("counts") != counts:
            ng = sum(counts)
            S_buf = torch.empty((3, ng), dtype=torch.float64, device=dev)
            n_buf = torch.empty((3, ng), dtype=torch.float64, device=dev)
            bc = torch.empty((4, ng), dtype=torch.float64, device=dev)
            bcv, off = [], 0
            for c in counts:
                bcv += [bc[f, off:off + c] for f in range(4)]
                off += c
            args = gcr.ForwardArgs(4, [f for fs in fieldsets for f in fs], kinds, bcv,
                                   nq=[nqp] * len(SCHEMES), xq=[xq] * len(SCHEMES),
                                   nrm=[nq] * len(SCHEMES), wq=[wq] * len(SCHEMES), p_field=3,
                                   u_first=0, mu=1.0, F=F3, sval=sval, sgrad=sgrad)
            pack.update(counts=counts, S=S_buf, n=n_buf, bc=bc, args=args)
        return pack

    def step(record=None):
        """The three schemes as one batch: shared build launches, boundary
        data for all foot points at once, then fill, surface values and
        force of every (scheme, field) in one persistent launch."""
        B = gcr.Batch([grid] * len(SCHEMES), [shape] * len(SCHEMES), list(SCHEMES))
        if record is not None:
            record.append(gcr.last_build_times())
        pk = buffers(tuple(p.n_ghost for p in B.plans))
        bc_sphere_fields(*B.foot_points(out=(pk["S"], pk["n"])), out=pk["bc"])
        B.forward(args=pk["args"])
        seg.append(B.plans[0].stats()["n_band_segments"])
        return sum(pk["counts"])

    # pipelined form: the build, foot points and boundary data of a step on
    # one stream, its forward on another, so a step's build overlaps the
    # previous step's forward.  Boundary data alternate between two buffer
    # sets (a set is rewritten only after the forward that read it, two
    # steps back, has run), and a batch is released only once its forward
    # has run, so no pooled memory is reused while still read.
    s_build = torch.cuda.Stream(device=dev)
    s_fwd = torch.cuda.Stream(device=dev)
    packs = [{}, {}]

    def buffers_k(k, counts):
        pk = packs[k]
        if pk.get("counts") != counts:
            ng = sum(counts)
            bc = torch.empty((4, ng), dtype=torch.float64, device=dev)
            bcv, off = [], 0
            for c in counts:
                bcv += [bc[f, off:off + c] for f in range(4)]
                off += c
            pk.update(counts=counts, bc=bc,
                      S=torch.empty((3, ng), dtype=torch.float64, device=dev),
                      n=torch.empty((3, ng), dtype=torch.float64, device=dev),
                      args=gcr.ForwardArgs(4, [f for fs in fieldsets for f in fs], kinds, bcv,
                                           nq=[nqp] * len(SCHEMES), xq=[xq] * len(SCHEMES),
                                           nrm=[nq] * len(SCHEMES), wq=[wq] * len(SCHEMES),
                                           p_field=3, u_first=0, mu=1.0, F=F3, sval=sval,
                                           sgrad=sgrad))
        return pk

    def bc_graph(pk):
        """The boundary-data evaluation on this buffer set captured as one
        HIP graph, or None if its replays do not reproduce the eager result
        bitwise (checked on several inputs, with eager work and
        synchronisations between the replays)."""
        if "graph" in pk:
            return pk["graph"]
        pk["graph"] = None
        S0 = pk["S"].clone()
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            bc_sphere_fields(pk["S"], pk["n"], out=pk["bc"])   # warm-up before capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        try:
            with torch.cuda.graph(g):
                bc_sphere_fields(pk["S"], pk["n"], out=pk["bc"])
            torch.cuda.synchronize()
        except RuntimeError:
            return None
        for r in range(4):
            pk["S"].copy_(S0 * (1.0 + 1e-3 * r))
            want = bc_sphere_fields(pk["S"], pk["n"])
            torch.cuda.synchronize()
            pk["bc"].fill_(float("nan"))
            g.replay()
            torch.cuda.synchronize()
            if not torch.equal(pk["bc"], want):
                return None
        pk["S"].copy_(S0)
        pk["graph"] = g
        return g

    def run_pipelined(nsteps):
        held = collections.deque()   # (batch, its forward's completion event)
        ng = 0
        for t in range(nsteps):
            with torch.cuda.stream(s_build):
                B = gcr.Batch([grid] * len(SCHEMES), [shape] * len(SCHEMES), list(SCHEMES),
                              stream=s_build)
                pk = buffers_k(t & 1, tuple(p.n_ghost for p in B.plans))
                if len(held) == 2:
                    s_build.wait_event(held[0][1])   # last reader of this buffer set
                B.foot_points(stream=s_build, out=(pk["S"], pk["n"]))
                if pk.get("graph") is not None:
                    pk["graph"].replay()
                else:
                    bc_sphere_fields(pk["S"], pk["n"], out=pk["bc"])
                ready = torch.cuda.Event()
                ready.record(s_build)
            s_fwd.wait_event(ready)
            B.forward(args=pk["args"], stream=s_fwd)
            done = torch.cuda.Event()
            done.record(s_fwd)
            held.append((B, done))
            if len(held) > 2:
                _, e0 = held.popleft()
                e0.synchronize()
            ng = sum(pk["counts"])
        for _, e in held:
            e.synchronize()
        return ng

    s_builds = [s_build] + [torch.cuda.Stream(device=dev) for _ in range(2)]

    def run_pipelined_threads(nsteps, nbuild=1):
        """The same steps with the host work split over threads: `nbuild`
        threads build batches (each on a build stream of its own), another
        takes each built batch and enqueues its foot points, boundary data
        and forward on the forward stream, so a build starts while earlier
        forwards are being enqueued and run (and, with two builders, while
        the other build waits for its read-backs).  A batch is handed over
        only once built (the build synchronises its stream; the forward
        stream also waits for an event recorded after it), everything after
        that is in order on the forward stream, and a batch is dropped only
        after its forward's event."""
        q = queue.Queue(maxsize=2)
        tickets = queue.Queue()
        for _ in range(nsteps):
            tickets.put(True)
        for _ in range(nbuild):
            tickets.put(None)
        err = []
        ng = [0]

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
                        pk = buffers_k(t & 1, tuple(p.n_ghost for p in B.plans))
                        B.foot_points(stream=s_fwd, out=(pk["S"], pk["n"]))
                        if pk.get("graph") is not None:
                            pk["graph"].replay()
                        else:
                            bc_sphere_fields(pk["S"], pk["n"], out=pk["bc"])
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
                        B = gcr.Batch([grid] * len(SCHEMES), [shape] * len(SCHEMES),
                                      list(SCHEMES), stream=st)
                        built = torch.cuda.Event()
                        built.record(st)
                    ng[0] = sum(p.n_ghost for p in B.plans)
                    q.put((B, built))
                    del B
            except Exception as e:
                err.append(e)
                while tickets.get() is not None:   # let the other builders finish
                    pass

        fw = threading.Thread(target=forwarder)
        fw.start()
        bs = [threading.Thread(target=builder, args=(st,))
              for st in s_builds[:nbuild]]
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
        return ng[0]

    def step_plain():
        """The same work one plan at a time: per-plan build, per-level fill
        launches, one surface and one force launch per scheme."""
        ng_total = 0
        for sch, fs in zip(SCHEMES, fieldsets):
            plan = gcr.Plan(grid, shape, sch)
            S, nrm = plan.foot_points()
            plan.fill(fs, kinds, list(bc_sphere_fields(S, nrm)))
            plan.surface(xq, fs)
            plan.forces(xq, nq, wq, fs[3], fs[:3], 1.0, out=F)
            ng_total += plan.n_ghost
            del plan
        return ng_total

    # the timed loop records events around the batched forward's kernels
    # only (the roofline's kernel time); build-stage times come from extra
    # steps after it
    gcr.set_profiling(gcr.PROFILE_FORWARD)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    gc.collect()
    gc.freeze()   # see below
    gcr.forward_times()   # drop the warm-up calls' events
    rec = []
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    wall0 = time.perf_counter()
    ng_step = 0
    for _ in range(args.steps):
        ng_step = step()
    t1.record(stream)
    torch.cuda.synchronize()
    ms_serial = t0.elapsed_time(t1) / args.steps
    # the headline: the same steps pipelined over streams, first from one
    # host thread, then with the forward's host work on a second thread,
    # then (timed for the headline) with `--build-threads` builders
    run_pipelined(2)
    torch.cuda.synchronize()
    use_graph = all(bc_graph(pk) is not None for pk in packs)
    if not use_graph:
        for pk in packs:
            pk["graph"] = None
    run_pipelined(4)
    torch.cuda.synchronize()
    # grow the library's device and pinned pools to the deepest pipeline
    # (up to three batches building, two queued, one being enqueued and
    # three held until their forwards end): as many batches built and
    # forwarded at once, then released, so no timed step meets an empty
    # pool (a hipMalloc there stalls the whole pipeline)
    with torch.cuda.stream(s_build):
        pool_fill = [gcr.Batch([grid] * len(SCHEMES), [shape] * len(SCHEMES), list(SCHEMES),
                               stream=s_build) for _ in range(12)]
        pk0 = buffers_k(0, tuple(p.n_ghost for p in pool_fill[0].plans))
        for Bp in pool_fill:
            Bp.forward(args=pk0["args"], stream=s_build)
    torch.cuda.synchronize()
    del pool_fill, Bp
    # the warm-ups have grown the device-memory pools to the pipelines'
    # depth; objects made so far are frozen out of the cycle collector's
    # scans (a full scan of torch's objects costs milliseconds), as a
    # long-running solver or server would
    gc.collect()
    gc.freeze()
    gcr.forward_times()   # drop the serial and warm-up calls' events
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    run_pipelined(args.steps)
    torch.cuda.synchronize()
    ms_pipe1 = (time.perf_counter() - w0) * 1e3 / args.steps
    run_pipelined_threads(8)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    run_pipelined_threads(args.steps)
    torch.cuda.synchronize()
    ms_pipe2 = (time.perf_counter() - w0) * 1e3 / args.steps
    nbuild = args.build_threads
    run_pipelined_threads(8 + 2 * nbuild, nbuild=nbuild)
    torch.cuda.synchronize()
    gcr.forward_times()   # drop the events of the runs before the timed one
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ng_step = run_pipelined_threads(args.steps, nbuild=nbuild)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = wall * 1e3 / args.steps
    value = ng_step / (ms_step * 1e-3)
    fwd_times = gcr.forward_times()   # events recorded around the kernels in the timed loop
    # build-stage times: as many steps again with stage events on
    gcr.set_profiling(gcr.PROFILE_BUILD)
    t0.record(stream)
    for _ in range(args.steps):
        step(rec)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_step_profiled = t0.elapsed_time(t1) / args.steps
    gcr.set_profiling(False)
    band_segments = seg[-1]

    # a static body: the batch built once and forwarded repeatedly (as a
    # solver fills every time step), level-by-level sweep against the tiled
    # fill (tiles set up on the first call, outside the timing)
    static = {}
    gcr.set_profiling(gcr.PROFILE_FORWARD)
    for mode, name in ((0, "sweep"), (2, "tiled")):
        gcr.set_batch_tiling(mode)
        Bs = gcr.Batch([grid] * len(SCHEMES), [shape] * len(SCHEMES), list(SCHEMES))
        pk = buffers(tuple(p.n_ghost for p in Bs.plans))
        bc_sphere_fields(*Bs.foot_points(out=(pk["S"], pk["n"])), out=pk["bc"])
        for _ in range(3):
            Bs.forward(args=pk["args"])
        torch.cuda.synchronize()
        gcr.forward_times()
        t0.record(stream)
        for _ in range(args.steps):
            Bs.forward(args=pk["args"])
        t1.record(stream)
        torch.cuda.synchronize()
        ft = gcr.forward_times()
        static[name] = {"ms_per_forward": round(t0.elapsed_time(t1) / args.steps, 4),
                        "kernel_ms": round(ft["forward"], 5), "path": Bs.tiled()}
        del Bs
    gcr.set_batch_tiling(1)
    gcr.set_profiling(False)

    # plain per-plan form of the same step, for comparison
    for _ in range(2):
        step_plain()
    torch.cuda.synchronize()
    plain_reps = max(3, args.steps // 2)
    t0.record(stream)
    for _ in range(plain_reps):
        ng_plain = step_plain()
    t1.record(stream)
    torch.cuda.synchronize()
    ms_plain = t0.elapsed_time(t1) / plain_reps

    # HBM-bound kernel: the classification store pass writes the dense tag
    # array, 1 byte per cell of the three instances, except the 16-cell row
    # segments near the body that the band pass writes; its duration from
    # HIP events recorded around the launch on the build stream (the
    # stage-event steps after the timed loop)
    cls_ms = float(np.mean([r["classify_store"] for r in rec]))
    stage_ms = {k: float(np.mean([r[k] for r in rec])) for k in rec[0]}
    ncell = grid.n[0] * grid.n[1] * grid.n[2]
    cls_bytes = len(SCHEMES) * ncell - 16 * band_segments
    achieved = cls_bytes / (cls_ms * 1e-3) / 1e9
    traffic = kernel_traffic("k_classify", "sphere256x3")
    roofline_classify = {"bound": "hbm", "kernel": "k_classify", "achieved": round(achieved, 2),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                         "algorithmic_bytes": cls_bytes, "avg_ms": round(cls_ms, 5)}
    # the step's longest kernel: the persistent fill + surface + force
    # launch.  Bytes it must move: per ghost and field, 2^d - 1 stencil
    # values, the boundary datum and the result (72 B in 3D); per ghost,
    # cell, code, unit, delta and normal once (60 B); per surface point,
    # position, normal, weight and anchor (60 B), and per field the 2^d
    # corner values read (64 B) and the value and gradient written (32 B).
    fwd_ms = fwd_times["forward"]
    fwd_bytes = ng_step * (4 * 72 + 60) + len(SCHEMES) * nqp * (60 + 4 * (64 + 32))
    fwd_gbs = fwd_bytes / (fwd_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "k_batch_forward", "achieved": round(fwd_gbs, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(fwd_gbs / HBM_PEAK_GBS, 4),
                "traffic": kernel_traffic("k_batch_forward", "sphere256x3"),
                "algorithmic_bytes": fwd_bytes, "avg_ms": round(fwd_ms, 5),
                "note": "latency-bound: 11-12 dependent levels, each a pass of dependent "
                        "loads and a barrier"}
    for name in ("sweep", "tiled"):
        km = static[name]["kernel_ms"]
        gbs = fwd_bytes / (km * 1e-3) / 1e9
        static[name]["achieved_gbs"] = round(gbs, 2)
        static[name]["frac"] = round(gbs / HBM_PEAK_GBS, 4)
    static["workload"] = ("the step's batch built once, then fill + surface + force of every "
                          "(scheme, field) repeated; kernel_ms: the fill, surface and force kernels "
                          "of one call (tiled: k_tile_fill + k_batch_forward)")
    plain = {"ms_per_step": round(ms_plain, 4), "ghosts_per_step": ng_plain,
             "ghost_cells_per_s": round(ng_plain / (ms_plain * 1e-3), 1),
             "batched_speedup": round(ms_plain / ms_serial, 3)}

    extras = {}
    if not args.no_extras:
        extras["batched"] = bench_batched(gcr, torch, synth, args.extra_reps)
        extras["fwd_bwd"] = bench_fwd_bwd(gcr, torch, synth, args.extra_reps)
        extras["layer2"] = bench_layer2(gcr, torch, synth, args.extra_reps)
        extras["moving"] = bench_moving(gcr, torch, synth, args.extra_reps)
        extras["large"] = bench_large(gcr, torch, synth, max(3, args.extra_reps // 2))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inst, args.cpu_seconds)

    out = {
        "metric": "ghost cells/s (plan + fill + surface + forces, all 3 schemes)",
        "value": round(value, 1),
        "unit": "ghost cells/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "sphere256: 256^3 grid on [-1,1]^3, sphere R=0.3 at sub-cell "
                               "offset, 4 FP64 fields (u,v,w Dirichlet, p Neumann), "
                               "CGC + CGC_ES + HGC per step as one batch, 2048 surface points; "
                               "steps pipelined: batches built by host threads on streams of "
                               "their own, each step's forward on another stream",
                   "ghosts_per_step": ng_step, "cells": ncell, "build_threads": nbuild},
        "roofline": roofline,
        "roofline_classify": roofline_classify,
        "static_forward": static,
        "plain_step": plain,
        "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "ms_per_step_stage_events": round(ms_step_profiled, 4),
        "bc_graph": use_graph,
        "serial_step": {"ms_per_step": round(ms_serial, 4),
                        "ghost_cells_per_s": round(ng_step / (ms_serial * 1e-3), 1),
                        "pipelined_speedup": round(ms_serial / ms_step, 3)},
        "pipelined_one_host_thread": {"ms_per_step": round(ms_pipe1, 4),
                                      "ghost_cells_per_s": round(ng_step / (ms_pipe1 * 1e-3), 1)},
        "pipelined_one_build_thread": {"ms_per_step": round(ms_pipe2, 4),
                                       "ghost_cells_per_s": round(ng_step / (ms_pipe2 * 1e-3), 1)},
        "wall_s": round(wall, 3),
        **extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _time(torch, fn, reps):
    """Median and mean ms of `fn` over `reps` calls, HIP events on the
    current stream, one untimed call first."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts)), float(np.mean(ts))


def bench_batched(gcr, torch, synth, reps):
    """64 uneven 2D instances: the persistent batched forward against the
    plain per-instance forward (one launch per level, uncaptured)."""
    insts = synth.stars64(seed=0)
    B = gcr.Batch([i.grid for i in insts], [i.shape for i in insts], [2] * len(insts))
    nf = 3
    fields, bcv, bct, xq, nr, wq, nqs = [], [], [], [], [], [], []
    ng = 0
    ncell = 0
    for inst, plan in zip(insts, B.plans):
        S, n = plan.foot_points()
        Sh, nh = S.cpu().numpy(), n.cpu().numpy()
        kk = [synth.mixed_kinds(Sh, inst.shape.center, b) for b in inst.mixed_beta]
        for f, k in zip(inst.fields, kk):
            fields.append(_dev(torch, synth.sample(f, inst.grid), torch.float64))
            bcv.append(_dev(torch, synth.bc_values(f, Sh, nh, k), torch.float64))
            bct.append(_dev(torch, k.astype(np.uint8)))
        q = inst.queries
        xq.append(_dev(torch, q.x))
        nr.append(_dev(torch, q.n))
        wq.append(_dev(torch, q.w))
        nqs.append(q.x.shape[1])
        ng += plan.n_ghost
        ncell += plan.n_cells
    F = torch.zeros((len(insts), 3), dtype=torch.float64, device="cuda")

    def batched():
        B.forward(nf, fields, [MIXED] * nf, bcv, bc_type=bct, nq=nqs, xq=xq, nrm=nr, wq=wq,
                  p_field=2, u_first=0, mu=1.0, F=F)

    for _ in range(3):          # the tuner settles on its first calls
        batched()
    torch.cuda.synchronize()
    tb, _ = _time(torch, batched, reps)
    for p in B.plans:
        p.set_schedule(1)

    def plain():
        for i, p in enumerate(B.plans):
            fs = fields[i * nf:(i + 1) * nf]
            p.fill(fs, [MIXED] * nf, bcv[i * nf:(i + 1) * nf], bc_type=bct[i * nf:(i + 1) * nf])
            p.forces(xq[i], nr[i], wq[i], fs[2], fs[:2], 1.0, out=F[i])

    tp, _ = _time(torch, plain, reps)
    return {"workload": "stars64: 64 2D star bodies, n ~ U{128..2048}, 3 fields mixed BC, HGC, "
                        "fill + force per instance",
            "instances": len(insts), "cells": ncell, "ghosts": ng, "fields": nf,
            "batched_ms": round(tb, 4), "plain_ms": round(tp, 4),
            "batched_ghost_cells_per_s": round(ng / (tb * 1e-3), 1),
            "plain_ghost_cells_per_s": round(ng / (tp * 1e-3), 1),
            "speedup_vs_plain": round(tp / tb, 3)}


def bench_fwd_bwd(gcr, torch, synth, reps):
    """384^3 spherical-harmonic star, HGC, u, v, w, p: forward (fill + drag)
    and forward + reverse-level adjoint (d drag / d interior field and
    boundary data).  The dense zero-fill of the gradient buffers is timed
    on its own and kept out of the adjoint figure."""
    inst = synth.shstar384(seed=0)
    plan = gcr.Plan(inst.grid, inst.shape, 2)
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

    def bwd():
        plan.forces_adjoint(xq, nr, wq, 1.0, gF, lam[3], lam[:3])
        plan.fill_adjoint(lam, kinds, lam_bc)

    def zero():
        for t in lam:
            t.zero_()

    def fwd_bwd():
        fwd()
        bwd()

    tf, _ = _time(torch, fwd, reps)
    # the adjoint accumulates into lam: zero it between timed calls, outside
    # the timed region
    ts = []
    for _ in range(reps + 1):
        zero()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fwd_bwd()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    tfb = float(np.median(ts[1:]))
    tz, _ = _time(torch, zero, reps)
    ng = plan.n_ghost
    return {"workload": "shstar384: 384^3 grid on [-1,1]^3, SH star (l=2..4), u,v,w Dirichlet + "
                        "p Neumann, HGC, fill + drag, then adjoint of drag",
            "cells": plan.n_cells, "ghosts": ng, "fields": nf, "levels": plan.n_levels,
            "fwd_ms": round(tf, 4), "fwd_bwd_ms": round(tfb, 4),
            "fwd_bwd_over_fwd": round(tfb / tf, 3),
            "fwd_ghost_cells_per_s": round(ng / (tf * 1e-3), 1),
            "fwd_bwd_ghost_cells_per_s": round(ng / (tfb * 1e-3), 1),
            "dense_grad_zero_ms": round(tz, 4)}


def bench_layer2(gcr, torch, synth, reps):
    """The headline sphere with a second ghost layer (HGC | LAYER2): plan,
    boundary data, fill of u, v, w, p and force, one plan at a time, beside
    the same step with HGC alone."""
    inst = synth.sphere256(seed=0)
    g = inst.grid
    dev = torch.device("cuda")
    fields = [_dev(torch, synth.sample(f, g), torch.float64) for f in inst.fields]
    kinds = [DIRICHLET, DIRICHLET, DIRICHLET, NEUMANN]
    q = inst.queries
    xq, nq, wq = (_dev(torch, a) for a in (q.x, q.n, q.w))
    F = torch.empty(3, dtype=torch.float64, device=dev)
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

        t, _ = _time(torch, step, reps)
        out[name] = {"ghosts": info["ghosts"], "levels": info["levels"], "step_ms": round(t, 4),
                     "ghost_cells_per_s": round(info["ghosts"] / (t * 1e-3), 1)}
    return out


def bench_moving(gcr, torch, synth, reps):
    """The headline sphere moving by 0.4 h per step (HGC with a second ghost
    layer, so that the cells the move exposes were ghosts before): per step
    a new plan at the new position, its fresh cells against the previous
    plan, boundary data, fill of u, v, w, p and force.  Every step's fresh
    cells must all be covered."""
    import numpy as np
    inst = synth.sphere256(seed=0)
    g, h = inst.grid, inst.grid.h[0]
    dev = torch.device("cuda")
    fields = [_dev(torch, synth.sample(f, g), torch.float64) for f in inst.fields]
    kinds = [DIRICHLET, DIRICHLET, DIRICHLET, NEUMANN]
    q = inst.queries
    xq, nq, wq = (_dev(torch, a) for a in (q.x, q.n, q.w))
    F = torch.empty(3, dtype=torch.float64, device=dev)
    step_v = 0.4 * h * np.array([0.8, 0.48, 0.36])   # |v| = 0.4 h
    state = {"k": 0, "prev": None, "counts": []}

    def step():
        k = state["k"]
        state["k"] += 1
        c = tuple(float(x) for x in np.asarray(inst.shape.center) + k * step_v)
        plan = gcr.Plan(g, synth.Shape(inst.shape.kind, c, inst.shape.r0), 2 | 4)
        if state["prev"] is not None:
            _, counts = state["prev"].fresh_cells(plan)
            state["counts"].append(counts)
        S, nrm = plan.foot_points()
        plan.fill(fields, kinds, list(bc_sphere_fields(S, nrm)))
        plan.forces(xq, nq, wq, fields[3], fields[:3], 1.0, out=F)
        state["prev"] = plan

    t, _ = _time(torch, step, reps)
    counts = torch.stack(state["counts"]).cpu().numpy()
    return {"workload": "sphere256 moving 0.4 h per step, HGC with a second ghost layer: "
                        "plan at the new position + fresh cells against the previous plan + "
                        "fill of u,v,w,p + force",
            "step_ms": round(t, 4), "fresh_per_step": int(counts[:, 0].mean()),
            "uncovered_total": int(counts[:, 1].sum()), "steps_checked": int(len(counts))}


def bench_large(gcr, torch, synth, reps):
    """The sphere of the headline workload on a 1024^3 grid (1.07e9 cells):
    the size at which the classification pass (1 byte per cell written)
    is bandwidth-scale.  HGC plan, fill of u, v, w, p, force; fields are
    generated on the device."""
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

    def step():
        plan = gcr.Plan(g, inst.shape, 2)
        times = gcr.last_build_times()
        times["band_segments"] = plan.stats()["n_band_segments"]
        S, nrm = plan.foot_points()
        plan.fill(fields, kinds, list(bc_sphere_fields(S, nrm)))
        plan.forces(xq, nq, wq, fields[3], fields[:3], 1.0, out=F)
        return plan.n_ghost, times

    gcr.set_profiling(True)
    step()
    torch.cuda.synchronize()
    ts, cls = [], []
    ng = 0
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        ng, times = step()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
        cls.append(times["classify_store"])
        nseg = times["band_segments"]
    gcr.set_profiling(False)
    t = float(np.median(ts))
    c = float(np.median(cls))
    ncell = g.n[0] * g.n[1] * g.n[2]
    cbytes = ncell - 16 * nseg

    # the same step as a batch of one: its forward (fill + surface + force
    # in one launch) with the launch shape the tuner picks (for one large
    # instance, a split sweep: many workgroups share each level), and with
    # the per-item sweep (one workgroup per field) forced, for comparison
    F2 = torch.zeros((1, 3), dtype=torch.float64, device=dev)
    nqp = q.x.shape[1]
    sv = [torch.empty(nqp, dtype=torch.float64, device=dev) for _ in range(4)]

    def bstep(shape):
        B = gcr.Batch([g], [inst.shape], [2])
        S, nrm = B.foot_points()
        bcv = list(bc_sphere_fields(S, nrm))
        gcr.set_batch_shape(*shape)
        try:
            B.forward(4, fields, kinds, bcv, nq=[nqp], xq=[xq], nrm=[nq], wq=[wq], p_field=3,
                      u_first=0, mu=1.0, F=F2, sval=sv)
        finally:
            gcr.set_batch_shape(0, 0)
        return B

    batched = {}
    for name, shape in (("tuned", (0, 0)), ("per_item", (1024, 1))):
        bstep(shape)
        torch.cuda.synchronize()
        gcr.set_profiling(gcr.PROFILE_FORWARD)
        gcr.forward_times()
        bt = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            bstep(shape)
            b.record()
            torch.cuda.synchronize()
            bt.append(a.elapsed_time(b))
        ft = gcr.forward_times()
        gcr.set_profiling(False)
        batched[name] = {"step_ms": round(float(np.median(bt)), 4),
                         "forward_kernel_ms": round(ft["forward"], 4)}
    del fields
    torch.cuda.empty_cache()
    return {"workload": "sphere1024: 1024^3 grid on [-1,1]^3, the headline sphere, HGC, "
                        "plan + fill of u,v,w,p + force",
            "cells": ncell, "ghosts": ng, "step_ms": round(t, 4),
            "ghost_cells_per_s": round(ng / (t * 1e-3), 1),
            "classify_store_ms": round(c, 5),
            "as_batch_of_one": batched,
            "classify_roofline": {"bound": "hbm", "kernel": "k_classify",
                                  "achieved": round(cbytes / (c * 1e-3) / 1e9, 2),
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(cbytes / (c * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "algorithmic_bytes": cbytes}}


def cpu_baseline(inst, seconds):
    """The oracle, as it stands, on the same workload (full size): passes
    over the three schemes until `seconds` of oracle time are spent (at
    least one); threads = OpenMP threads of its per-cell loops."""
    import oracle
    import synth

    grid = inst.grid
    vals = np.stack([synth.sample(f, grid) for f in inst.fields])
    kinds = [DIRICHLET, DIRICHLET, DIRICHLET, NEUMANN]
    q = inst.queries
    ng_total = 0
    t = 0.0
    passes = 0
    while passes == 0 or t < seconds:
        for sch in SCHEMES:
            t0 = time.perf_counter()
            p = oracle.OraclePlan(grid, inst.shape, sch)
            t += time.perf_counter() - t0
            c = p.ghost_cell
            idx = [c % grid.n[0], (c // grid.n[0]) % grid.n[1], c // (grid.n[0] * grid.n[1])]
            S = np.stack([grid.lo[i] + (idx[i] + 0.5) * grid.h[i] for i in range(3)]) + p.delta
            b = np.stack([synth.bc_values(f, S, p.normal, k) for f, k in zip(inst.fields, kinds)])
            t0 = time.perf_counter()
            out = p.fill(vals, kinds, b)
            p.surface_query(q.x, out)
            p.forces(q.x, q.n, q.w, out[3], out[:3], 1.0)
            t += time.perf_counter() - t0
            ng_total += p.n_ghost
        passes += 1
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(ng_total / t, 1), "unit": "ghost cells/s", "cores": cores,
            "kind": "oracle", "sample": f"full sphere256 workload, {passes} passes x 3 schemes "
                                        f"({t:.1f} s of oracle time)"}


if __name__ == "__main__":
    main()
