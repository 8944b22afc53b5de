"""Benchmark: occupancy-grid ray sampling on one MI355X.

One step = one full sampling pass of the VDB + hierarchical-DDA sampler over
the 800x800-ray object-scene workload (128^3 grid, 6 % occupied): per-ray
counts, their exclusive scan, and the fill of the packed (ray id, t0, t1)
samples, inputs resident in HBM.  The dense-grid DDA marcher (the plain
method) is timed with the same protocol on the same rays.  `value` is the
VDB sampler's rays/s over K back-to-back steps with three batches in flight
(consecutive steps take turns on three streams, each with its own workspace
and outputs; `pipelined`); `latency` holds the same call timed
step by step on one stream, which the rooflines use.  --primary-only and
--no-pipeline time the single stream only (then `value` is its rate).

Prints one JSON line.  `roofline` divides the call's algorithmic bytes
(24 B per ray read, 8 B per offset and 12 B per sample written, the grid read
once) by the summed durations of its kernels, measured with HIP events on the
stream they run on, and splits both by kernel (`per_kernel`: the walk owns the
rays and the grid, the expansion the offsets and samples).  `cpu_baseline`
times the CPU oracle (dense DDA and VDB + hierarchical DDA) on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/s + samples/s, VDB+HDDA vs dense-OG march, 800×800 rays, sample-exact"
# comparison samplers on the headline workload: the other loop of the VDB walk,
# row-major lanes, the dense march (the plain method) in both loops and with
# row-major lanes, the chessboard-distance march, the VDB walked voxel by voxel
# in both loops, and the VDB walk with sub-leaf steps
VARIANTS = ["vdb_other", "vdb_rows", "dense", "dense_skip", "dense_rows", "chessboard", "voxel", "voxel_other",
            "subleaf"]
HBM_PEAK_GBS = 8000.0
# batches in flight for the whole-job figures (streams of the default priority): three measured
# 0.199-0.200 ms a step on the object workload, two 0.210-0.218, four 0.211
IN_FLIGHT = 3
# MI355X: 256 CUs x 4 SIMDs at 2.4 GHz; a 64-lane wave's VALU instruction
# takes 4 clocks on a 16-lane SIMD
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--variant", default="branch", choices=["skip", "branch"],
                   help="loop structure of the timed VDB sampler (Alg. 1 branch / Alg. 2 skip)")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    p.add_argument("--cpu-stride", type=int, default=1, help="oracle baseline uses every k-th object-scene ray")
    p.add_argument("--no-side", action="store_true", help="skip the composite and batched side measurements")
    p.add_argument("--primary-only", action="store_true",
                   help="time only the headline VDB step (no variant or dense comparisons; for profiling)")
    p.add_argument("--variants", default=",".join(VARIANTS),
                   help="comma list of the comparison samplers to time beside the headline (default: all of "
                        + ", ".join(VARIANTS) + ")")
    p.add_argument("--no-pipeline", action="store_true",
                   help="time the headline on one stream only (no whole-job figure with batches in flight)")
    p.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                   help="first run a plain device copy of MIB MiB (3 times), to calibrate HBM byte counters")
    return p.parse_args()


def copy_calibration(mib):
    """A plain copy kernel of known size: FETCH_SIZE / WRITE_SIZE read on it
    give the factor from counter units to HBM bytes."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "launches": 3}), flush=True)


class Timed:
    """One sampling pass of one grid: the one-call path (ogv_sample_rays:
    the walk, then one launch that scans and fills) is the step; the
    three-call path (count_raw, scan, fill) is timed beside it for the split
    into walk, scan and fill.  Events on the launch stream."""

    def __init__(self, api, torch, grid, w, o, d, variant, image_width=0):
        self.torch = torch
        self.sp = api.Sampler(grid, w.n_rays, w.near, w.far, w.step, variant, image_width=image_width)
        self.o, self.d = o, d
        self.sp.count(o, d)
        torch.cuda.synchronize()
        self.S = int(self.sp.offsets[w.n_rays].item())
        self.ids = torch.empty(self.S, dtype=torch.int32, device="cuda")
        self.t0 = torch.empty(self.S, dtype=torch.float32, device="cuda")
        self.t1 = torch.empty(self.S, dtype=torch.float32, device="cuda")

    def step(self, ev=None):
        # one call: walk (pool reset + count kernel, which also sums the scan
        # tiles and chunks), then the expansion, which scans and fills
        if ev is not None:
            ev[0].record()
        self.sp.rays(self.o, self.d, self.ids, self.t0, self.t1)
        if ev is not None:
            ev[1].record()

    def step3(self, ev):
        # three calls: walk, scan (one apply launch), fill (expansion)
        ev[0].record()
        self.sp.count_raw(self.o, self.d)
        ev[1].record()
        self.sp.scan()
        ev[2].record()
        self.sp.fill(self.o, self.d, self.ids, self.t0, self.t1)
        ev[3].record()

    def run(self, steps, warmup):
        """(ms per one-call step, walk ms, scan ms, fill ms of the three-call
        path), events on the current stream."""
        torch = self.torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for k in range(steps):
            self.step(evs[k])
        end.record()
        torch.cuda.synchronize()
        total_ms = start.elapsed_time(end)
        per = sorted(e[0].elapsed_time(e[1]) for e in evs)   # each step alone
        self.step_stats = {"median_ms": per[len(per) // 2], "min_ms": per[0],
                           "p90_ms": per[min(len(per) - 1, (9 * len(per)) // 10)]}
        for _ in range(warmup):
            self.step3([torch.cuda.Event(enable_timing=True) for _ in range(4)])
        torch.cuda.synchronize()
        ev3 = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for k in range(steps):
            self.step3(ev3[k])
        b.record()
        torch.cuda.synchronize()
        self.three_call_ms = a.elapsed_time(b) / steps
        stage = [sum(e[i].elapsed_time(e[i + 1]) for e in ev3) / steps for i in range(3)]
        return total_ms / steps, stage[0], stage[1], stage[2]


_EXTRA_STREAMS = []


def extra_streams(torch, n):
    """n streams of the default priority besides the current one, created once
    and reused by every phase that keeps batches in flight, so each phase runs
    on the same hardware queues (streams map onto a few hardware queues in
    creation order, and one that shares the current stream's queue is
    serialized behind it)."""
    while len(_EXTRA_STREAMS) < n:
        _EXTRA_STREAMS.append(torch.cuda.Stream())
    return _EXTRA_STREAMS[:n]


def pipelined(api, torch, grid, w, o, d, variant, image_width, ref, steps, warmup, n_streams=2):
    """Whole-job throughput with n_streams batches in flight: consecutive
    steps alternate between n_streams streams of the default priority, each
    with its own sampler workspace and outputs, so one step's expansion
    (bound by HBM writes) runs during the next step's walk (bound by issue
    and latency, with a drain that leaves most of the chip idle).  Every step
    is a whole one-call pass over the whole batch.  Events on the current
    stream bracket all steps: the other streams wait for the start event and
    the current stream waits for their last step before the end event.
    Returns ms per step; every stream's offsets and samples must equal ref's
    (the single-stream headline call's)."""
    cur = torch.cuda.current_stream()
    streams = [cur] + extra_streams(torch, n_streams - 1)
    ts = [Timed(api, torch, grid, w, o, d, variant, image_width) for _ in range(n_streams)]

    def go(k):
        j = k % n_streams
        with torch.cuda.stream(streams[j]):
            ts[j].sp.rays(o, d, ts[j].ids, ts[j].t0, ts[j].t1, stream=streams[j])

    for k in range(warmup * n_streams):
        go(k)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(cur)
    for s in streams[1:]:
        s.wait_event(start)
    for k in range(steps):
        go(k)
    for s in streams[1:]:
        e = torch.cuda.Event()
        e.record(s)
        cur.wait_event(e)
    end.record(cur)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    for t in ts:
        same = t.S == ref.S and torch.equal(t.sp.offsets, ref.sp.offsets) and torch.equal(t.ids, ref.ids) \
            and torch.equal(t.t0, ref.t0) and torch.equal(t.t1, ref.t1)
        assert same, "a pipelined stream's samples differ from the single-stream call's"
    return ms


def time_events(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def composite_side(api, torch, scenes, hdda, N, steps):
    """Fused composite forward and backward over the step's packed samples
    (sigma ~ exp(N(0,1)), rgb ~ U[0,1]^3 per sample)."""
    S = hdda.S
    sigma, rgb, _ = scenes.composite_inputs(S, N)
    sig = torch.from_numpy(sigma).cuda()
    col = torch.from_numpy(rgb).cuda()
    off = hdda.sp.offsets
    g_rgb = torch.ones((N, 3), device="cuda")
    g_a = torch.ones(N, device="cuda")
    fwd = time_events(torch, lambda: api.composite_forward(off, hdda.t0, hdda.t1, sig, col), steps, 2)
    bwd = time_events(torch, lambda: api.composite_backward(off, hdda.t0, hdda.t1, sig, col, g_rgb, g_a), steps, 2)
    # algorithmic bytes: each sample's t0, t1, sigma, rgb read once (24 B), offsets read,
    # per-ray rgb + opacity written (forward) or read as gradients (backward), and the
    # backward's d_sigma, d_rgb written (16 B per sample)
    fb = 24 * S + 8 * (N + 1) + 16 * N
    bb = 24 * S + 8 * (N + 1) + 16 * N + 16 * S
    return {"forward_ms": fwd, "backward_ms": bwd, "forward_GBps": fb / (fwd * 1e-3) / 1e9,
            "backward_GBps": bb / (bwd * 1e-3) / 1e9, "samples": S}


def cascades_side(api, torch, scenes, steps, warmup, pipe=True):
    """Four nested 128^3 cascades over [-2^k, 2^k]^3, growing step (cone 1/256,
    dt_min 1e-3, near 0.05, far 1e3), 1280x832 rays from inside the scene:
    count + scan + fill with the VDB + hierarchical DDA and with the dense march,
    each also with IN_FLIGHT batches in flight (`pipelined`) unless pipe is false."""
    w = scenes.workload("unbounded")
    occ = torch.from_numpy(w.occ).cuda()
    o = torch.from_numpy(w.origins).cuda()
    d = torch.from_numpy(w.dirs).cuda()
    out = {"rays": w.n_rays, "levels": int(w.occ.shape[0])}
    vdb = api.build_vdb(occ, w.boxes, w.ilog2)
    dense = api.build_dense(occ, w.boxes)
    ref = None
    for name, grid, variant in (("vdb", vdb, "branch"), ("vdb_subleaf", vdb, "subleaf_branch"),
                                ("dense", dense, "branch")):
        t = Timed(api, torch, grid, w, o, d, variant, w.image[0])
        ms, walk, scan, fill = t.run(steps, warmup)
        N, S, G = w.n_rays, t.S, grid.info()["bytes"]
        step_bytes = 24 * N + 8 * (N + 1) + 12 * S + G   # the call's inputs and outputs, as for the headline
        out[name] = {"ms_per_step": ms, "walk_ms": walk, "scan_fill_ms": ms - walk,
                     "three_call": {"ms_per_step": t.three_call_ms, "scan_ms": scan, "fill_ms": fill},
                     "rays_per_s": N / (ms * 1e-3), "samples_per_s": S / (ms * 1e-3), "samples": S,
                     "step_hbm_frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if ref is None:
            ref = t
        del t
    if pipe:
        pv = pipelined(api, torch, vdb, w, o, d, "branch", w.image[0], ref, steps, warmup, IN_FLIGHT)
        pd = pipelined(api, torch, dense, w, o, d, "branch", w.image[0], ref, steps, warmup, IN_FLIGHT)
        out["pipelined"] = {"streams": IN_FLIGHT, "ms_per_step": pv, "rays_per_s": w.n_rays / (pv * 1e-3),
                            "dense_ms_per_step": pd, "dense_rays_per_s": w.n_rays / (pd * 1e-3),
                            "speedup_vs_dense": pd / pv}
    del ref
    out["speedup_vs_dense"] = out["dense"]["ms_per_step"] / out["vdb"]["ms_per_step"]
    out["subleaf_speedup_vs_dense"] = out["dense"]["ms_per_step"] / out["vdb_subleaf"]["ms_per_step"]
    return out


def cameras_side(api, torch, scenes, w, vdb, dense, variant, primary, steps, warmup):
    """The object grid seen from four more seeded cameras (same grid, same
    lattice): the one-call step with the VDB + hierarchical DDA and with the
    dense march per view, and the medians over the five views (the primary
    one included).  primary: (vdb ms, dense ms, samples) of the headline view."""
    import numpy as np
    views = [{"seed": "primary", "vdb_ms": primary[0], "dense_ms": primary[1], "samples": primary[2]}]
    for seed, o_h, d_h in scenes.object_extra_cameras(4, *w.image):
        o = torch.from_numpy(o_h).cuda()
        d = torch.from_numpy(d_h).cuda()
        tv = Timed(api, torch, vdb, w, o, d, variant, w.image[0])
        td = Timed(api, torch, dense, w, o, d, "branch", w.image[0])
        assert tv.S == td.S, "samplers disagree on the sample count"
        views.append({"seed": seed, "vdb_ms": tv.run(steps, warmup)[0], "dense_ms": td.run(steps, warmup)[0],
                      "samples": tv.S})
        del tv, td
    N = w.n_rays
    for v in views:
        v["rays_per_s"] = N / (v["vdb_ms"] * 1e-3)
        v["samples_per_s"] = v["samples"] / (v["vdb_ms"] * 1e-3)
        v["speedup_vs_dense"] = v["dense_ms"] / v["vdb_ms"]
    med = lambda k: float(np.median([v[k] for v in views]))
    return {"views": views, "median_rays_per_s": med("rays_per_s"), "median_samples_per_s": med("samples_per_s"),
            "median_speedup_vs_dense": med("speedup_vs_dense"), "median_vdb_ms": med("vdb_ms"),
            "median_dense_ms": med("dense_ms")}


def render_side(api, torch, scenes, hdda, w, steps):
    """End-to-end frame on the 800x800 object workload: the sampler's step
    (count + scan + fill) then one fused pass that evaluates a 12-blob
    Gaussian field at every sample's midpoint and composites each ray.  The
    field stands in for a trained one (random parameters, no weights)."""
    blobs = scenes.blob_field()
    field = api.blob_field(*blobs)
    off = hdda.sp.offsets
    render = lambda: api.render_blobs(off, hdda.o, hdda.d, hdda.t0, hdda.t1, field)
    r_ms = time_events(torch, render, steps, 2)

    def frame():
        hdda.step()
        render()

    f_ms = time_events(torch, frame, steps, 2)
    S, N, K = hdda.S, w.n_rays, len(blobs[1])
    return {"blobs": K, "render_ms": r_ms, "frame_ms": f_ms, "frames_per_s": 1e3 / f_ms,
            "render_GBps": (8 * S + 24 * N + 8 * (N + 1) + 16 * N) / (r_ms * 1e-3) / 1e9,
            "samples": S}


def batched_side(api, torch, scenes, steps, pipe=True):
    """16 scenes (grids 64^3..256^3, 2-20 % occupied, 64^2..1024^2 rays):
    one graph-captured batched pass vs 16 sequential single-scene calls, and
    (unless pipe is false) two graph-captured passes in flight on two streams,
    each batch with its own workspace and outputs (`pipelined`)."""
    ws = scenes.batched()
    gs = []
    for w in ws:
        occ = torch.from_numpy(w.occ).cuda()
        gs.append((api.build_vdb(occ, w.boxes, w.ilog2), torch.from_numpy(w.origins).cuda(),
                   torch.from_numpy(w.dirs).cuda(), w.near, w.far, w.step, w.image[0]))
    batch = api.Batch(gs, "branch")
    info = batch.info()
    z = torch.zeros(1, dtype=torch.int32, device="cuda")
    zf = torch.zeros(1, device="cuda")
    batch.launch(z[:0], zf[:0], zf[:0], graph=False)
    torch.cuda.synchronize()
    S = int(batch.offsets[-1].item())
    ids = torch.empty(S, dtype=torch.int32, device="cuda")
    t0 = torch.empty(S, device="cuda")
    t1 = torch.empty(S, device="cuda")
    graph_ms = time_events(torch, lambda: batch.launch(ids, t0, t1, graph=True), steps, 2)
    eager_ms = time_events(torch, lambda: batch.launch(ids, t0, t1, graph=False), steps, 2)
    seq = []
    for g, o, d, near, far, step, width in gs:
        sp = api.Sampler(g, o.shape[0], near, far, step, "branch", image_width=width)
        sp.count(o, d)
        torch.cuda.synchronize()
        n = int(sp.offsets[-1].item())
        seq.append((sp, o, d, torch.empty(n, dtype=torch.int32, device="cuda"), torch.empty(n, device="cuda"),
                    torch.empty(n, device="cuda")))

    def sequential():
        for sp, o, d, i_, a_, b_ in seq:
            sp.rays(o, d, i_, a_, b_)

    seq_ms = time_events(torch, sequential, steps, 2)
    N = info["n_rays"]
    pipelined_rec = None
    if pipe:
        b2 = api.Batch(gs, "branch", tune=(info["chunk"], info["blocks_per_cu"]))
        out2 = (torch.empty(S, dtype=torch.int32, device="cuda"), torch.empty(S, device="cuda"),
                torch.empty(S, device="cuda"))
        cur = torch.cuda.current_stream()
        streams = [cur] + extra_streams(torch, 1)
        runs = [(batch, (ids, t0, t1)), (b2, out2)]

        def go(k):
            j = k % 2
            with torch.cuda.stream(streams[j]):
                runs[j][0].launch(*runs[j][1], graph=True, stream=streams[j])

        for k in range(4):
            go(k)
        torch.cuda.synchronize()
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(cur)
        streams[1].wait_event(a)
        for k in range(2 * steps):
            go(k)
        last = torch.cuda.Event()
        last.record(streams[1])
        cur.wait_event(last)
        e.record(cur)
        torch.cuda.synchronize()
        pms = a.elapsed_time(e) / (2 * steps)
        assert torch.equal(batch.offsets, b2.offsets) and all(torch.equal(x, y) for x, y in zip((ids, t0, t1), out2)), \
            "the two in-flight batched passes disagree"
        pipelined_rec = {"streams": 2, "ms_per_pass": pms, "rays_per_s": N / (pms * 1e-3),
                         "speedup_vs_sequential": seq_ms / pms}
        b2.close()
    return {"scenes": len(ws), "rays": N, "samples": S, "graph_ms": graph_ms, "eager_ms": eager_ms,
            "pipelined": pipelined_rec,
            "sequential_ms": seq_ms, "rays_per_s": N / (graph_ms * 1e-3),
            "sequential_rays_per_s": N / (seq_ms * 1e-3), "speedup_vs_sequential": seq_ms / graph_ms,
            "tune": {"chunk": info["chunk"], "blocks_per_cu": info["blocks_per_cu"], "tuned": info["tuned"]}}


def host_threads():
    """Threads the oracle may use: the CPUs this process may run on, at most
    16 (the host share that goes with one GPU of the box; more threads than
    that share would only time-slice)."""
    try:
        n = len(os.sched_getaffinity(0))
    except Exception:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _median3(fn):
    ts, out = [], None
    for _ in range(3):
        t = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t)
    return sorted(ts)[1], out


def hbm_floor(torch, S, steps):
    """The box's practical HBM rates for the fill's traffic, with torch's own
    kernels: a write-only fill of three S-element float arrays (the 12 B per
    sample the expansion writes) and a device-to-device copy of as many bytes
    (read + write).  The write-only time is the floor under the expansion."""
    a = [torch.empty(S, dtype=torch.float32, device="cuda") for _ in range(3)]

    def fill():
        for x in a:
            x.fill_(1.0)

    fill_ms = time_events(torch, fill, steps, 2)
    src = torch.ones(3 * S, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    copy_ms = time_events(torch, lambda: dst.copy_(src), steps, 2)
    B = 12 * S
    return {"bytes_written": B, "write_only_ms": fill_ms, "write_only_GBps": B / (fill_ms * 1e-3) / 1e9,
            "copy_ms": copy_ms, "copy_GBps": 2 * B / (copy_ms * 1e-3) / 1e9}


def refresh_side(api, torch, scenes, steps):
    """In-place VDB refresh at 128^3 (the object grid) and 256^3 (the same
    grid upsampled twofold): the full re-classify from a uint8 occupancy, and
    the density-cache refresh (threshold fused into the classification) on
    its two paths -- bits changed only inside leaves (the tree keeps its
    numbering; the changed leaves are rewritten) and block kinds changed (the
    tree is renumbered).  Each call alternates between two densities that
    differ in that way, with decay 0, so every call changes the grid."""
    import numpy as np
    w = scenes.workload("object")
    rng = np.random.default_rng(9100)
    out = {}
    for R in (128, 256):
        occ = w.occ if R == 128 else np.repeat(np.repeat(np.repeat(w.occ, 2, 1), 2, 2), 2, 3)
        occ = np.ascontiguousarray(occ)
        dens = np.where(occ > 0, rng.uniform(2.0, 20.0, occ.shape), rng.uniform(0.0, 0.9, occ.shape))
        a = dens.astype(np.float32)
        # b: one occupied voxel cleared in 200 mixed blocks holding at least two (kinds unchanged)
        L = occ.shape[0]
        cnt = occ.reshape(L, R // 8, 8, R // 8, 8, R // 8, 8).sum(axis=(2, 4, 6))
        cand = np.argwhere((cnt >= 2) & (cnt < 512))
        b = a.copy()
        for l, bx, by, bz in cand[rng.choice(len(cand), 200, replace=False)]:
            i, j, k = np.argwhere(occ[l, 8 * bx:8 * bx + 8, 8 * by:8 * by + 8, 8 * bz:8 * bz + 8])[0]
            b[l, 8 * bx + i, 8 * by + j, 8 * bz + k] = 0.0
        c = a.copy()
        c[:, : R // 4] = 0.0                      # a quarter of the grid emptied: leaves and tiles change
        occ_d = torch.from_numpy(occ).cuda()
        g = api.build_vdb(occ_d, w.boxes, w.ilog2)
        cache = torch.from_numpy(a).cuda()
        A, B, C = (torch.from_numpy(x).cuda() for x in (a, b, c))
        changed = torch.zeros(2, dtype=torch.int32, device="cuda")
        state = {"i": 0}

        def alternate(x, y):
            def f():
                state["i"] += 1
                g.refresh_density(cache, x if state["i"] % 2 else y, 0.0, 1.0, changed)
            return f

        rec = {"voxels": int(occ.size), "full_reclassify_uint8_ms": time_events(torch, lambda: g.refresh(occ_d), steps, 2)}
        rec["density_leaves_only_ms"] = time_events(torch, alternate(A, B), steps, 2)
        torch.cuda.synchronize()
        rec["leaves_only_changed"] = changed.cpu().tolist()
        rec["density_structure_ms"] = time_events(torch, alternate(A, C), steps, 2)
        torch.cuda.synchronize()
        rec["structure_changed"] = changed.cpu().tolist()
        rec["density_threshold_only_ms"] = time_events(
            torch, lambda: g.refresh_density(cache, None, 0.0, 1.0, changed), steps, 2)
        out[f"{R}^3"] = rec
        del g, cache, A, B, C, occ_d
    return out


def cpu_baseline(obj_stride=1, unb_stride=2):
    """The oracle as it stands (count + fill of every ray, OpenMP over rays),
    timed on the host cores: the plain dense DDA (O2) and the VDB +
    hierarchical DDA (O3), both in the Alg. 1 loop the GPU bench times, on
    the object workload (every `obj_stride`-th ray), the four-cascade
    workload (every `unb_stride`-th ray) and the 16-scene batch (O2 on one
    ray in 4 of each scene, O3 on one in 32), each the median of 3 runs; O3 and O2 on one
    thread over every 64th object ray; brute force (O1) on all of the 64x64
    small workload and a seeded 4,096-ray subset of the object workload.
    `value` is O3 on the object workload.  Also the cells per ray that the
    dense, hierarchical and sub-leaf walks visit."""
    import numpy as np
    import oracle
    from paper_2404_10272_amd import scenes
    threads = host_threads()
    methods = {}
    spent = 0.0

    def leg(name, ws, sel, method, nthreads, sample):
        # ws: the workloads the leg walks (one, or the batch's scenes); sel
        # picks each one's rays (a slice or an index array)
        nonlocal spent
        prepared = []
        for w in ws:
            scene = oracle.Scene(w.occ, w.boxes)
            if method.startswith("hdda"):
                scene.vdb(w.ilog2)   # built outside the timed region, as on the GPU
            prepared.append((w, scene, np.ascontiguousarray(w.origins[sel]), np.ascontiguousarray(w.dirs[sel])))

        def run():
            return sum(int(oracle.sample_rays(sc, o, d, w.near, w.far, w.step, method, ilog2=w.ilog2,
                                              threads=nthreads)["offsets"][-1]) for w, sc, o, d in prepared)

        med, S = _median3(run)
        spent += 3 * med
        n = sum(p[2].shape[0] for p in prepared)
        methods[name] = {"value": n / med, "unit": "rays/s", "median_s": med, "rays": n, "samples": S,
                         "threads": nthreads, "method": method, "sample": sample}

    every = lambda name, k: f"{name} workload, " + ("every ray" if k == 1 else f"one ray in {k}")
    obj = scenes.workload("object")
    leg("object_hdda", [obj], slice(None, None, obj_stride), "hdda_branch", threads, every("object", obj_stride))
    leg("object_dense_dda", [obj], slice(None, None, obj_stride), "dense_branch", threads,
        every("object", obj_stride))
    leg("object_hdda_1thread", [obj], slice(None, None, 64 * obj_stride), "hdda_branch", 1,
        every("object", 64 * obj_stride))
    leg("object_dense_dda_1thread", [obj], slice(None, None, 64 * obj_stride), "dense_branch", 1,
        every("object", 64 * obj_stride))
    pick = np.sort(np.random.default_rng(2000).choice(obj.n_rays, 4096, replace=False))
    leg("object_brute_force", [obj], pick, "brute", threads, "object workload, a seeded 4,096-ray subset")
    unb = scenes.workload("unbounded")
    leg("unbounded_hdda", [unb], slice(None, None, unb_stride), "hdda_branch", threads,
        every("unbounded", unb_stride))
    leg("unbounded_dense_dda", [unb], slice(None, None, unb_stride), "dense_branch", threads,
        every("unbounded", unb_stride))
    leg("small_brute_force", [scenes.workload("small")], slice(None), "brute", threads, "small workload, every ray")
    bat = scenes.batched()
    leg("batched_hdda", bat, slice(None, None, 32), "hdda_branch", threads,
        "16-scene batch, one ray in 32 of each scene")
    leg("batched_dense_dda", bat, slice(None, None, 4), "dense_branch", threads,
        "16-scene batch, one ray in 4 of each scene")
    # cells a ray's walk visits, per traversal (every 16th ray): what the walk
    # kernels' time scales with
    cells = {}
    for w in (obj, unb):
        scene = oracle.Scene(w.occ, w.boxes)
        o = np.ascontiguousarray(w.origins[::16])
        d = np.ascontiguousarray(w.dirs[::16])
        for m in ("dense_branch", "hdda_branch", "subleaf_branch"):
            c = oracle.cell_counts(scene, o, d, w.near, w.far, w.step, m, ilog2=w.ilog2, threads=threads)
            cells[f"{w.name}_{m}"] = {"mean": float(c.mean()), "max": int(c.max()), "rays": int(c.shape[0])}
    model = ""
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except Exception:
        pass
    head = methods["object_hdda"]
    return {"value": head["value"], "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"{head['sample']} ({head['rays']} rays, {head['samples']} samples), "
                      f"VDB + hierarchical DDA (Alg. 1 loop), count + fill, median of 3 runs on {threads} threads; "
                      f"{spent:.1f} s of oracle time over all legs",
            "methods": methods, "cells_per_ray": cells,
            "host": {"cpus": os.cpu_count(), "threads_allowed": threads, "model": model}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is a design "
                                   "note (rays split in contiguous ranges, grid replicated), not a measured path",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2404_10272_amd import api, scenes

    torch.cuda.set_device(0)
    if args.copy_calib:
        copy_calibration(args.copy_calib)
    w = scenes.workload("object")
    occ = torch.from_numpy(w.occ).cuda()
    o = torch.from_numpy(w.origins).cuda()
    d = torch.from_numpy(w.dirs).cuda()

    torch.cuda.synchronize()
    t = time.perf_counter()
    vdb = api.build_vdb(occ, w.boxes, w.ilog2)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t) * 1e3
    # second build, warm (the first pays module load)
    t = time.perf_counter()
    vdb2 = api.build_vdb(occ, w.boxes, w.ilog2)
    torch.cuda.synchronize()
    build_ms = min(build_ms, (time.perf_counter() - t) * 1e3)
    del vdb2
    dense = api.build_dense(occ, w.boxes)
    vinfo, dinfo = vdb.info(), dense.info()

    other = "skip" if args.variant == "branch" else "branch"
    W = w.image[0]
    hdda = Timed(api, torch, vdb, w, o, d, args.variant, W)
    ms, walk_ms, scan_ms, fill_ms = hdda.run(args.steps, args.warmup)
    # the Python wrapper end to end (count, the total read back to the host, outputs allocated, fill),
    # host wall clock: a secondary figure beside the event-timed call
    wall = []
    for _ in range(12):
        torch.cuda.synchronize()
        t = time.perf_counter()
        api.sample_rays(vdb, o, d, w.near, w.far, api.make_step(w.step), args.variant, image_width=W)
        torch.cuda.synchronize()
        wall.append((time.perf_counter() - t) * 1e3)
    wrapper_wall_ms = sorted(wall[2:])[len(wall[2:]) // 2]
    # in-place asynchronous refresh of the tree (same occupancy, so the grid is unchanged)
    refresh_ms = time_events(torch, lambda: vdb.refresh(occ), 10, 2)
    compare = {}
    want = set() if args.primary_only else set(v for v in args.variants.split(",") if v)
    unknown = want - set(VARIANTS)
    if unknown:
        raise SystemExit(f"unknown variants {sorted(unknown)}; choose from {VARIANTS}")
    if want:
        distg = api.build_dist(occ, w.boxes) if "chessboard" in want else None
        # (record name, grid, loop variant, lane layout); every sampler must find the headline's samples
        spec = {"vdb_other": ("vdb_" + other, vdb, other, W), "vdb_rows": ("vdb_row_major_lanes", vdb, args.variant, 0),
                "dense": ("dense", dense, "branch", W), "dense_skip": ("dense_skip", dense, "skip", W),
                "dense_rows": ("dense_row_major_lanes", dense, "branch", 0),
                "chessboard": ("chessboard", distg, "branch", W),
                "voxel": ("vdb_voxel_steps", vdb, "voxel_" + args.variant, W),
                "voxel_other": ("vdb_voxel_steps_" + other, vdb, "voxel_" + other, W),
                "subleaf": ("vdb_subleaf", vdb, "subleaf_" + args.variant, W)}
        timed = {v: Timed(api, torch, spec[v][1], w, o, d, spec[v][2], spec[v][3]) for v in VARIANTS if v in want}
        assert all(t.S == hdda.S for t in timed.values()), "samplers disagree on the sample count"
        N_ = w.n_rays

        def rec(t):
            tms, tw, ts, tf = t.run(args.steps, args.warmup)
            return {"ms_per_step": tms, "walk_ms": tw, "scan_fill_ms": tms - tw, "rays_per_s": N_ / (tms * 1e-3),
                    "three_call": {"ms_per_step": t.three_call_ms, "scan_ms": ts, "fill_ms": tf}}

        for v, t in timed.items():
            compare[spec[v][0]] = rec(t)
        if "dense" in compare:
            compare["dense"].update(bytes=dinfo["bytes"], variant="branch",
                                    samples_per_s=timed["dense"].S / (compare["dense"]["ms_per_step"] * 1e-3))
            compare["speedup_vs_dense"] = compare["dense"]["ms_per_step"] / ms
        if "chessboard" in compare:
            compare["chessboard"]["bytes"] = distg.info()["bytes"]
        del timed
    count_ms = walk_ms + scan_ms
    N, S = w.n_rays, hdda.S
    # whole-job throughput with IN_FLIGHT batches in flight, for the VDB sampler and
    # the dense march alike (both checked sample for sample against the headline)
    pipe = None
    if not (args.primary_only or args.no_pipeline):
        pv = pipelined(api, torch, vdb, w, o, d, args.variant, W, hdda, args.steps, args.warmup, IN_FLIGHT)
        pd = pipelined(api, torch, dense, w, o, d, "branch", W, hdda, args.steps, args.warmup, IN_FLIGHT)
        pipe = {"streams": IN_FLIGHT, "ms_per_step": pv, "rays_per_s": N / (pv * 1e-3), "samples_per_s": S / (pv * 1e-3),
                "dense_ms_per_step": pd, "dense_rays_per_s": N / (pd * 1e-3), "speedup_vs_dense": pd / pv,
                "single_stream_ms_per_step": ms, "gain_over_single_stream": ms / pv,
                "what": f"K back-to-back steps taking turns on {IN_FLIGHT} streams of the default priority, each "
                        "with its own workspace and outputs, bracketed by events; every step is a whole "
                        "one-call pass over all 640,000 rays"}
    value_ms = pipe["ms_per_step"] if pipe else ms
    G = vinfo["bytes"]
    # maximal lattice-contiguous runs (what the count kernel stores), from the
    # packed output, outside the timed region
    ids, t0, t1 = hdda.ids, hdda.t0, hdda.t1
    runs = int(1 + ((ids[1:] != ids[:-1]) | (t0[1:] != t1[:-1])).sum().item()) if S > 0 else 0
    # Algorithmic bytes of one call (what the method itself must move): rays
    # read (24 B each), offsets written (8 B each), samples written (12 B
    # each), the grid read once.  Split by kernel: the walk reads the rays and
    # the grid, the expansion writes offsets-indexed samples (and reads the
    # offsets); the scan moves only workspace.
    step_bytes = 24 * N + 8 * (N + 1) + 12 * S + G
    # the step's two launches (after the pool reset): the walk, and the
    # expansion that scans and fills; its time is the step's less the walk's
    scan_fill_ms = ms - walk_ms
    kern_bytes = {"count_kernel": 24 * N + G, "expand_kernel": 12 * S + 8 * (N + 1)}
    kern_ms = {"count_kernel": walk_ms, "expand_kernel": scan_fill_ms}
    # workspace traffic the two-pass design adds (not algorithmic): per-ray
    # counts, run counts and chain heads, 8 B per kept run (written, merged,
    # read back), the counts and sums the expansion's scan reads
    ws_bytes = {"count_kernel": 12 * N + 16 * runs, "expand_kernel": 8 * N + 8 * runs}
    sum_ms = ms
    achieved = step_bytes / (sum_ms * 1e-3) / 1e9

    counters = None
    issue = None
    tpath = os.path.join(ROOT, "profiles", "traffic_object800.json")
    if os.path.exists(tpath):
        try:
            rec = json.load(open(tpath))
            if rec.get("kernel_source_sha") == _kernel_sha():
                counters = rec.get("bytes_per_launch", {})
                issue = rec.get("issue_per_launch", {}).get("count_kernel")
        except Exception:
            counters = None
            issue = None
    per_kernel = {}
    for k in kern_bytes:
        b, t = kern_bytes[k], kern_ms[k]
        per_kernel[k] = {"algorithmic_bytes": b, "avg_ms": t, "achieved_GBps": b / (t * 1e-3) / 1e9,
                         "frac": b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, "workspace_bytes": ws_bytes[k]}
        if counters is not None:
            names = ["count_kernel", "pool_reset_kernel"] if k == "count_kernel" else [k]
            tr = sum(counters.get(n, 0.0) for n in names)
            per_kernel[k]["traffic"] = tr
            per_kernel[k]["traffic_over_algorithmic"] = tr / b if b else None
    traffic = sum(v.get("traffic", 0.0) for v in per_kernel.values()) if counters is not None else None
    if issue is not None:
        # the walk is bound by instruction issue, not HBM: its wave-level VALU
        # instructions per launch (SQ_INSTS_VALU of the committed counter run
        # of these sources) over its event-timed duration, against one VALU
        # instruction per SIMD every 4 clocks (a 64-lane wave on 16-lane SIMDs)
        v = issue["SQ_INSTS_VALU"]
        achieved_i = v / (walk_ms * 1e-3)
        per_kernel["count_kernel"]["issue"] = {
            "bound": "valu_issue", "valu_wave_insts": v, "achieved": achieved_i, "peak": VALU_ISSUE_PEAK,
            "unit": "wave instructions/s", "frac": achieved_i / VALU_ISSUE_PEAK,
            "lane_utilisation": issue["SQ_THREAD_CYCLES_VALU"] / (64.0 * issue["SQ_ACTIVE_INST_VALU"]),
            "salu_wave_insts": issue["SQ_INSTS_SALU"], "branch_wave_insts": issue["SQ_INSTS_BRANCH"]}

    line = {
        "metric": METRIC,
        "value": N / (value_ms * 1e-3),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": value_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded object-scene grid and cameras; no dataset)",
        "config": {"workload": "object-scene: 128^3 occupancy grid over [-1.5,1.5]^3 (6.0% occupied, "
                               "noise on 12 ellipsoid shells), 800x800 rays from radius 4, 40 deg FOV, "
                               "near 2, far 6, step 5e-3; VDB internal nodes 16^3 over 8^3 leaves",
                   "rays": N, "samples": S, "variant": args.variant, "lanes": "8x8 pixel tiles"},
        "samples_per_s": S / (value_ms * 1e-3),
        "pipelined": pipe,
        "latency": {"ms_per_step": ms, "rays_per_s": N / (ms * 1e-3), "step_stats": hdda.step_stats,
                    "what": "one stream, steps back to back with events around each (the rooflines use it)"},
        "paper_context": "end-to-end FPS with trained Instant-NGP fields on 1x NVIDIA A100, no sampler-only figure: "
                         "VDB + HDDA +12% over NerfAcc on NeRF-Synthetic (Tab. 1), +4% on Mip-NeRF 360 (Tab. 2); "
                         "context, not comparable (vs_baseline is null)",
        "vdb": {"ms_per_step": ms, "walk_ms": walk_ms, "scan_fill_ms": scan_fill_ms,
                "three_call": {"ms_per_step": hdda.three_call_ms, "walk_ms": walk_ms, "scan_ms": scan_ms,
                               "fill_ms": fill_ms, "count_scan_ms": count_ms},
                "rays_per_s": N / (ms * 1e-3),
                "bytes": G, "leaves": vinfo["n_leaves"], "build_ms": build_ms, "refresh_ms": refresh_ms,
                "wrapper_wall_ms": wrapper_wall_ms,
                "step_stats": hdda.step_stats},
        "step_bytes": step_bytes,
        "step_hbm_frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "runs": runs,
        "roofline": {"bound": "hbm", "kernel": "sampling call (ogv_sample_rays): count_kernel, then expand_kernel "
                                               "with the scan inside",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes": step_bytes,
                     "algorithmic_bytes_formula": "24N + 8(N+1) + 12S + G",
                     "avg_ms": sum_ms, "per_kernel": per_kernel,
                     "dominant_kernel": max(kern_ms, key=kern_ms.get),
                     "stages_ms": {"walk": walk_ms, "scan_and_fill": scan_fill_ms}},
    }
    pr = torch.cuda.get_device_properties(0)
    line["device"] = {k: getattr(pr, k, None) for k in (
        "name", "gcnArchName", "multi_processor_count", "warp_size", "total_memory", "L2_cache_size",
        "shared_memory_per_block", "regs_per_multiprocessor", "max_threads_per_multi_processor")}
    line["hbm_floor"] = hbm_floor(torch, S, min(args.steps, 20))
    line["hbm_floor"]["fill_vs_write_only"] = line["hbm_floor"]["write_only_ms"] / scan_fill_ms
    line.update(compare)
    if not args.no_side:
        dense_ms = compare["dense"]["ms_per_step"] if "dense" in compare else \
            Timed(api, torch, dense, w, o, d, "branch", W).run(min(args.steps, 20), 2)[0]
        line["cameras"] = cameras_side(api, torch, scenes, w, vdb, dense, args.variant, (ms, dense_ms, S),
                                       min(args.steps, 20), 2)
        line["composite"] = composite_side(api, torch, scenes, hdda, N, min(args.steps, 20))
        line["batched"] = batched_side(api, torch, scenes, min(args.steps, 10),
                                       pipe=not (args.primary_only or args.no_pipeline))
        line["cascades"] = cascades_side(api, torch, scenes, min(args.steps, 10), 2,
                                         pipe=not (args.primary_only or args.no_pipeline))
        line["render"] = render_side(api, torch, scenes, hdda, w, min(args.steps, 20))
        line["refresh"] = refresh_side(api, torch, scenes, min(args.steps, 20))
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_stride)
    print(json.dumps(line), flush=True)


def _kernel_sha():
    """Hash of what the step's kernels are built from: their sources and the
    build script that holds the compiler flags."""
    import hashlib
    h = hashlib.sha256()
    for f in ["csrc/sample.hip", "csrc/count.hpp", "csrc/trace.hpp", "csrc/geometry.hpp", "csrc/scan.hpp",
              "csrc/internal.hpp", "build.py"]:
        with open(os.path.join(ROOT, "paper_2404_10272_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
