"""Benchmark: forward + backward ms/iter and Gaussian-pixel evals/s of the
dilated rasterizer at 4K (3M Gaussians, SH degree 3, stride 2, offsets
cycling through the 4 phases), against the plain full-resolution path on the
same view.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline] [--no-plain]
                    [--no-batched | --only-batched] [--no-sweep | --only-sweep]
                    [--no-autograd | --only-autograd] [--no-order-study]

One step = preprocess -> pairs + sort + ranges -> dilated blend -> L1 loss
gradient against the full-resolution target -> blend backward -> preprocess
backward with densification statistics, on inputs already resident in HBM.
Prints ONE JSON line (diagnostics go to stderr).

Unless --no-sweep, it carries "sweep": per-stage ms, pair counts,
evaluation counts, rasterizer VALU fractions and workspace bytes of the same
scene at 1080p, 1440p and 4K at strides 1, 2 and 4 (the runtime breakdown
and memory against resolution).  Unless --no-order-study, it carries
"raster_fwd_tile_order_ms": the forward with a cold tile order (per-tile
weights zeroed, as on a fresh workspace) and with the warm order.

Unless --no-autograd, it carries "autograd": a training step through the
torch.autograd functions (1M Gaussians, 2560x1440, stride 2, fused Adam)
against the same step at stride 1.

Unless --no-batched, the JSON line also carries "batched": the 12-view batch
(2M Gaussians, views of mixed resolution and stride) stepped by the batched
calls and replayed from one captured graph, against the same views through
the single-view calls and against the plain full-resolution batch.

Gaussian-pixel evaluations: forward = list entries examined per rendered
pixel until its walk ends (stop entry included); backward = entries up to the
pixel's last blended one.  Both are counted by the kernels themselves
(per-pixel outputs checked against the CPU oracle in the tests).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12                    # B/s, MI355X HBM3E
# FP32 vector rate in lane operations, an FMA counted once: 256 CU x 4 SIMD x
# 16 lanes x 2.4 GHz = 39.3 T/s (78.6 TFLOP/s), one wave64 instruction per
# 4 cycles per SIMD without packed FP32 instructions, which this build does
# not use.  The published 157.3 TFLOP/s (78.65 T lane operations/s) counts
# packed FP32, two per lane and cycle, and is the bound; fractions against
# it are reported beside.  Hardware counters (profiles/) show the
# rasterizers issuing about one VALU instruction per 4 cycles per SIMD at
# the 4K d = 2 view and one per 3.3 cycles at 4K d = 1, so the 4-cycle rate
# is a reference, not a ceiling.
PEAK_VALU = 256 * 4 * 16 * 2.4e9
PEAK_VALU_PACKED = 157.3e12 / 2.0
# The least FP32 arithmetic the method needs per list entry and pixel (lane
# operations, an FMA counts 1; per-splat work such as scaling the conic or
# the per-splat skip threshold is not counted).
# Forward:
#   examined entry (up to the pixel's stop), decided for the pixel's
#   wavefront (8 x 8 threads of 1-4 pixels) at once by a bound on the
#   exponent over its pixel rectangle: 56 per entry and wavefront,
#   56 / (pixels of the wavefront) per pixel
#   tested entry (one the bound does not exclude, evaluated pixel by pixel):
#   offset 2, quadratic form 5, test of the exponent against the splat's
#   threshold 1                                                          -> 8
#   hit (alpha >= 1/255: the entry blends, or stops the pixel): exp 1,
#   opacity product 1, clamp 1, exact skip test 1, alpha T 1, T after the
#   entry 1, stop test 1                                                 -> 7
#   blended entry: colour accumulation 3                                 -> 3
# Backward (each pixel's blended entries, from the last back to the first;
# the forward records which entries a wavefront blended, so nothing else
# has to be evaluated):
#   blended entry: alpha at the pixel (offset 2, quadratic form 5, exp 1,
#   opacity product 1, clamp 1) 10; 1 - alpha, its reciprocal and T in
#   front 3; weight 1; dL/dC . rgb 3; d/dalpha against the colour behind and
#   its update 3; clamp test, d/dpower, d/do 3; d/d(u, v, A, B, C) 5 and
#   d/drgb 3 moments; the sums of the nine values over pixels 9        -> 40
# Hits are counted as blends plus one per rendered pixel (its stop, an upper
# bound).  Tested entries are counted by the counting forward (n_tested).
OPS_BOUND, OPS_EXAMINE, OPS_HIT, OPS_BLEND_FWD, OPS_BLEND_BWD = 56, 8, 7, 3, 40


def wave_pixels(tile=16):
    """Pixels of one rasterizer wavefront at the default launch of `tile`."""
    from paper_2412_13547_amd import api
    return 64 * api.default_launch(tile)[1]


def raster_labels(tile=16):
    """Kernel names of the default rasterizer launch of `tile`."""
    from paper_2412_13547_amd import api
    lds, ppt = api.default_launch(tile)
    return (f"raster_fwd_kernel<{tile},{ppt},{lds},false>", f"raster_bwd_kernel<{tile},{ppt},{lds}>")


def launch_ppt(tiles, tile=16):
    """Pixels per thread of the library's default launch of `tiles` tiles of
    16 x 16 (the rule tgs_default_launch documents)."""
    assert tile == 16
    return 4 if tiles >= 6144 else 2 if tiles >= 3072 else 1


def fwd_ops(evals, tested, blended, pixels, wpix):
    return (OPS_BOUND / wpix * evals + OPS_EXAMINE * tested + OPS_HIT * (blended + pixels)
            + OPS_BLEND_FWD * blended)


def bwd_ops(blended):
    return OPS_BLEND_BWD * blended
STAGES = ("preprocess_fwd", "bin_sort", "raster_fwd", "l1_grad", "raster_bwd", "preprocess_bwd")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--n", type=int, default=None, help="override the Gaussian count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB device copy (reference kernel for HBM counters)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 12-view batch (2M Gaussians, mixed resolutions and strides)")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the 12-view batch (for profiling); prints its own JSON")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--no-autograd", action="store_true",
                    help="skip the autograd training step (1M Gaussians, 1440p, stride 2)")
    ap.add_argument("--only-autograd", action="store_true",
                    help="run only the autograd training step; prints its own JSON")
    ap.add_argument("--lds-batch", type=int, default=0)
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the resolution x stride sweep (per-stage ms and workspace bytes)")
    ap.add_argument("--only-sweep", action="store_true",
                    help="run only the resolution x stride sweep; prints its own JSON")
    ap.add_argument("--no-order-study", action="store_true",
                    help="skip the cold vs warm tile-order forward timing (for profiling)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Runner:
    """One view of one scene: every buffer allocated once, steps reuse them."""

    def __init__(self, api, torch, dev, cam, target, stride, tile=16):
        self.api, self.torch, self.dev = api, torch, dev
        self.stride = stride
        self.ctx = api.Context(0)
        self.view = api.View(self.ctx, dev.n, cam, stride, 0, 0, tile)
        # size the workspace once (the pairs do not depend on the phase), then
        # step without reading the pair count back (the library's default)
        self.view.fit_capacity(dev)
        self.view.sync_check = False
        self.target = target
        n = dev.n
        self.grads = dev.zeros_like()
        self.pos = torch.empty(n, dtype=torch.float32, device="cuda")
        self.col = torch.empty(n, dtype=torch.float32, device="cuda")
        self.vis = torch.empty(n, dtype=torch.uint8, device="cuda")
        self.images = {}
        self.loss = torch.empty(1, dtype=torch.float64, device="cuda")

    def _bufs(self):
        shape = self.view.image_shape
        if shape not in self.images:
            t = self.torch
            self.images[shape] = (t.empty(shape, dtype=t.float32, device="cuda"),
                                  t.empty(shape, dtype=t.float32, device="cuda"))
        return self.images[shape]

    def _phase(self, k):
        from paper_2412_13547_amd import scenes
        ox, oy = scenes.phase_offsets(k, self.stride)
        v = self.view
        if (int(v.dil.off_x), int(v.dil.off_y)) != (ox, oy):
            v.set_offsets(ox, oy)

    def step(self, k, events=None):
        self._phase(k)
        v = self.view
        img, dL = self._bufs()
        rec = (lambda i: events[i].record()) if events else (lambda i: None)
        rec(0)
        v.preprocess_fwd(self.dev)
        rec(1)
        v.bin_sort(self.dev)
        rec(2)
        v.raster_fwd(img)
        rec(3)
        v.l1_grad(img, self.target, dL, self.loss)
        rec(4)
        v.raster_bwd(dL)
        rec(5)
        v.preprocess_bwd(self.dev, self.grads, self.pos, self.col, self.vis)
        rec(6)

    def counts(self, k):
        """Per-step sums of n_eval, last_contrib and n_blend, the pair count and
        the sum of n_tested for phase k (one counting forward of the view as a
        one-view batch, which carries the n_tested output)."""
        t = self.torch
        from paper_2412_13547_amd import scenes
        ox, oy = scenes.phase_offsets(k, self.stride)
        b = self.api.Batch(self.ctx, self.dev.n, [(self.view.cam, self.stride, ox, oy)], tile=16,
                           counts=True, pair_capacity=int(self.view.state.pair_capacity))
        b.fit_capacity(self.dev)
        b.forward(self.dev)
        t.cuda.synchronize()
        s = lambda x: int(x[0].sum(dtype=t.int64))
        res = (s(b.n_eval), s(b.last_contrib), s(b.n_blend), b.pair_counts()[0],
               s(b.n_tested))
        del b
        t.cuda.empty_cache()
        return res

    def forward_orders(self, reps=4):
        """Mean ms of raster_fwd with a cold tile order (tile_work zeroed, as on
        a fresh workspace) and with the warm order the cold forward left (the
        order every step after the first uses)."""
        t = self.torch
        v = self.view
        img, _ = self._bufs()
        cold, warm = [], []
        for k in range(reps):
            self._phase(k)
            v.preprocess_fwd(self.dev)
            v.bin_sort(self.dev)
            v.tile_work().zero_()
            ev = [t.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record()
            v.raster_fwd(img)
            ev[1].record()
            ev[2].record()
            v.raster_fwd(img)
            ev[3].record()
            t.cuda.synchronize()
            cold.append(ev[0].elapsed_time(ev[1]))
            warm.append(ev[2].elapsed_time(ev[3]))
        return statistics.mean(cold), statistics.mean(warm)

    def timed(self, steps, warmup):
        t = self.torch
        for k in range(warmup):
            self.step(k)
        t.cuda.synchronize()
        ev = [[t.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(steps)]
        t.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            self.step(warmup + k, ev[k])
        t.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_step = [e[0].elapsed_time(e[6]) for e in ev]
        stage = {s: statistics.mean([e[i].elapsed_time(e[i + 1]) for e in ev])
                 for i, s in enumerate(STAGES)}
        return wall, per_step, stage


def _oracle_tiles_worker(job):
    """One process of the CPU baseline: the oracle's blend forward and
    backward (float64) over its share of the sampled tiles, until the tiles
    or the time budget run out.  Returns (evaluations, tiles, seconds)."""
    import time as _time
    import torch
    torch.set_num_threads(1)
    from oracle import backward as obw
    from oracle import binning as obn
    from oracle import raster as ors
    (width, height, stride, tile), tiles, seconds = job
    g = obn.grid(width, height, stride, 0, 0, tile)
    evals = done = 0
    t0 = _time.perf_counter()
    for t, rec in tiles:
        if _time.perf_counter() - t0 >= seconds:
            break
        rec = {k: torch.as_tensor(v) for k, v in rec.items()}
        L = int(rec["u"].numel())
        vals = torch.arange(L)
        ranges = torch.zeros(g.num_tiles, 2, dtype=torch.int64)
        ranges[t] = torch.tensor([0, L])
        o = ors.raster_forward(rec, vals, ranges, g, tiles=[t])
        dl = torch.zeros(3, g.h_ds, g.w_ds, dtype=torch.float64)
        ii, jj, _, _ = ors.pixel_grid(g, t)
        dl[:, jj, ii] = 1.0 / dl.numel()
        obw.raster_backward(rec, vals, ranges, g, dl, tiles=[t])
        evals += int(o["n_eval"].sum()) + int(o["last_contrib"].sum())
        done += 1
    return evals, done, _time.perf_counter() - t0


def cpu_baseline(runner, seconds):
    """The CPU oracle beside the GPU (a baseline, not the target).

    value: the oracle's float64 blend forward + backward on a sample of random
    non-empty tiles of the benchmark view (phase (0,0)), fed the HIP path's
    records and tile lists, spread over min(os.cpu_count(), 12) processes of
    one thread each for about `seconds`; evaluations counted as in the metric.
    Beside it, the oracle's whole step (preprocess, binning, blend, L1 loss,
    backward, statistics) on the 1,024-Gaussian 128x128 scene in full."""
    import multiprocessing as mp
    import numpy as np
    import torch
    from oracle import pipeline as opipe
    from paper_2412_13547_amd import scenes
    v = runner.view
    v.set_offsets(0, 0)
    v.forward(runner.dev, runner._bufs()[0])
    torch.cuda.synchronize()
    r = v.records().cpu().to(torch.float64)
    vals = v.pair_vals().cpu().to(torch.int64)
    ranges = v.ranges().cpu().to(torch.int64)
    cam = v.cam
    # a worker's torch import opens the GPU device, and the machine counts
    # every process that holds it open: 12 workers stay well inside 16
    procs = max(1, min(os.cpu_count() or 1, 12))
    rng = np.random.default_rng(0)
    nonempty = np.nonzero((ranges[:, 1] - ranges[:, 0]).numpy() > 0)[0]
    picks = rng.choice(nonempty, min(len(nonempty), 150 * procs), replace=False)
    fields = dict(u=0, v=1, A=2, B=3, C=4, opacity=5)
    shares = [[] for _ in range(procs)]
    for k, t in enumerate(picks.tolist()):
        ids = vals[ranges[t, 0]:ranges[t, 1]]
        rr = r[ids]
        rec = {name: rr[:, c].numpy().copy() for name, c in fields.items()}
        rec["rgb"] = rr[:, 6:9].numpy().copy()
        shares[k % procs].append((t, rec))
    geom = (cam.width, cam.height, int(v.dil.stride), int(v.opt.tile))
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_oracle_tiles_worker, [(geom, sh, seconds) for sh in shares])
    evals = sum(e for e, _d, _s in res)
    tiles = sum(d for _e, d, _s in res)
    wall = max(s_ for _e, _d, s_ in res)
    # the whole oracle step on the small scene, in full
    sc0, cam0, tgt0 = scenes.workload(0)
    t0 = time.perf_counter()
    o = opipe.forward_backward(sc0, cam0, tgt0, 1, 0, 0, 16)
    el0 = time.perf_counter() - t0
    ev0 = int(o["n_eval"].sum()) + int(o["last_contrib"].sum())
    return {"value": evals / wall, "unit": "Gaussian-pixel evals/s", "cores": procs,
            "kind": "oracle",
            "sample": f"{tiles} random non-empty tiles of the 4K view at phase (0,0): float64 "
                      f"blend forward + backward of the oracle on the HIP path's records and "
                      f"lists, {procs} processes x 1 thread, {wall:.1f} s; evals counted as in "
                      f"the metric",
            "whole_step_small_scene": {"workload": scenes.WORKLOADS[0]["name"],
                                       "seconds": el0, "evals": ev0,
                                       "evals_per_s": ev0 / el0, "threads": torch.get_num_threads()}}


SWEEP_RESOLUTIONS = ((1920, 1080), (2560, 1440), (3840, 2160))
SWEEP_STRIDES = (1, 2, 4)


def run_sweep(args, api, torch, np, dev=None, steps=5, warmup=2):
    """Per-stage ms and memory against resolution and stride (the analogs of
    the paper's runtime breakdown, Fig. 1, and memory curve, Fig. 9): the 3M
    Gaussian scene of the benchmark seen from its camera angle at 1080p,
    1440p and 4K, each at strides 1, 2 and 4 (phases cycling)."""
    from paper_2412_13547_amd import scenes
    w = scenes.WORKLOADS[2]
    n = args.n or w["n"]
    if dev is None:
        dev = api.DeviceScene.from_scene(scenes.cluster_scene(2, n, w["sh_degree"]))
    angle = scenes.ring_angle(2002)
    rows = []
    for (W, H) in SWEEP_RESOLUTIONS:
        cam = scenes.ring_camera(W, H, angle)
        target = torch.as_tensor(scenes.target_image(W, H, 1002)).cuda()
        for d in SWEEP_STRIDES:
            r = Runner(api, torch, dev, cam, target, d)
            wall, per_step, stage = r.timed(steps, warmup)
            v = r.view
            pairs = r.view.pair_count()
            sz = v.sizes
            pix = int(sz.w_ds) * int(sz.h_ds)
            cap = int(v.state.pair_capacity)
            # evaluation counts of phase 0 (stage times average the phases)
            fe, be, bl, _, te = r.counts(0)
            tiles = int(sz.num_tiles)
            ppt = launch_ppt(tiles)
            rows.append({"width": W, "height": H, "stride": d, "pixels": pix, "pairs": pairs,
                         "ms_per_step": 1000.0 * wall / steps, "stages_ms": stage,
                         "fwd_evals": fe, "bwd_evals": be, "blended": bl, "tested": te,
                         "tiles": tiles, "pixels_per_thread": ppt,
                         "raster_waves": tiles * 256 // (64 * ppt),
                         "ps_per_fwd_eval": 1e9 * stage["raster_fwd"] / max(fe, 1),
                         "ps_per_bwd_eval": 1e9 * stage["raster_bwd"] / max(be, 1),
                         "fwd_frac": _alu(fwd_ops(fe, te, bl, pix, 64 * ppt), stage["raster_fwd"])["frac"],
                         "bwd_frac": _alu(bwd_ops(bl), stage["raster_bwd"])["frac"],
                         "workspace_bytes": int(sz.workspace_bytes),
                         "pair_list_bytes": 4 * pairs,
                         "entry_bytes_capacity": 12 * cap,
                         "per_pixel_state_bytes": 8 * pix})
            log(f"# sweep {W}x{H} d={d}: {rows[-1]['ms_per_step']:.3f} ms, {pairs} pairs, "
                f"workspace {int(sz.workspace_bytes) / 2**30:.2f} GiB")
            del r, v
            torch.cuda.empty_cache()
        del target
    return {"workload": f"{w['name']} views at 1080p/1440p/4K x stride 1/2/4", "gaussians": n,
            "steps": steps, "warmup": warmup, "rows": rows}


def _time_events(torch, fn, steps):
    """Per-step milliseconds of fn() between events on the current stream."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def run_batched(args, api, torch, np):
    """The multi-view batch: views of mixed resolution and stride rendered by
    the batched calls, replayed from one captured graph; compared with the
    same step enqueued eagerly, with the views processed one by one through
    the single-view calls, and with the plain full-resolution batch."""
    from paper_2412_13547_amd import scenes
    w = scenes.WORKLOADS[3]
    n = args.n or w["n"]
    sc = scenes.cluster_scene(3, n, w["sh_degree"])
    vspec = scenes.batched_views(2003, w["views"])
    dev = api.DeviceScene.from_scene(sc)
    del sc
    targets = [torch.as_tensor(scenes.target_image(c.width, c.height, 1003 + k)).cuda()
               for k, (c, _d) in enumerate(vspec)]
    ctx = api.Context(0)
    grads = dev.zeros_like()
    pos = torch.empty(n, dtype=torch.float32, device="cuda")
    col = torch.empty(n, dtype=torch.float32, device="cuda")
    vis = torch.empty(n, dtype=torch.uint8, device="cuda")
    views = [(c, d) + scenes.phase_offsets(k, d) for k, (c, d) in enumerate(vspec)]
    log("# batch views: " + ", ".join(f"{c.width}x{c.height}/d{d}" for c, d, _x, _y in views))

    def make(vs, counts=False):
        b = api.Batch(ctx, n, vs, tile=16, lds_batch=args.lds_batch, counts=counts)
        b.set_targets(targets)
        b.fit_capacity(dev)
        return b

    def graph_of(b):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            b.step(dev, grads, pos, col, vis)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            b.step(dev, grads, pos, col, vis)
        return g

    K = args.batched_steps
    res = {"workload": w["name"], "gaussians": n, "sh_degree": w["sh_degree"],
           "views": [f"{c.width}x{c.height}/d{d}/o{ox}{oy}" for c, d, ox, oy in views]}
    # evaluation counts (one forward with the per-pixel counters)
    b = make(views, counts=True)
    b.forward(dev)
    pc = b.pair_counts()
    s64 = lambda ts: int(sum(int(t.sum(dtype=torch.int64)) for t in ts))
    fwd_e, bwd_e, blended = s64(b.n_eval), s64(b.last_contrib), s64(b.n_blend)
    tested = s64(b.n_tested)
    batch_pixels = sum(int(vw.image_shape[1]) * int(vw.image_shape[2]) for vw in b.views)
    res.update(pairs=int(sum(pc)), fwd_evals=fwd_e, bwd_evals=bwd_e, blended=blended,
               tested=tested)
    del b
    torch.cuda.empty_cache()
    b = make(views)
    # eager, staged: per-stage means
    stage_names = ("preprocess_fwd", "bin_sort", "raster_fwd", "l1_grad", "raster_bwd",
                   "preprocess_bwd")
    fns = (lambda: b.preprocess_fwd(dev), lambda: b.bin_sort(dev), lambda: b.raster_fwd(),
           lambda: b.l1_grad(), lambda: b.raster_bwd(),
           lambda: b.preprocess_bwd(dev, grads, pos, col, vis))
    for _ in range(2):
        for f in fns:
            f()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(K)]
    torch.cuda.synchronize()
    for k in range(K):
        ev[k][0].record()
        for i, f in enumerate(fns):
            f()
            ev[k][i + 1].record()
    torch.cuda.synchronize()
    res["stages_ms"] = {s: statistics.mean([e[i].elapsed_time(e[i + 1]) for e in ev])
                        for i, s in enumerate(stage_names)}
    eager = _time_events(torch, lambda: b.step(dev, grads, pos, col, vis), K)
    g = graph_of(b)
    g.replay()
    graphed = _time_events(torch, g.replay, K)
    res["ms_per_step"] = float(np.median(graphed))
    res["ms_eager"] = float(np.median(eager))
    res["ms_p10"], res["ms_p90"] = float(np.percentile(graphed, 10)), float(np.percentile(graphed, 90))
    res["evals_per_s"] = (fwd_e + bwd_e) / (res["ms_per_step"] / 1000.0)
    log(f"# batched: graph {res['ms_per_step']:.3f} ms, eager {res['ms_eager']:.3f} ms, "
        f"stages {res['stages_ms']}")
    del g, b
    torch.cuda.empty_cache()
    # one view at a time through the single-view calls (each binning reads its
    # pair count back)
    singles = [api.View(ctx, n, c, d, ox, oy, 16, lds_batch=args.lds_batch) for c, d, ox, oy in views]
    imgs = [torch.empty(v.image_shape, dtype=torch.float32, device="cuda") for v in singles]
    dls = [torch.empty_like(t) for t in imgs]
    loss = torch.empty(1, dtype=torch.float64, device="cuda")

    def per_view():
        for v, img, dl, tg in zip(singles, imgs, dls, targets):
            v.forward(dev, img)
            v.l1_grad(img, tg, dl, loss)
            v.backward(dev, dl, grads, pos, col, vis)
    per_view()
    res["ms_per_view_calls"] = float(np.median(_time_events(torch, per_view, max(3, K // 2))))
    del singles, imgs, dls
    torch.cuda.empty_cache()
    # plain: every view at full resolution, batched and graphed
    if not args.no_plain:
        plain_views = [(c, 1, 0, 0) for c, _d, _x, _y in views]
        b = make(plain_views, counts=True)
        b.forward(dev)
        ppc = b.pair_counts()
        pe = s64(b.n_eval) + s64(b.last_contrib)
        del b
        torch.cuda.empty_cache()
        b = make(plain_views)
        g = graph_of(b)
        g.replay()
        pt = _time_events(torch, g.replay, max(3, K // 2))
        res["plain"] = {"ms_per_step": float(np.median(pt)), "pairs": int(sum(ppc)), "evals": pe,
                        "evals_per_s": pe / (float(np.median(pt)) / 1000.0)}
        res["speedup_vs_plain"] = res["plain"]["ms_per_step"] / res["ms_per_step"]
        log(f"# plain batch: {res['plain']['ms_per_step']:.3f} ms")
        del g, b
        torch.cuda.empty_cache()
    res["speedup_vs_per_view_calls"] = res["ms_per_view_calls"] / res["ms_per_step"]
    res["speedup_graph_vs_eager"] = res["ms_eager"] / res["ms_per_step"]
    st = res["stages_ms"]
    wpix = wave_pixels()
    res["roofline_raster_bwd"] = dict(**_alu(bwd_ops(blended), st["raster_bwd"]))
    res["roofline_raster_fwd"] = dict(**_alu(fwd_ops(fwd_e, tested, blended, batch_pixels, wpix),
                                             st["raster_fwd"]))
    return res


def run_autograd(args, api, torch, np, steps=20):
    """The training step through the autograd functions: parameters (means,
    log-scales, raw quaternions, opacity logits, SH) -> activations -> dilated
    image -> L1 loss -> backward -> fused Adam, phases cycling; against the
    same step at stride 1."""
    from paper_2412_13547_amd import autograd, scenes
    w = scenes.WORKLOADS[4]
    sc, cam, tgt = scenes.workload(4, n=args.n)
    target = torch.as_tensor(tgt).cuda()
    del tgt
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).cuda().requires_grad_(True)
    P = [f(sc.means), f(np.log(sc.scales)), f(sc.quats),
         f(np.log(sc.opacities / (1.0 - sc.opacities))), f(sc.sh)]
    deg, n = sc.sh_degree, sc.n
    del sc
    ctx = api.Context(0)
    res = {"workload": w["name"], "gaussians": n, "width": cam.width, "height": cam.height}
    for stride in (w["stride"], 1):
        view = api.View(ctx, n, cam, stride, 0, 0, 16)
        adam = api.Adam(ctx, [p.detach() for p in P], [1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3])
        stats = autograd.Stats(n)

        def step(k):
            view.set_offsets(*scenes.phase_offsets(k, stride))
            img = autograd.rasterize(view, P[0], torch.exp(P[1]), P[2], torch.sigmoid(P[3]),
                                     P[4], sh_degree=deg, stats=stats)
            loss = autograd.l1_loss(view, img, target)
            grads = torch.autograd.grad(loss, P)
            adam.step([g.contiguous() for g in grads])
        for k in range(3):
            step(k)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(ev):
            a.record()
            step(3 + k)
            b.record()
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        key = "dilated" if stride > 1 else "plain"
        res[key] = {"stride": stride, "ms_per_step": ms}
        log(f"# autograd {key}: {ms:.3f} ms/step")
        del view, adam, stats
        torch.cuda.empty_cache()
    res["speedup_vs_plain"] = res["plain"]["ms_per_step"] / res["dilated"]["ms_per_step"]
    return res


def measured_traffic(kernel_source: str, record: str):
    """HBM bytes per launch (fetch + write) from a committed counter record,
    or None when the kernel's source has changed since it was taken."""
    import hashlib
    try:
        fields = {}
        for line in open(os.path.join(ROOT, record)):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        sha = hashlib.sha256(open(os.path.join(ROOT, kernel_source), "rb").read()).hexdigest()
        if fields.get("source_sha256") != sha:
            return None
        return float(fields["fetch_bytes_per_launch"]) + float(fields["write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _alu(ops, t_ms):
    a = ops / (t_ms / 1000.0) / 1e12
    return {"bound": "alu", "achieved": a, "peak": PEAK_VALU / 1e12, "unit": "T lane-ops/s",
            "frac": a / (PEAK_VALU / 1e12), "peak_packed": PEAK_VALU_PACKED / 1e12,
            "frac_packed": a / (PEAK_VALU_PACKED / 1e12)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2412_13547_amd import api, scenes

    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")      # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("# calibration copy: 1 GiB read + 1 GiB written")

    if getattr(args, "only_autograd", False):
        print(json.dumps(run_autograd(args, api, torch, np)), flush=True)
        return
    if args.only_batched:
        print(json.dumps(run_batched(args, api, torch, np)), flush=True)
        return
    if args.only_sweep:
        print(json.dumps(run_sweep(args, api, torch, np)), flush=True)
        return
    sc, cam, tgt = scenes.workload(args.workload, n=args.n)
    w = scenes.WORKLOADS[args.workload]
    stride = w.get("stride", 1)
    dev = api.DeviceScene.from_scene(sc)
    target = torch.as_tensor(tgt).cuda()
    del tgt
    log(f"# scene ready: n={sc.n} {cam.width}x{cam.height} stride={stride}")

    dil = Runner(api, torch, dev, cam, target, stride)
    wall, per_step, stage = dil.timed(args.steps, args.warmup)
    ms = 1000.0 * wall / args.steps
    cnt = [dil.counts(k) for k in range(stride * stride)]
    fwd_evals = float(np.mean([c[0] for c in cnt]))
    bwd_evals = float(np.mean([c[1] for c in cnt]))
    blended = float(np.mean([c[2] for c in cnt]))
    tested = float(np.mean([c[4] for c in cnt]))
    dil_pixels = int(dil.view.image_shape[1]) * int(dil.view.image_shape[2])
    fwd_orders = None
    if not args.no_order_study:
        fwd_cold, fwd_warm = dil.forward_orders()
        fwd_orders = {"cold": fwd_cold, "warm": fwd_warm}
    pairs = float(np.mean([c[3] for c in cnt]))
    log(f"# dilated: {ms:.3f} ms/step, pairs {pairs:.0f}, stages {stage}")

    plain = None
    if not args.no_plain and stride > 1:
        pr = Runner(api, torch, dev, cam, target, 1)
        psteps = max(3, args.steps // 2)
        pwall, pper, pstage = pr.timed(psteps, 2)
        pc = pr.counts(0)
        pms = 1000.0 * pwall / psteps
        plain = {"ms_per_step": pms, "evals_per_s": (pc[0] + pc[1]) / (pms / 1000.0),
                 "pairs": pc[3], "stages_ms": pstage, "fwd_evals": pc[0], "bwd_evals": pc[1]}
        log(f"# plain: {pms:.3f} ms/step, stages {pstage}")
        del pr

    # rooflines: the two raster kernels against FP32 VALU issue, the binning
    # stage against HBM (bytes the implementation has to move)
    alu = _alu
    n = sc.n
    label_fwd, label_bwd = raster_labels()
    wpix = wave_pixels()
    roof_bwd = dict(kernel=label_bwd, **alu(bwd_ops(blended), stage["raster_bwd"]),
                    traffic=measured_traffic("paper_2412_13547_amd/csrc/raster.hip",
                                             "profiles/raster_bwd_dilated4k_traffic.txt"))
    roof_fwd = dict(kernel=label_fwd,
                    **alu(fwd_ops(fwd_evals, tested, blended, dil_pixels, wpix), stage["raster_fwd"]))
    # the least the stage must move: the pair list (4 B per pair) and, per
    # Gaussian, its rectangle inputs (u, v, radius: 12 B) and depth key and
    # index written and read by the depth sort (16 B)
    sort_bytes = 4.0 * pairs + 28.0 * n
    roof_sort = {"stage": "bin_sort", "bound": "hbm",
                 "achieved": sort_bytes / (stage["bin_sort"] / 1000.0) / 1e9,
                 "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    roof_sort["frac"] = roof_sort["achieved"] / roof_sort["peak"]

    out = {
        "metric": "fwd+bwd ms/iter & Gaussian-pixel evals/s, 4K dilated batched vs plain",
        "value": (fwd_evals + bwd_evals) / (ms / 1000.0),
        "unit": "Gaussian-pixel evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_p10": float(np.percentile(per_step, 10)), "ms_p50": float(np.median(per_step)),
        "ms_p90": float(np.percentile(per_step, 90)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": w["name"], "gaussians": n, "sh_degree": sc.sh_degree,
                   "width": cam.width, "height": cam.height, "stride": stride, "tile": 16,
                   "phases": "cycle (0,0),(1,0),(0,1),(1,1)" if stride == 2 else "single"},
        "pairs": pairs, "fwd_evals": fwd_evals, "bwd_evals": bwd_evals, "blended": blended,
        "tested": tested,
        "stages_ms": stage,
        "raster_fwd_tile_order_ms": fwd_orders,
        "plain": plain,
        "speedup_vs_plain": (plain["ms_per_step"] / ms) if plain else None,
        "roofline": roof_bwd,
        "rooflines_other": [roof_fwd, roof_sort],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dil, args.cpu_seconds)
    del dil
    torch.cuda.empty_cache()
    if not args.no_sweep:
        out["sweep"] = run_sweep(args, api, torch, np, dev=dev)
    if not args.no_batched:
        del dev, target
        torch.cuda.empty_cache()
        out["batched"] = run_batched(args, api, torch, np)
    if not args.no_autograd:
        torch.cuda.empty_cache()
        out["autograd"] = run_autograd(args, api, torch, np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
