"""Launch autotuner of the batched rasterizer: times one graph-replayed fitting
step (forward, L1 gradient, backward of every view) for each tile size T in
{8, 16, 32}, each work split (pixels per thread P: 1 for T = 8; 1, 2, 4 for
T = 16; 2, 4 for T = 32) and each LDS batch B in {64, 128, 256}.

P and B only change speed, so ``best_launch`` maps every tile size to its
fastest (P, B), which can be applied without changing any result.  T changes
which Gaussians a pixel considers (the tile grid is part of the method's
definition, Sec. 4.1), so ``best`` -- the fastest (T, P, B) overall -- is a
suggestion for callers that accept another tile size.

    python -m paper_2412_13547_amd.autotune [--n 2000000] [--views 12] [--steps 5]

Results can be cached in a JSON file keyed by device name and workload
signature (``cache=`` / ``--cache``).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys

TILES = (8, 16, 32)
LDS_BATCHES = (64, 128, 256)
SPLITS = {8: (1,), 16: (1, 2, 4), 32: (2, 4)}


def _signature(n, views, sh_degree) -> str:
    vs = ";".join(f"{c.width}x{c.height}/{d}/{ox}{oy}" for c, d, ox, oy in views)
    return f"n={n}|deg={sh_degree}|{vs}"


def time_config(api, torch, ctx, dev, views, targets, tile, lds, steps, ppt=0):
    """Median ms of a graph-replayed batch step for one (tile, split, lds batch)."""
    n = dev.n
    b = api.Batch(ctx, n, views, tile=tile, lds_batch=lds, pixels_per_thread=ppt)
    b.set_targets(targets)
    b.fit_capacity(dev)
    grads = dev.zeros_like()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.step(dev, grads)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.step(dev, grads)
    g.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        e.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(e))
    del g, b, grads
    torch.cuda.empty_cache()
    return statistics.median(times)


def tune(dev, views, targets, steps=5, tiles=TILES, lds_batches=LDS_BATCHES, cache=None,
         log=None):
    """Sweep (tile, lds batch) over a batch of views; returns a dict with the
    table of timings, the fastest LDS batch per tile and the fastest pair."""
    import torch
    from . import api
    key = None
    if cache:
        name = torch.cuda.get_device_name(0)
        key = f"{name}|{_signature(dev.n, views, dev.sh_degree)}"
        if os.path.exists(cache):
            with open(cache) as f:
                stored = json.load(f)
            if key in stored:
                return stored[key]
    ctx = api.Context(0)
    table = []
    for t in tiles:
        for ppt in SPLITS[t]:
            for lb in lds_batches:
                ms = time_config(api, torch, ctx, dev, views, targets, t, lb, steps, ppt)
                table.append({"tile": t, "pixels_per_thread": ppt, "lds_batch": lb, "ms": ms})
                if log:
                    log(f"# autotune T={t} P={ppt} B={lb}: {ms:.3f} ms")
    best_launch = {}
    for t in tiles:
        r = min((r for r in table if r["tile"] == t), key=lambda r: r["ms"])
        best_launch[str(t)] = {"pixels_per_thread": r["pixels_per_thread"],
                               "lds_batch": r["lds_batch"], "ms": r["ms"]}
    best = min(table, key=lambda r: r["ms"])
    out = {"table": table, "best_launch": best_launch, "best": dict(best)}
    if cache:
        stored = {}
        if os.path.exists(cache):
            with open(cache) as f:
                stored = json.load(f)
        stored[key] = out
        with open(cache, "w") as f:
            json.dump(stored, f, indent=1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--views", type=int, default=12)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--cache", default=None)
    args = ap.parse_args()
    import torch
    from . import api, scenes
    w = scenes.WORKLOADS[3]
    n = args.n or w["n"]
    sc = scenes.cluster_scene(3, n, w["sh_degree"])
    vspec = scenes.batched_views(2003, args.views)
    views = [(c, d) + scenes.phase_offsets(k, d) for k, (c, d) in enumerate(vspec)]
    dev = api.DeviceScene.from_scene(sc)
    targets = [torch.as_tensor(scenes.target_image(c.width, c.height, 1003 + k)).cuda()
               for k, (c, _d) in enumerate(vspec)]
    res = tune(dev, views, targets, steps=args.steps, cache=args.cache,
               log=lambda *a: print(*a, file=sys.stderr, flush=True))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
