"""The launch autotuner (``autotune.tune``) on a tiny two-view batch: it times
every work split and LDS batch of the tile size, stores the result in its
JSON cache and returns it from there on a second call without timing
anything, and the launch it picks renders bit for bit what the default
launch renders (work split and LDS batch change speed only)."""
import json

import numpy as np
import pytest
import torch

from gpu_helpers import ctx, say
from paper_2412_13547_amd import api, autotune, scenes

pytestmark = pytest.mark.gpu


def _views():
    sc, cams = scenes.small_multiview(31, 300, [(160, 120), (96, 64)], sh_degree=1)
    views = [(cams[0], 2, 1, 0), (cams[1], 1, 0, 0)]
    targets = [torch.as_tensor(scenes.target_image(c.width, c.height, 40 + k)).cuda()
               for k, c in enumerate(cams)]
    return sc, views, targets


def _render(sc, dev, views, **launch):
    b = api.Batch(ctx(), sc.n, views, tile=16, counts=True, **launch)
    b.fit_capacity(dev)
    b.forward(dev)
    torch.cuda.synchronize()
    return [t.cpu() for t in b.images], [t.cpu() for t in b.n_eval], [t.cpu() for t in b.t_final]


def test_autotune_times_caches_and_picks_an_equivalent_launch(tmp_path, monkeypatch):
    sc, views, targets = _views()
    dev = api.DeviceScene.from_scene(sc)
    cache = tmp_path / "autotune.json"
    res = autotune.tune(dev, views, targets, steps=2, tiles=(16,), lds_batches=(64, 128),
                        cache=str(cache))
    rows = res["table"]
    assert sorted((r["pixels_per_thread"], r["lds_batch"]) for r in rows) == \
        [(p, b) for p in (1, 2, 4) for b in (64, 128)]
    assert all(r["tile"] == 16 and np.isfinite(r["ms"]) and r["ms"] > 0 for r in rows)
    best = res["best_launch"]["16"]
    assert best["ms"] == min(r["ms"] for r in rows)
    assert res["best"]["ms"] == best["ms"]
    stored = json.loads(cache.read_text())
    assert len(stored) == 1 and list(stored.values())[0] == res
    say(f"[gpu] autotune: {len(rows)} launches timed, best P={best['pixels_per_thread']} "
        f"B={best['lds_batch']} at {best['ms']:.3f} ms")

    # a second call is answered from the cache: nothing is timed
    def refuse(*_a, **_k):
        raise AssertionError("a cached workload was timed again")
    monkeypatch.setattr(autotune, "time_config", refuse)
    again = autotune.tune(dev, views, targets, steps=2, tiles=(16,), lds_batches=(64, 128),
                          cache=str(cache))
    assert again == res

    # the chosen launch renders what the default launch renders, bit for bit
    want = _render(sc, dev, views)
    got = _render(sc, dev, views, lds_batch=best["lds_batch"],
                  pixels_per_thread=best["pixels_per_thread"])
    for a, b in zip(want, got):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
    say("[gpu] autotune: cache round trip, chosen launch bit-identical to the default")
