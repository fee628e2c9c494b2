"""The batched multi-view path against the single-view path and the oracle.

A batch renders several views (each with its own resolution, stride and
offsets) of one Gaussian set with one preprocess launch, per-view binning and
one rasterizer launch per direction; its gradients are summed over the views.

Bars: per view, records, pair lists, ranges, images and per-pixel counters
bit-exact against the single-view calls (the same kernels and arithmetic);
summed gradients and statistics within the gradient tolerance of the sum of
the single-view results (float atomics make neither side bit-reproducible);
each view's blend backward and the summed preprocess backward against the
oracle (stage isolation); graph replays match the eager step.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import ctx, grad_close, quat_floor, records_to_oracle, run_gpu, say
from oracle import backward as obw
from oracle import binning as obn
from oracle import preprocess as opre
from oracle import raster as ors
from paper_2412_13547_amd import api, scenes

pytestmark = pytest.mark.gpu
F64 = torch.float64
PARAMS = ("means", "scales", "quats", "opacities", "sh")

# (width, height, stride, off_x, off_y)
SPECS = [(160, 120, 2, 1, 0), (96, 64, 1, 0, 0), (200, 150, 4, 3, 2), (128, 96, 3, 2, 1)]
_CACHE = {}


def _setup(tile=16, lds_batch=0, specs=SPECS, seed=7, n=400, deg=3):
    key = (tile, lds_batch, tuple(specs), seed, n, deg)
    if key in _CACHE:
        return _CACHE[key]
    sc, cams = scenes.small_multiview(seed, n, [(w, h) for (w, h, *_rest) in specs], sh_degree=deg)
    targets = [scenes.target_image(c.width, c.height, 900 + k) for k, c in enumerate(cams)]
    say(f"[gpu] batch T={tile} lds={lds_batch} views={len(specs)} n={sc.n}")
    dev = api.DeviceScene.from_scene(sc)
    views = [(cams[k], d, ox, oy) for k, (_w, _h, d, ox, oy) in enumerate(specs)]
    b = api.Batch(ctx(), sc.n, views, tile=tile, lds_batch=lds_batch, counts=True,
                  view_stats=True)
    b.set_targets([torch.as_tensor(t).cuda() for t in targets])
    counts = b.fit_capacity(dev)
    grads = dev.zeros_like()
    n_ = sc.n
    pos = torch.empty(n_, dtype=torch.float32, device="cuda")
    col = torch.empty(n_, dtype=torch.float32, device="cuda")
    vis = torch.empty(n_, dtype=torch.uint8, device="cuda")
    b.step(dev, grads, pos, col, vis)
    b.pair_counts()
    torch.cuda.synchronize()
    out = dict(sc=sc, cams=cams, targets=targets, dev=dev, batch=b, counts=counts,
               grads={k: getattr(grads, k).cpu() for k in PARAMS}, pos=pos.cpu(), col=col.cpu(),
               vis=vis.cpu(), grads_dev=grads,
               images=[t.cpu() for t in b.images], dL=[t.cpu() for t in b.dL],
               loss=b.loss.cpu(),
               t_final=[t.cpu() for t in b.t_final], last=[t.cpu() for t in b.last_contrib],
               n_eval=[t.cpu() for t in b.n_eval], n_blend=[t.cpu() for t in b.n_blend],
               n_tested=[t.cpu() for t in b.n_tested],
               records=[v.records().cpu() for v in b.views],
               pair_vals=[v.pair_vals().cpu() for v in b.views],
               ranges=[v.ranges().cpu() for v in b.views],
               grad2d=[v.grad2d().cpu() for v in b.views],
               view_pos=[t.cpu() for t in b.view_pos], view_col=[t.cpu() for t in b.view_col],
               view_vis=[t.cpu() for t in b.view_vis])
    out["singles"] = [run_gpu(sc, cams[k], d, ox, oy, tile, target=targets[k])
                      for k, (_w, _h, d, ox, oy) in enumerate(specs)]
    _CACHE[key] = out
    return out


def test_batch_forward_bitwise_equals_single_views():
    r = _setup()
    for k, s in enumerate(r["singles"]):
        assert r["counts"][k] == s["pair_count"] > 0
        assert torch.equal(r["records"][k], s["records"]), k
        assert torch.equal(r["pair_vals"][k], s["pair_vals"]), k
        assert torch.equal(r["ranges"][k], s["ranges"]), k
        assert torch.equal(r["images"][k], s["image"]), k
        assert torch.equal(r["t_final"][k], s["t_final"]), k
        assert torch.equal(r["last"][k], s["last_contrib"]), k
        assert torch.equal(r["n_eval"][k], s["n_eval"]), k
        assert torch.equal(r["n_blend"][k], s["n_blend"]), k
        assert torch.equal(r["dL"][k], s["dL"]), k
        assert abs(float(r["loss"][k]) - float(s["loss"].item())) <= 1e-12 * float(r["loss"][k])
    say(f"[gpu] batch forward bit-exact on {len(r['singles'])} views, pairs {r['counts']}")


def test_batch_tested_entries_lie_between_blends_and_examined():
    """An entry is tested pixel by pixel unless the bound over the pixel's
    wavefront excludes it, and every blended entry must have been tested."""
    r = _setup()
    for k in range(len(r["singles"])):
        nt, ne, nb = r["n_tested"][k], r["n_eval"][k], r["n_blend"][k]
        assert bool((nb <= nt).all()) and bool((nt <= ne).all()), k
        assert int(nt.sum()) > 0, k
    say(f"[gpu] tested/examined {[int(t.sum()) for t in r['n_tested']]} / "
        f"{[int(t.sum()) for t in r['n_eval']]}")


def test_batch_gradients_are_sums_of_single_views():
    r = _setup()
    singles = r["singles"]
    for name in PARAMS:
        want = sum(s["grads"][name].to(F64) for s in singles)
        grad_close(r["grads"][name], want, name=f"batch {name}",
                   floor=_qfloor(r) if name == "quats" else None)
    grad_close(r["pos"], sum(s["pos_stat"].to(F64) for s in singles), name="pos_stat")
    grad_close(r["col"], sum(s["col_stat"].to(F64) for s in singles), name="col_stat")
    assert torch.equal(r["vis"].to(torch.int64), sum(s["visible"].to(torch.int64) for s in singles))
    assert int(r["vis"].max()) == len(singles)


def test_batch_statistics_per_view_equal_single_views():
    """Each view's own densification statistics from the batched backward
    (Sec. 4.3's positional and appearance gradient norms and visibility)
    equal the single-view call's; they also add up to the summed ones."""
    r = _setup()
    for k, s in enumerate(r["singles"]):
        assert torch.equal(r["view_vis"][k], s["visible"]), k
        grad_close(r["view_pos"][k], s["pos_stat"].to(F64), name=f"view {k} pos_stat")
        grad_close(r["view_col"][k], s["col_stat"].to(F64), name=f"view {k} col_stat")
    assert torch.equal(sum(t.to(torch.int64) for t in r["view_vis"]), r["vis"].to(torch.int64))
    grad_close(r["pos"], sum(t.to(F64) for t in r["view_pos"]), name="pos_stat of the per-view sums")
    grad_close(r["col"], sum(t.to(F64) for t in r["view_col"]), name="col_stat of the per-view sums")
    say(f"[gpu] per-view statistics of {len(r['singles'])} views match the single-view calls")


def test_batch_backward_against_oracle():
    """Each view's blend backward, then the summed preprocess backward, by the
    oracle from the HIP path's own upstream outputs.  Pixels the oracle
    flags (a float decision on its threshold) take no upstream gradient on
    either side: the batch's backward is re-run with those dL values zeroed."""
    r = _setup()
    sc, b, dev = r["sc"], r["batch"], r["dev"]
    params = opre.params(sc, requires_grad=True)
    masked = []
    for k, (_w, _h, d, ox, oy) in enumerate(SPECS):
        cam = r["cams"][k]
        g = obn.grid(cam.width, cam.height, d, ox, oy, 16)
        rec = records_to_oracle(r["records"][k])
        o = ors.raster_forward(rec, r["pair_vals"][k].to(torch.int64),
                               r["ranges"][k].to(torch.int64), g)
        say(f"[gpu] view {k}: {int(o['flag'].sum())} flagged pixels")
        dl = r["dL"][k].to(F64) * (~o["flag"]).to(F64)[None]
        masked.append(dl)
        b.dL[k].copy_(dl.to(torch.float32).cuda())
    b.raster_bwd()
    grads = dev.zeros_like()
    b.preprocess_bwd(dev, grads)
    torch.cuda.synchronize()
    total = qfloor = None
    for k, (_w, _h, d, ox, oy) in enumerate(SPECS):
        cam = r["cams"][k]
        g = obn.grid(cam.width, cam.height, d, ox, oy, 16)
        rec = records_to_oracle(r["records"][k])
        want2d = obw.raster_backward(rec, r["pair_vals"][k].to(torch.int64),
                                     r["ranges"][k].to(torch.int64), g, masked[k])
        got2d = b.views[k].grad2d().cpu()
        for c, nm in enumerate(("u", "v", "A", "B", "C", "opacity", "r", "g", "b")):
            grad_close(got2d[:, c], want2d[:, c], name=f"view {k} d{nm}")
        g2d = got2d.to(F64).clone()
        near = (opre.preprocess(opre.params(sc), opre.camera(cam))["rgb_raw"].abs() < 1e-5).any(1)
        assert not bool(near.any())
        part = obw.preprocess_backward(params, opre.camera(cam), g2d)
        total = part if total is None else {n: total[n] + part[n] for n in total}
        qf = quat_floor(sc, cam, g2d)
        qfloor = qf if qfloor is None else qfloor + qf
    got = {k: getattr(grads, k).cpu() for k in PARAMS}
    grad_close(got["means"].T, total["means"], name="means")
    grad_close(got["scales"].T, total["scales"], name="scales")
    grad_close(got["quats"].T, total["quats"], name="quats", floor=qfloor)
    grad_close(got["opacities"], total["opacities"], name="opacities")
    grad_close(got["sh"].permute(2, 0, 1), total["sh"], name="sh")
    for k in range(len(SPECS)):                  # the batch's own upstream gradients back
        b.dL[k].copy_(r["dL"][k].cuda())


def _qfloor(r):
    """Quaternion allowance of a batch's summed gradient: the single views'
    allowances (gpu_helpers.quat_floor) summed, laid out like the HIP
    gradient (4 x N)."""
    if "qfloor" not in r:
        r["qfloor"] = sum(quat_floor(r["sc"], r["cams"][k], s["grad2d"])
                          for k, s in enumerate(r["singles"])).T
    return r["qfloor"]


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_batch_gradients_other_sh_degrees(deg):
    """The multi-view preprocess backward at SH degrees 0-2 (its sums of the
    SH gradients over the views are kept in LDS, (deg + 1)^2 x 3 floats per
    thread): the summed gradients and statistics equal the sums of the
    single views' (Sec. 4.3 statistics included)."""
    r = _setup(deg=deg, specs=SPECS[:3])
    singles = r["singles"]
    assert r["grads"]["sh"].shape[0] >= (deg + 1) ** 2
    for name in PARAMS:
        want = sum(s["grads"][name].to(F64) for s in singles)
        grad_close(r["grads"][name], want, name=f"batch SH{deg} {name}",
                   floor=_qfloor(r) if name == "quats" else None)
    grad_close(r["pos"], sum(s["pos_stat"].to(F64) for s in singles), name=f"SH{deg} pos_stat")
    grad_close(r["col"], sum(s["col_stat"].to(F64) for s in singles), name=f"SH{deg} col_stat")
    assert torch.equal(r["vis"].to(torch.int64), sum(s["visible"].to(torch.int64) for s in singles))


@pytest.mark.parametrize("lds_batch", [64, 128])
def test_lds_batch_does_not_change_results(lds_batch):
    base = _setup()
    r = _setup(lds_batch=lds_batch)
    for k in range(len(SPECS)):
        assert torch.equal(r["images"][k], base["images"][k])
        assert torch.equal(r["n_eval"][k], base["n_eval"][k])
        assert torch.equal(r["last"][k], base["last"][k])
    for name in PARAMS:
        grad_close(r["grads"][name], base["grads"][name].to(F64), name=f"lds{lds_batch} {name}",
                   floor=_qfloor(base) if name == "quats" else None)


@pytest.mark.parametrize("tile", [8, 32])
def test_batch_other_tile_sizes_match_single_views(tile):
    r = _setup(tile=tile)
    for k, s in enumerate(r["singles"]):
        assert torch.equal(r["pair_vals"][k], s["pair_vals"]), k
        assert torch.equal(r["images"][k], s["image"]), k
        assert torch.equal(r["n_eval"][k], s["n_eval"]), k
    for name in PARAMS:
        grad_close(r["grads"][name], sum(s["grads"][name].to(F64) for s in r["singles"]),
                   name=f"T{tile} {name}", floor=_qfloor(r) if name == "quats" else None)


def test_overflowing_view_renders_background_and_is_reported():
    base = _setup()
    sc, cams = base["sc"], base["cams"]
    views = [(cams[k], d, ox, oy) for k, (_w, _h, d, ox, oy) in enumerate(SPECS)]
    caps = [c + 16 for c in base["counts"]]
    caps[1] = base["counts"][1] // 2            # view 1 cannot hold its pairs
    b = api.Batch(ctx(), sc.n, views, tile=16, bg=(0.25, 0.5, 0.75), pair_capacity=caps,
                  counts=True)
    b.set_targets([torch.as_tensor(t).cuda() for t in base["targets"]])
    dev = base["dev"]
    grads = dev.zeros_like()
    b.step(dev, grads)
    with pytest.raises(api.TgsError) as e:
        b.pair_counts()
    assert e.value.status == api.TGS_ERR_CAPACITY and "view 1" in str(e.value)
    torch.cuda.synchronize()
    assert [int(s.pair_count) for s in b.states] == base["counts"]
    img1 = b.images[1].cpu()
    for c, v in enumerate((0.25, 0.5, 0.75)):
        assert bool((img1[c] == v).all())
    assert int(b.n_eval[1].cpu().abs().sum()) == 0
    assert not bool(b.views[1].grad2d().cpu().any())
    # the other views are unaffected (background enters only through T bg)
    single = run_gpu(sc, cams[0], 2, 1, 0, 16, bg=(0.25, 0.5, 0.75), backward=False)
    assert torch.equal(b.images[0].cpu(), single["image"])


def test_graph_capture_replays_match_eager_step():
    r = _setup()
    b, dev = r["batch"], r["dev"]
    grads = dev.zeros_like()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.step(dev, grads)                       # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.step(dev, grads)
    for rep in range(3):
        for t in b.images:
            t.fill_(-1.0)                        # eager work between replays
        grads.means.fill_(123.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in range(len(SPECS)):
            assert torch.equal(b.images[k].cpu(), r["images"][k]), (rep, k)
            assert torch.equal(b.n_eval[k].cpu(), r["n_eval"][k]), (rep, k)
        for name in PARAMS:
            grad_close(getattr(grads, name).cpu(), r["grads"][name].to(F64), name=f"replay {rep} {name}",
                       floor=_qfloor(r) if name == "quats" else None)
    say("[gpu] 3 graph replays match the eager step")


def test_one_view_backward_after_batched_forward_reads_the_coefficients():
    """A one-view preprocess backward takes the colour's gradient in the view
    direction (Sec. 3, view-dependent SH colour) from the Jacobian rows that a
    one-view forward leaves in the workspace.  After a batched forward of
    several views, which leaves none and clears the word beside the
    non-finite counter, it reads the SH coefficients instead.  From the same
    grad2d the two give bit-equal gradients of every parameter but the means,
    where only the rounding order of the colour term differs."""
    r = _setup()
    b, dev = r["batch"], r["dev"]
    n = r["sc"].n
    b.step(dev, dev.zeros_like())                # a batched forward: no Jacobian rows
    torch.cuda.synchronize()
    for k, v in enumerate(b.views):
        current = v._view(v.state.off_nonfinite_count + 4, 1, torch.int32)
        assert int(current.item()) == 0, k
        outs = []
        for step in ("coefficients", "jacobian"):
            if step == "jacobian":
                v.preprocess_fwd(dev)            # records as before, plus the rows
                torch.cuda.synchronize()
                assert int(current.item()) == 1, k
            g = dev.zeros_like()
            pos = torch.empty(n, dtype=torch.float32, device="cuda")
            col = torch.empty(n, dtype=torch.float32, device="cuda")
            vis = torch.empty(n, dtype=torch.uint8, device="cuda")
            v.preprocess_bwd(dev, g, pos, col, vis)
            torch.cuda.synchronize()
            outs.append(({p: getattr(g, p).cpu() for p in PARAMS}, pos.cpu(), col.cpu(), vis.cpu()))
        (ga, pa, ca, va), (gb, pb, cb, vb) = outs
        assert torch.equal(pa, pb) and torch.equal(ca, cb) and torch.equal(va, vb), k
        assert int(va.sum()) > 0, k
        for p in ("scales", "quats", "opacities", "sh"):
            assert torch.equal(ga[p], gb[p]), (k, p)
        grad_close(gb["means"], ga["means"].to(F64), name=f"view {k} means, Jacobian rows vs SH")
    say(f"[gpu] {len(b.views)} views: one-view backward after a batched forward matches the rows")
