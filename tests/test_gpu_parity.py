"""GPU parity of every stage against the CPU oracle (stage isolation: each
oracle stage is fed the HIP path's own upstream outputs, upcast to float64).

Bars: sort keys, pair lists, tile ranges, tiles_touched bit-exact;
last_contrib / n_eval exact except at pixels whose float decision lies within
a hair of its threshold (the oracle flags them); images within 1e-4 absolute;
gradients within 1e-3 relative (norm-wise and element-wise)."""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import grad_close, l1_matches_oracle, quat_floor, records_to_oracle, run_gpu, say
from oracle import backward as obw
from oracle import binning as obn
from oracle import loss as ols
from oracle import pipeline as opipe
from oracle import preprocess as opre
from oracle import raster as ors
from paper_2412_13547_amd import scenes

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _tiny():
    sc, cam, tgt = scenes.workload(0)
    return sc, cam, tgt


def _small(seed, n, w, h, deg):
    sc, cam = scenes.small_scene(seed, n, w, h, sh_degree=deg)
    return sc, cam, scenes.target_image(w, h, 500 + seed)


CASES = {
    "tiny128-d1-T16": (_tiny, 1, 0, 0, 16, (0.0, 0.0, 0.0)),
    "sh3-160x120-d2-o10-T16": (lambda: _small(1, 300, 160, 120, 3), 2, 1, 0, 16, (0.0, 0.0, 0.0)),
    "sh2-101x77-d3-o21-T8-bg": (lambda: _small(2, 200, 101, 77, 2), 3, 2, 1, 8, (0.1, 0.2, 0.3)),
    "sh1-150x130-d4-o32-T32": (lambda: _small(3, 250, 150, 130, 1), 4, 3, 2, 32, (0.0, 0.0, 0.0)),
    "sh3-96x64-d1-T8": (lambda: _small(4, 300, 96, 64, 3), 1, 0, 0, 8, (0.0, 0.5, 0.0)),
    "sh0-333x200-d2-o11-T16": (lambda: _small(5, 600, 333, 200, 0), 2, 1, 1, 16, (0.0, 0.0, 0.0)),
    # wide grids: 263 tile columns (5 column groups of the scatter, one part
    # each) and the 1024-column maximum (16 groups, 1024 threads)
    "sh1-2100x40-d1-T8": (lambda: _small(6, 400, 2100, 40, 1), 1, 0, 0, 8, (0.0, 0.0, 0.0)),
    "sh0-8192x24-d1-T8": (lambda: _small(7, 500, 8192, 24, 0), 1, 0, 0, 8, (0.0, 0.0, 0.0)),
    # tall grids: 263 tile rows, and the 4096-row maximum
    "sh1-40x2100-d1-T8": (lambda: _small(8, 400, 40, 2100, 1), 1, 0, 0, 8, (0.0, 0.0, 0.0)),
    "sh0-16x32768-d1-T8": (lambda: _small(9, 300, 16, 32768, 0), 1, 0, 0, 8, (0.0, 0.0, 0.0)),
}
_CACHE = {}


def _case(name):
    if name not in _CACHE:
        make, d, ox, oy, T, bg = CASES[name]
        sc, cam, tgt = make()
        say(f"[gpu] case {name}: n={sc.n} {cam.width}x{cam.height} d={d} o=({ox},{oy}) T={T}")
        g = run_gpu(sc, cam, d, ox, oy, T, bg, target=tgt)
        _CACHE[name] = (sc, cam, tgt, g)
    return _CACHE[name]


def _oracle_raster(g):
    rec = records_to_oracle(g["records"])
    return rec, ors.raster_forward(rec, g["pair_vals"].to(torch.int64), g["ranges"].to(torch.int64),
                                   g["grid"], bg=g["bg"])


@pytest.mark.parametrize("name", list(CASES))
def test_preprocess_matches_oracle(name):
    sc, cam, _, g = _case(name)
    o = opre.preprocess(opre.params(sc), opre.camera(cam))
    rec = records_to_oracle(g["records"])
    assert torch.equal(rec["culled"], o["culled"])
    ok = ~o["culled"]
    # integer decisions taken from floats: radius, flagged where 3 sqrt(lambda)
    # lies within 1e-5 (relative) of an integer
    ts = o["three_sigma"]
    near = (ts - torch.round(ts)).abs() < 1e-5 * ts.clamp(min=1.0)
    same_r = rec["radius"] == o["radius"]
    assert bool((same_r | near)[ok].all())
    scale_u = o["u"].abs() + abs(cam.cx) + cam.width
    assert float(((rec["u"] - o["u"]).abs() / scale_u)[ok].max()) < 2e-6
    assert float(((rec["v"] - o["v"]).abs() / (o["v"].abs() + abs(cam.cy) + cam.height))[ok].max()) < 2e-6
    qs = torch.maximum(o["A"].abs(), o["C"].abs())
    for k in ("A", "B", "C"):
        assert float(((rec[k] - o[k]).abs() / qs)[ok].max()) < 1e-4, k
    assert float((rec["rgb"] - o["rgb"]).abs()[ok].max()) < 2e-6
    assert float(((rec["z"] - o["z"]).abs() / o["z"].abs())[ok].max()) < 1e-6
    assert torch.equal(rec["opacity"][ok], torch.as_tensor(sc.opacities, dtype=F64)[ok])
    # colour clamp decisions: exact except where the raw colour is within 1e-6 of 0
    near0 = o["rgb_raw"].abs() < 1e-6
    assert bool(((rec["clamp"] == o["clamp"]) | near0)[ok].all())


@pytest.mark.parametrize("name", list(CASES))
def test_binning_sort_ranges_bit_exact(name):
    sc, cam, _, g = _case(name)
    rec = records_to_oracle(g["records"])
    b = obn.bin_gaussians(rec["u"], rec["v"], rec["z"], rec["radius"], rec["culled"], g["grid"])
    assert torch.equal(g["tiles_touched"].to(torch.int64), b["tiles_touched"])
    assert g["pair_count"] == b["keys"].numel()
    vals = g["pair_vals"].to(torch.int64)
    rg = g["ranges"].to(torch.int64)
    tiles = torch.repeat_interleave(torch.arange(rg.shape[0]), rg[:, 1] - rg[:, 0])
    assert tiles.numel() == vals.numel()
    keys = tiles * (1 << 32) + b["zbits"][vals]
    assert torch.equal(keys, b["keys"])
    assert torch.equal(vals, b["vals"])
    assert torch.equal(g["ranges"].to(torch.int64), b["ranges"])
    say(f"[gpu] {name}: {g['pair_count']} pairs bit-exact")


def _expected_depth_order(b):
    """Ids of the Gaussians with tiles, by depth bits, equal bits by id."""
    ids = torch.nonzero(b["tiles_touched"] > 0).flatten().numpy()
    zb = b["zbits"].numpy()[ids]
    return ids[np.lexsort((ids, zb))]


@pytest.mark.parametrize("name", list(CASES))
def test_depth_order_is_the_sorted_gaussians_with_tiles(name):
    sc, cam, _, g = _case(name)
    rec = records_to_oracle(g["records"])
    b = obn.bin_gaussians(rec["u"], rec["v"], rec["z"], rec["radius"], rec["culled"], g["grid"])
    got = g["_view"].depth_order().cpu().to(torch.int64).numpy()
    want = _expected_depth_order(b)
    assert got.shape == want.shape and np.array_equal(got, want)
    say(f"[gpu] {name}: depth order of {got.size} of {sc.n} Gaussians bit-exact")


def test_depth_order_ties_and_culled():
    """Exact depth ties (duplicated Gaussians) keep id order; Gaussians
    behind the camera and off-screen ones are left out of the order."""
    sc, cam = scenes.small_scene(7, 400, 128, 96, sh_degree=1)
    sc = sc.copy()
    sc.means[:, 200:300] = sc.means[:, 0:100]           # 100 exact depth ties
    sc.scales[:, 200:300] = sc.scales[:, 0:100]
    sc.quats[:, 200:300] = sc.quats[:, 0:100]
    r = cam.w2c[:, :3].astype(np.float64)
    t = cam.w2c[:, 3].astype(np.float64)
    behind = r.T @ (np.array([[0.0], [0.0], [-1.0]]) - t[:, None])
    sc.means[:, 300:340] = behind.astype(np.float32)     # behind the camera: culled
    sc.means[:, 340:360] = (r.T @ (np.array([[50.0], [0.0], [3.0]]) - t[:, None])).astype(np.float32)
    g = run_gpu(sc, cam, 2, 1, 0, 16, target=scenes.target_image(128, 96, 7))
    rec = records_to_oracle(g["records"])
    b = obn.bin_gaussians(rec["u"], rec["v"], rec["z"], rec["radius"], rec["culled"], g["grid"])
    got = g["_view"].depth_order().cpu().to(torch.int64).numpy()
    want = _expected_depth_order(b)
    assert np.array_equal(got, want)
    assert not np.isin(np.arange(300, 360), got).any()
    zb = b["zbits"].numpy()
    tied = [k for k in range(100) if zb[k] == zb[200 + k] and k in set(got.tolist())]
    assert len(tied) > 10
    pos = {int(v): i for i, v in enumerate(got)}
    assert all(pos[k] < pos[200 + k] for k in tied)
    say(f"[gpu] depth order with {len(tied)} exact ties and 60 culled or off-screen: bit-exact")


def test_depth_order_across_sort_tiles():
    """40,000 Gaussians: ten tiles of the depth sort, whose later tiles take
    their offsets from the earlier ones' published counts.  10,000 exact
    depth ties between Gaussians 20,000 indices apart (so in different
    tiles) keep id order, 4,000 culled or off-screen Gaussians interleaved
    with the rest are left out; the depth order and the pair lists are
    bit-exact."""
    n = 40_000
    sc, cam = scenes.small_scene(11, n, 320, 240, sh_degree=0)
    sc = sc.copy()
    sc.means[:, 20000:30000] = sc.means[:, 0:10000]      # exact depth ties across tiles
    sc.scales[:, 20000:30000] = sc.scales[:, 0:10000]
    sc.quats[:, 20000:30000] = sc.quats[:, 0:10000]
    r = cam.w2c[:, :3].astype(np.float64)
    t = cam.w2c[:, 3].astype(np.float64)
    behind = (r.T @ (np.array([[0.0], [0.0], [-1.0]]) - t[:, None])).astype(np.float32)
    off = (r.T @ (np.array([[50.0], [0.0], [3.0]]) - t[:, None])).astype(np.float32)
    sc.means[:, 5:n:20] = behind                         # every 20th: culled
    sc.means[:, 15:n:40] = off                           # every 40th: no tiles
    g = run_gpu(sc, cam, 1, 0, 0, 16, target=scenes.target_image(320, 240, 11), backward=False)
    rec = records_to_oracle(g["records"])
    b = obn.bin_gaussians(rec["u"], rec["v"], rec["z"], rec["radius"], rec["culled"], g["grid"])
    got = g["_view"].depth_order().cpu().to(torch.int64).numpy()
    want = _expected_depth_order(b)
    assert got.size > 4096 * 5
    assert np.array_equal(got, want)
    zb = b["zbits"].numpy()
    kept = set(got.tolist())
    tied = [k for k in range(10000) if zb[k] == zb[20000 + k] and k in kept and 20000 + k in kept]
    assert len(tied) > 1000
    pos = {int(v): i for i, v in enumerate(got)}
    assert all(pos[k] < pos[20000 + k] for k in tied)
    assert g["pair_count"] == b["keys"].numel()
    assert torch.equal(g["pair_vals"].to(torch.int64), b["vals"])
    assert torch.equal(g["ranges"].to(torch.int64), b["ranges"])
    say(f"[gpu] depth order over {got.size} Gaussians ({(got.size + 4095) // 4096} sort tiles), "
        f"{len(tied)} ties across tiles: bit-exact; {g['pair_count']} pairs bit-exact")


SPLITS = {8: (1,), 16: (1, 2, 4), 32: (2, 4)}


@pytest.mark.parametrize("name", ["sh2-101x77-d3-o21-T8-bg", "sh1-150x130-d4-o32-T32",
                                  "sh0-333x200-d2-o11-T16", "sh1-40x2100-d1-T8",
                                  "sh0-16x32768-d1-T8"])
def test_backward_tile_order_leaves_gradients_unchanged(name):
    """The forward records per tile the entries it walked (never more than the
    tile's pairs, none in an empty tile); the backward, and the next forward,
    take the tiles heaviest first by them.  With those weights replaced by
    arbitrary values (the order a stale or foreign workspace would give) the
    backward returns the same gradients up to the order of the float atomics,
    and the forward the same image and the same weights, bit for bit."""
    sc, cam, tgt, ref = _case(name)
    view, dev, image = ref["_view"], ref["_dev"], ref["_image"]
    work = view.tile_work().cpu().to(torch.int64) & 0xFFFFFFFF
    r = ref["ranges"].to(torch.int64)
    span = r[:, 1] - r[:, 0]
    assert bool((work <= span).all()), "a tile walked more entries than it holds"
    assert bool((work[span == 0] == 0).all())
    assert bool((work > 0).any())
    say(f"[gpu] {name}: {int((work > 0).sum())} of {work.numel()} tiles walked, at most {int(work.max())}")
    gen = torch.Generator().manual_seed(7)
    for trial in range(2):
        w = torch.randint(-2**31, 2**31 - 1, (work.numel(),), generator=gen, dtype=torch.int64)
        if trial == 1:
            w[::3] = -1                                          # 0xFFFFFFFF: the top bucket
        view.tile_work().copy_(w.to(torch.int32).cuda())
        dL = ref["dL"].cuda()
        grads = view.backward(dev, dL)
        torch.cuda.synchronize()
        a, b = view.grad2d().cpu().to(F64), ref["grad2d"].to(F64)
        assert float((a - b).abs().max()) <= 1e-5 * float(b.abs().max()) + 1e-12, trial
        # the parameter gradients at the gradient bar (the quaternion's with
        # its projection allowance: another atomic order moves a component
        # that is a near-cancelling difference by more than 1e-5 of the max)
        qfloor = quat_floor(sc, cam, ref["grad2d"])
        for k in ("means", "scales", "quats", "opacities", "sh"):
            a, b = getattr(grads, k).cpu().to(F64), ref["grads"][k].to(F64)
            grad_close(a, b, name=f"{name} order {trial} {k}", quiet=True,
                       floor=qfloor.T if k == "quats" else None)
        # the forward takes its order from the weights left in the workspace
        view.tile_work().copy_(w.to(torch.int32).cuda())
        img = torch.empty_like(image)
        view.raster_fwd(img)
        torch.cuda.synchronize()
        assert torch.equal(img.cpu(), ref["image"]), trial
        assert torch.equal((view.tile_work().cpu().to(torch.int64) & 0xFFFFFFFF), work), trial
    view.tile_work().copy_(work.to(torch.int32).cuda())
    say(f"[gpu] {name}: image and gradients unchanged under arbitrary tile weights")


@pytest.mark.parametrize("name", ["sh3-160x120-d2-o10-T16", "sh1-150x130-d4-o32-T32"])
def test_backward_after_a_forward_with_another_work_split(name):
    """The blend bits describe the forward's wavefronts; a backward launched
    with another work split cannot use them and visits every entry, with the
    same gradients up to the order of the float atomics."""
    from paper_2412_13547_amd import api
    sc, cam, tgt, ref = _case(name)
    _, d, ox, oy, T, bg = CASES[name]
    view = ref["_view"]
    default = view.opt
    for ppt in SPLITS[T]:
        view.opt = api.options_struct(T, bg, 0, ppt)
        view.raster_bwd(ref["dL"].cuda())
        torch.cuda.synchronize()
        grad_close(view.grad2d().cpu(), ref["grad2d"].to(F64), name=f"{name} backward P={ppt}",
                   quiet=True)
    view.opt = default
    say(f"[gpu] {name}: backward with every work split after one forward: same gradients")


@pytest.mark.parametrize("name", ["tiny128-d1-T16", "sh2-101x77-d3-o21-T8-bg",
                                  "sh1-150x130-d4-o32-T32", "sh0-333x200-d2-o11-T16"])
def test_work_split_and_lds_batch_leave_results_unchanged(name):
    """Every (pixels per thread, LDS batch) of the tile size renders the same
    image, transmittance and counters bit for bit as the checked default
    (the wavefront skips depend on the split: each must be exact), and the
    same gradients up to the order of the float atomics."""
    sc, cam, tgt, ref = _case(name)
    _, d, ox, oy, T, bg = CASES[name]
    for ppt in SPLITS[T]:
        for lds in (64, 128, 256):
            say(f"[gpu] {name}: P={ppt} B={lds}")
            g = run_gpu(sc, cam, d, ox, oy, T, bg, target=tgt, lds_batch=lds, pixels_per_thread=ppt)
            for k in ("image", "t_final", "last_contrib", "n_eval", "n_blend"):
                assert torch.equal(g[k], ref[k]), (ppt, lds, k)
            assert torch.equal(g["pair_vals"], ref["pair_vals"])
            a, b = g["grad2d"].to(F64), ref["grad2d"].to(F64)
            assert float((a - b).abs().max()) <= 1e-5 * float(b.abs().max()) + 1e-12, (ppt, lds)
            for k in ("means", "opacities", "sh"):
                a, b = g["grads"][k].to(F64), ref["grads"][k].to(F64)
                assert float((a - b).abs().max()) <= 1e-5 * float(b.abs().max()) + 1e-12, (ppt, lds, k)
    say(f"[gpu] {name}: every split and LDS batch bit-exact in the forward")


@pytest.mark.parametrize("name", list(CASES))
def test_raster_forward_matches_oracle(name):
    sc, cam, _, g = _case(name)
    _, o = _oracle_raster(g)
    flag = o["flag"]
    say(f"[gpu] {name}: flagged pixels {int(flag.sum())} of {flag.numel()}")
    assert float(flag.float().mean()) < 0.01
    err = (g["image"].to(F64) - o["image"]).abs()
    assert float(err.max()) <= 1e-4, float(err.max())
    keep = ~flag
    assert torch.equal(g["last_contrib"].to(torch.int64)[keep], o["last_contrib"][keep])
    assert torch.equal(g["n_eval"].to(torch.int64)[keep], o["n_eval"][keep])
    assert torch.equal(g["n_blend"].to(torch.int64)[keep], o["n_blend"][keep])
    assert float((g["t_final"].to(F64) - o["t_final"]).abs()[keep].max()) <= 1e-5


@pytest.mark.parametrize("name", list(CASES))
def test_raster_backward_matches_oracle(name):
    sc, cam, _, g = _case(name)
    rec, o = _oracle_raster(g)
    dL = g["dL"].to(F64) * (~o["flag"]).to(F64)[None]
    view = g["_view"]
    view.raster_bwd(dL.to(torch.float32).cuda())
    torch.cuda.synchronize()
    got = view.grad2d().cpu()
    want = obw.raster_backward(rec, g["pair_vals"].to(torch.int64), g["ranges"].to(torch.int64),
                               g["grid"], dL, bg=g["bg"])
    names = ("u", "v", "A", "B", "C", "opacity", "r", "g", "b")
    for c, nm in enumerate(names):
        grad_close(got[:, c], want[:, c], name=f"{name} d{nm}")


@pytest.mark.parametrize("name", list(CASES))
def test_preprocess_backward_matches_oracle(name):
    sc, cam, _, g = _case(name)
    c = opre.camera(cam)
    o = opre.preprocess(opre.params(sc), c)
    # Gaussians whose colour clamp or FoV guard sits on its threshold are
    # excluded: their derivative is discontinuous there
    lim_x = 1.3 * cam.width / (2 * cam.fx)
    lim_y = 1.3 * cam.height / (2 * cam.fy)
    tz = torch.as_tensor(sc.means.T.astype(np.float64)) @ c.R.T + c.t
    rx, ry = tz[:, 0] / tz[:, 2], tz[:, 1] / tz[:, 2]
    bad = (o["rgb_raw"].abs() < 1e-5).any(1) | ((rx.abs() - lim_x).abs() < 1e-5) | \
          ((ry.abs() - lim_y).abs() < 1e-5)
    view = g["_view"]
    g2d_dev = view.grad2d()
    g2d_dev[bad.cuda()] = 0.0
    grads = g["_dev"].zeros_like()
    view.preprocess_bwd(g["_dev"], grads)
    torch.cuda.synchronize()
    g2d = g2d_dev.cpu().to(F64)
    p = opre.params(sc, requires_grad=True)
    want = obw.preprocess_backward(p, c, g2d)
    got = {k: getattr(grads, k).cpu() for k in ("means", "scales", "quats", "opacities", "sh")}
    grad_close(got["means"].T, want["means"], name=f"{name} means")
    grad_close(got["scales"].T, want["scales"], name=f"{name} scales")
    grad_close(got["quats"].T, want["quats"], name=f"{name} quats", floor=quat_floor(sc, c, g2d))
    grad_close(got["opacities"], want["opacities"], name=f"{name} opacities")
    grad_close(got["sh"].permute(2, 0, 1), want["sh"], name=f"{name} sh")


@pytest.mark.parametrize("name", list(CASES))
def test_statistics_match_oracle(name):
    sc, cam, _, g = _case(name)
    g2d = g["grad2d"].to(F64)
    vis = g["tiles_touched"] > 0
    pos, col = obw.densification_stats(g2d, vis, cam.width, cam.height)
    assert torch.equal(g["visible"].bool(), vis)
    np.testing.assert_allclose(g["pos_stat"].numpy(), pos.numpy(), rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(g["col_stat"].numpy(), col.numpy(), rtol=1e-5, atol=1e-12)


@pytest.mark.parametrize("name", list(CASES))
def test_l1_gradient_matches_oracle(name):
    """Stage a6 element by element: the loss gradient the HIP path computed
    from its own image, against the oracle's from the same image."""
    sc, cam, tgt, g = _case(name)
    rel = l1_matches_oracle(g["image"], g["dL"], g["loss"][0], tgt, g["grid"], name)
    nz = int((g["dL"] == 0).sum())
    say(f"[gpu] {name}: dL/dimage bit-compatible with the oracle ({g['dL'].numel()} values, "
        f"{nz} zero residuals), loss rel {rel:.1e}")


@pytest.mark.parametrize("name", ["tiny128-d1-T16", "sh3-160x120-d2-o10-T16", "sh2-101x77-d3-o21-T8-bg"])
def test_end_to_end_against_pure_oracle(name):
    """No stage isolation: the whole HIP path against the float64 oracle."""
    sc, cam, tgt, g = _case(name)
    make, d, ox, oy, T, bg = CASES[name]
    o = opipe.forward_backward(sc, cam, tgt, d, ox, oy, T, bg)
    loss = float(g["loss"][0])
    assert abs(loss - float(o["loss"])) <= 1e-5 * float(o["loss"]), (loss, float(o["loss"]))
    keep = ~o["flag"]
    err = (g["image"].to(F64) - o["image"].detach()).abs().amax(0)[keep]
    assert float(err.max()) <= 1e-4
    frac = float((g["last_contrib"].to(torch.int64) != o["last_contrib"]).float().mean())
    say(f"[gpu] {name}: end-to-end last_contrib mismatch fraction {frac:.2e}")
    assert frac < 1e-3
    # gradients, compared on every run: pixels where a float decision sits on
    # its threshold (oracle flags), where the L1 residual's sign differs, or
    # where the walk ended at a different entry take no upstream gradient on
    # either side; both sides then backpropagate the same float32 values
    same = ~o["flag"] & (torch.sign(g["dL"].to(F64)) == torch.sign(o["dL_dimage"])).all(0) & \
        (g["last_contrib"].to(torch.int64) == o["last_contrib"])
    masked = float((~same).float().mean())
    say(f"[gpu] {name}: end-to-end gradient comparison, {masked:.2e} of the pixels masked")
    assert masked < 0.01
    dL = (o["dL_dimage"] * same.to(F64)[None]).to(torch.float32).contiguous()
    om = opipe.forward_backward(sc, cam, tgt, d, ox, oy, T, bg, dL_dimage=dL.to(F64))
    view, dev = g["_view"], g["_dev"]
    grads = view.backward(dev, dL.cuda())
    torch.cuda.synchronize()
    compared = 0
    qfloor = quat_floor(sc, cam, om["g2d"])
    for k, shape_fn in (("means", lambda t: t.T), ("scales", lambda t: t.T),
                        ("quats", lambda t: t.T), ("opacities", lambda t: t),
                        ("sh", lambda t: t.permute(2, 0, 1))):
        grad_close(shape_fn(getattr(grads, k).cpu()), om["grads"][k], name=f"{name} e2e {k}",
                   floor=qfloor if k == "quats" else None)
        compared += 1
    assert compared == 5


# ---- closed forms and degenerate inputs through the whole HIP path --------

def _scene(means, scales, quats, opac, rgb):
    means = np.asarray(means, np.float32).reshape(3, -1)
    n = means.shape[1]
    rgb = np.asarray(rgb, np.float64).reshape(3, n)
    sh = ((rgb - 0.5) * 2.0 * math.sqrt(math.pi))[None].astype(np.float32)
    return scenes.Scene(means, np.asarray(scales, np.float32).reshape(3, n),
                        np.asarray(quats, np.float32).reshape(4, n),
                        np.asarray(opac, np.float32).reshape(n), sh, 0)


def test_single_gaussian_peak_is_opacity_times_colour():
    cam = scenes.identity_camera(65, 49, 65.0)           # centre pixel (32, 24)
    sc = _scene([0, 0, 3.0], [0.05] * 3, [1, 0, 0, 0], [0.7], [0.2, 0.6, 0.9])
    g = run_gpu(sc, cam, backward=False)
    np.testing.assert_allclose(g["image"][:, 24, 32].numpy(), 0.7 * np.array([0.2, 0.6, 0.9]),
                               atol=2e-6)
    sc = _scene([0, 0, 3.0], [0.05] * 3, [1, 0, 0, 0], [1.0], [0.2, 0.6, 0.9])
    g = run_gpu(sc, cam, backward=False)
    np.testing.assert_allclose(g["image"][:, 24, 32].numpy(), 0.99 * np.array([0.2, 0.6, 0.9]),
                               atol=2e-6)


def test_saturation_stops_before_fourth_splat():
    cam = scenes.identity_camera(65, 49, 65.0)
    z = [2.0, 2.5, 3.0, 3.5]
    cols = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0], [1.0, 1.0, 1.0]]).T
    sc = _scene([[0] * 4, [0] * 4, z], [[0.05] * 4] * 3, [[1] * 4, [0] * 4, [0] * 4, [0] * 4],
                [0.95] * 4, cols)
    g = run_gpu(sc, cam, backward=False)
    want = np.array([0.95, 0.0475, 0.002375])
    np.testing.assert_allclose(g["image"][:, 24, 32].numpy(), want, atol=2e-6)
    assert int(g["last_contrib"][24, 32]) == 3 and int(g["n_eval"][24, 32]) == 4
    assert abs(float(g["t_final"][24, 32]) - 1.25e-4) < 1e-8


def test_empty_scene_renders_background():
    cam = scenes.identity_camera(40, 30, 40.0)
    sc = _scene(np.zeros((3, 0)), np.zeros((3, 0)), np.zeros((4, 0)), np.zeros(0), np.zeros((3, 0)))
    bg = (0.25, 0.5, 0.75)
    g = run_gpu(sc, cam, bg=bg, target=np.zeros((3, 30, 40), np.float32))
    for c in range(3):
        assert float((g["image"][c] - bg[c]).abs().max()) == 0.0
    assert g["pair_count"] == 0
    assert abs(float(g["loss"][0]) - np.mean(bg)) < 1e-7


def test_all_culled_and_zero_opacity():
    cam = scenes.identity_camera(48, 32, 48.0)
    n = 50
    rng = np.random.default_rng(0)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-3, 0.19, n)])
    sc = _scene(means, np.full((3, n), 0.1), np.tile([[1], [0], [0], [0]], n), np.full(n, 0.5),
                np.full((3, n), 0.5))
    g = run_gpu(sc, cam, target=np.ones((3, 32, 48), np.float32))
    assert g["pair_count"] == 0 and float(g["image"].abs().max()) == 0.0
    for k, v in g["grads"].items():
        assert float(v.abs().max()) == 0.0, k
    means[2] = rng.uniform(2, 4, n)
    sc = _scene(means, np.full((3, n), 0.1), np.tile([[1], [0], [0], [0]], n), np.zeros(n),
                np.full((3, n), 0.5))
    g = run_gpu(sc, cam, target=np.ones((3, 32, 48), np.float32))
    assert g["pair_count"] > 0 and float(g["image"].abs().max()) == 0.0
    assert float(g["grads"]["means"].abs().max()) == 0.0
    assert float(g["grads"]["sh"].abs().max()) == 0.0


def test_non_finite_gaussians_are_culled():
    sc, cam, tgt = _small(8, 60, 64, 48, 1)
    sc.means[0, 3] = np.nan
    sc.scales[1, 7] = np.inf
    sc.sh[2, 1, 11] = np.nan
    g = run_gpu(sc, cam, target=tgt)
    rec = records_to_oracle(g["records"])
    assert bool(rec["culled"][[3, 7, 11]].all())
    assert g["_view"].nonfinite_count() == 3
    assert bool(torch.isfinite(g["image"]).all())
    for k, v in g["grads"].items():
        assert bool(torch.isfinite(v).all()), k


def test_capacity_growth_and_error():
    """A workspace too small for the pairs reports TGS_ERR_CAPACITY with the count."""
    from gpu_helpers import ctx
    from paper_2412_13547_amd import api
    sc, cam, tgt = _small(9, 200, 128, 96, 0)
    dev = api.DeviceScene.from_scene(sc)
    view = api.View(ctx(), sc.n, cam, pair_capacity=16)
    view.preprocess_fwd(dev)
    with pytest.raises(api.TgsError) as e:
        view.bin_sort(dev, grow=False)
    assert e.value.status == api.TGS_ERR_CAPACITY
    need = int(view.state.pair_count)
    assert need > 16
    img = view.forward(dev)       # grows and re-runs
    torch.cuda.synchronize()
    assert int(view.state.pair_count) == need and view.state.pair_capacity >= need
    assert bool(torch.isfinite(img).all())


def test_pair_count_past_32_bits_is_reported_not_wrapped():
    """1025 Gaussians that each cover all 4,194,304 tiles of a 1024 x 4096
    tile grid (8192 x 32768 pixels, T = 8) make 1025 * 2^22 pairs, more than
    a uint32 counts.  The device count saturates instead of wrapping (a
    wrapped count, 2^22, would pass the capacity check and the emission
    would write past the buffers): the synchronous bin/sort and the
    asynchronous one with its later readback both report
    TGS_ERR_UNSUPPORTED, and the asynchronous one leaves every range empty."""
    from gpu_helpers import ctx
    from paper_2412_13547_amd import api
    n = 1025
    cam = scenes.identity_camera(8192, 32768, 8192.0)
    sc = _scene(np.tile([[0.0], [0.0], [3.0]], n), np.full((3, n), 4.0), np.tile([[1], [0], [0], [0]], n),
                np.full(n, 0.5), np.full((3, n), 0.5))
    dev = api.DeviceScene.from_scene(sc)
    for sync in (True, False):
        view = api.View(ctx(), n, cam, 1, 0, 0, 8, pair_capacity=5_000_000, sync_check=sync)
        assert (view.sizes.grid_x, view.sizes.grid_y) == (1024, 4096)
        view.preprocess_fwd(dev)
        touched = view.tiles_touched().cpu().to(torch.int64)
        assert int(touched.sum()) == n * (1 << 22) >= (1 << 32)
        say(f"[gpu] {n * (1 << 22)} pairs requested (sync={sync})")
        with pytest.raises(api.TgsError) as e:
            view.bin_sort(dev, grow=False)
            view.pair_count()
        assert e.value.status == api.TGS_ERR_UNSUPPORTED
        assert int(view.state.pair_count) == (1 << 32) - 1
        if not sync:
            assert int(view.ranges().abs().max()) == 0
    torch.cuda.synchronize()
