"""torch.autograd layer: gradients through ``rasterize`` / ``l1_loss`` equal
the direct C-ABI backward; recomputation and interleaved forwards give the
same gradients; the batched function sums views; a 200-iteration fit follows
the oracle's own fit (float64, same optimiser) iteration by iteration."""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import ctx, grad_close, quat_floor, run_gpu, say
from oracle import pipeline as opipe
from paper_2412_13547_amd import api, autograd, scenes

pytestmark = pytest.mark.gpu
F64 = torch.float64
PARAMS = ("means", "scales", "quats", "opacities", "sh")


def _leaves(sc):
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).cuda().requires_grad_(True)
    return [f(getattr(sc, k)) for k in PARAMS]


def _case():
    sc, cam = scenes.small_scene(1, 300, 160, 120, sh_degree=3)
    tgt = scenes.target_image(160, 120, 501)
    return sc, cam, tgt


def test_autograd_matches_direct_backward():
    sc, cam, tgt = _case()
    ref = run_gpu(sc, cam, 2, 1, 0, 16, target=tgt)
    view = api.View(ctx(), sc.n, cam, 2, 1, 0, 16)
    leaves = _leaves(sc)
    stats = autograd.Stats(sc.n)
    img = autograd.rasterize(view, *leaves, sh_degree=3, stats=stats)
    loss = autograd.l1_loss(view, img, torch.as_tensor(tgt).cuda())
    loss.backward()
    torch.cuda.synchronize()
    assert torch.equal(img.detach().cpu(), ref["image"])
    assert abs(float(loss) - float(ref["loss"].item())) <= 1e-12 * float(loss)
    qfloor = quat_floor(sc, cam, ref["grad2d"])
    for k, t in zip(PARAMS, leaves):
        grad_close(t.grad.cpu(), ref["grads"][k].to(F64), name=f"autograd {k}",
                   floor=qfloor.T if k == "quats" else None)
    assert torch.equal(stats.count.cpu().to(torch.uint8), ref["visible"])
    grad_close(stats.pos.cpu(), ref["pos_stat"].to(F64), name="pos_stat")


@pytest.mark.parametrize("mode", ["recompute", "interleaved"])
def test_recomputation_gives_the_same_gradients(mode):
    sc, cam, tgt = _case()
    target = torch.as_tensor(tgt).cuda()
    view = api.View(ctx(), sc.n, cam, 2, 1, 0, 16)
    base = _leaves(sc)
    loss = autograd.l1_loss(view, autograd.rasterize(view, *base, sh_degree=3), target)
    loss.backward()
    leaves = _leaves(sc)
    if mode == "recompute":
        img = autograd.rasterize(view, *leaves, sh_degree=3, recompute=True)
    else:
        img = autograd.rasterize(view, *leaves, sh_degree=3)
        # another forward on the same view, with other parameters, before the backward
        other = sc.copy()
        other.means = other.means + np.float32(0.05)
        with torch.no_grad():
            autograd.rasterize(view, *[t.detach() for t in _leaves(other)], sh_degree=3)
    autograd.l1_loss(view, img, target).backward()
    qfloor = quat_floor(sc, cam, view.grad2d().cpu())
    for k, a, b in zip(PARAMS, leaves, base):
        grad_close(a.grad.cpu(), b.grad.cpu().to(F64), name=f"{mode} {k}",
                   floor=qfloor.T if k == "quats" else None)


def test_batched_autograd_sums_views():
    sc, cams = scenes.small_multiview(7, 400, [(160, 120), (96, 64), (200, 150)], sh_degree=3)
    specs = [(cams[0], 2, 1, 0), (cams[1], 1, 0, 0), (cams[2], 4, 3, 2)]
    targets = [torch.as_tensor(scenes.target_image(c.width, c.height, 900 + k)).cuda()
               for k, c in enumerate(cams)]
    b = api.Batch(ctx(), sc.n, specs, tile=16)
    b.set_targets(targets)
    dev = api.DeviceScene.from_scene(sc)
    b.fit_capacity(dev)
    leaves = _leaves(sc)
    imgs = autograd.rasterize_batch(b, *leaves, sh_degree=3)
    total = sum(autograd.l1_loss(b.views[k], imgs[k], targets[k]) for k in range(3))
    total.backward()
    ref = dev.zeros_like()
    b.step(dev, ref)
    torch.cuda.synchronize()
    assert abs(float(total) - float(b.loss.sum())) <= 1e-12 * float(total)
    qfloor = sum(quat_floor(sc, cams[k], b.views[k].grad2d().cpu()) for k in range(3))
    for k, t in zip(PARAMS, leaves):
        grad_close(t.grad.cpu(), getattr(ref, k).cpu().to(F64), name=f"batch autograd {k}",
                   floor=qfloor.T if k == "quats" else None)


def _perturbed(sc, seed):
    rng = np.random.default_rng(seed)
    p = sc.copy()
    p.means = (p.means + rng.normal(0, 0.03, p.means.shape)).astype(np.float32)
    p.scales = (p.scales * np.exp(rng.normal(0, 0.15, p.scales.shape))).astype(np.float32)
    lo = np.log(p.opacities / (1 - p.opacities)) + rng.normal(0, 0.4, p.opacities.shape)
    p.opacities = (1 / (1 + np.exp(-lo))).astype(np.float32)
    p.sh = (p.sh + rng.normal(0, 0.08, p.sh.shape)).astype(np.float32)
    return p


LR = dict(means=2e-4, log_scales=2e-3, quats=5e-4, logit=5e-3, sh=2e-3)


def _fit_gpu(sc, cam, target, iters, T):
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).cuda()
    P = dict(means=dev(sc.means), log_scales=dev(np.log(sc.scales)), quats=dev(sc.quats),
             logit=dev(np.log(sc.opacities / (1 - sc.opacities))), sh=dev(sc.sh))
    for t in P.values():
        t.requires_grad_(True)
    opt = torch.optim.Adam([{"params": [P[k]], "lr": LR[k]} for k in LR], eps=1e-15)
    view = api.View(ctx(), sc.n, cam, 2, 0, 0, T)
    tg = torch.as_tensor(target).cuda()
    losses = []
    for k in range(iters):
        view.set_offsets(*scenes.phase_offsets(k, 2))
        img = autograd.rasterize(view, P["means"], torch.exp(P["log_scales"]), P["quats"],
                                 torch.sigmoid(P["logit"]), P["sh"], sh_degree=sc.sh_degree)
        loss = autograd.l1_loss(view, img, tg)
        opt.zero_grad()
        loss.backward()
        opt.step()
        losses.append(float(loss))
    return losses


def _fit_oracle(sc, cam, target, iters, T, probe=None, probe_every=20):
    t64 = lambda a: torch.as_tensor(np.asarray(a, np.float64)).clone()
    P = dict(means=t64(sc.means), log_scales=t64(np.log(sc.scales)), quats=t64(sc.quats),
             logit=t64(np.log(sc.opacities.astype(np.float64) / (1 - sc.opacities))), sh=t64(sc.sh))
    opt = torch.optim.Adam([{"params": [P[k]], "lr": LR[k]} for k in LR], eps=1e-15)
    losses = []
    for k in range(iters):
        ox, oy = scenes.phase_offsets(k, 2)
        o = torch.sigmoid(P["logit"])
        s = torch.exp(P["log_scales"])
        scene = scenes.Scene(P["means"].numpy(), s.numpy(), P["quats"].numpy(), o.numpy(),
                             P["sh"].numpy(), sc.sh_degree)
        res = opipe.forward_backward(scene, cam, target, 2, ox, oy, T)
        g = res["grads"]
        if probe is not None and k % probe_every == 0:
            probe(k, scene, (ox, oy), g)
        P["means"].grad = g["means"].T.contiguous()
        P["log_scales"].grad = (g["scales"].T * s).contiguous()
        P["quats"].grad = g["quats"].T.contiguous()
        P["logit"].grad = g["opacities"] * o * (1 - o)
        P["sh"].grad = g["sh"].permute(1, 2, 0).contiguous()
        opt.step()
        losses.append(float(res["loss"]))
    return losses


def test_200_iteration_fit_follows_the_oracle():
    """Fit a 64-Gaussian scene (64x64, stride 2, phases cycling) to a target
    the oracle renders from a perturbed copy.

    Teacher-forced: every 20 iterations the HIP path's gradients, taken at the
    oracle's own parameters of that iteration, match the oracle's (1e-3 of
    the norm).  Free-running: the two loss curves agree to 1e-3 over the first
    50 iterations and stay within a 3e-2 band to 200; near convergence the
    sign-dominated L1 gradient amplifies float32 rounding of the trajectory
    chaotically (1e-2 has been observed), so the late band is looser."""
    sc, cam = scenes.small_scene(11, 64, 64, 64, sh_degree=3)
    T = 8
    pert = _perturbed(sc, 12)
    target = np.ascontiguousarray(opipe.forward(pert, cam, 1, 0, 0, T)["image"].numpy(),
                                  dtype=np.float32)
    iters = 200
    gl = _fit_gpu(sc, cam, target, iters, T)
    say(f"[gpu] fit: HIP loss {gl[0]:.6f} -> {gl[-1]:.6f}")
    view = api.View(ctx(), sc.n, cam, 2, 0, 0, T)
    tg = torch.as_tensor(target).cuda()
    worst = []

    def probe(k, scene, offs, g_oracle):
        view.set_offsets(*offs)
        leaves = _leaves(scene)
        img = autograd.rasterize(view, *leaves, sh_degree=scene.sh_degree)
        autograd.l1_loss(view, img, tg).backward()
        want = dict(means=g_oracle["means"].T, scales=g_oracle["scales"].T,
                    quats=g_oracle["quats"].T, opacities=g_oracle["opacities"],
                    sh=g_oracle["sh"].permute(1, 2, 0))
        for name, t in zip(PARAMS, leaves):
            got = t.grad.cpu().to(F64)
            rel = float(torch.linalg.norm(got - want[name]) / torch.linalg.norm(want[name]))
            worst.append(rel)
            assert rel <= 1e-3, (k, name, rel)

    ol = _fit_oracle(sc, cam, target, iters, T, probe=probe)
    rel = [abs(a - b) / b for a, b in zip(gl, ol)]
    say(f"[gpu] fit: oracle loss {ol[0]:.6f} -> {ol[-1]:.6f}; max rel diff {max(rel):.2e} "
        f"(first 50: {max(rel[:50]):.2e}); teacher-forced gradients: worst {max(worst):.2e} "
        f"over {len(worst)} checks")
    assert gl[-1] < 0.8 * gl[0] and ol[-1] < 0.8 * ol[0]
    assert max(rel[:50]) <= 1e-3
    assert max(rel) <= 3e-2
    assert not any(math.isnan(x) for x in gl)


def test_binding_refuses_strided_and_host_tensors():
    sc, cam, tgt = _case()
    view = api.View(ctx(), sc.n, cam, 2, 1, 0, 16)
    img = autograd.rasterize(view, *[t.detach() for t in _leaves(sc)], sh_degree=3)
    hwc = torch.as_tensor(np.ascontiguousarray(tgt.transpose(1, 2, 0))).cuda().permute(2, 0, 1)
    with pytest.raises(ValueError, match="contiguous"):
        autograd.l1_loss(view, img, hwc)
    with pytest.raises(ValueError, match="device memory"):
        autograd.l1_loss(view, img, torch.as_tensor(tgt))
