"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare each stage with the CPU oracle fed the HIP path's own upstream
outputs (stage isolation)."""
from __future__ import annotations

import sys

import numpy as np
import torch

from oracle import backward as obw
from oracle import binning as obn
from oracle import loss as ols
from oracle import preprocess as opre
from oracle import raster as ors
from paper_2412_13547_amd import api

F64 = torch.float64
_CTX = None


def ctx() -> api.Context:
    global _CTX
    if _CTX is None:
        _CTX = api.Context(0)
    return _CTX


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(scene, cam, stride=1, off_x=0, off_y=0, tile=16, bg=(0.0, 0.0, 0.0), target=None,
            dL_dimage=None, backward=True, lds_batch=0, pixels_per_thread=0):
    """Forward (+ loss + backward) on cuda:0; every result copied to the host."""
    dev = api.DeviceScene.from_scene(scene)
    view = api.View(ctx(), scene.n, cam, stride, off_x, off_y, tile, bg, lds_batch=lds_batch,
                    pixels_per_thread=pixels_per_thread)
    shape = view.image_shape
    image = torch.empty(shape, dtype=torch.float32, device="cuda")
    tfin = torch.empty(shape[1:], dtype=torch.float32, device="cuda")
    last = torch.empty(shape[1:], dtype=torch.int32, device="cuda")
    neval = torch.empty(shape[1:], dtype=torch.int32, device="cuda")
    nblend = torch.empty(shape[1:], dtype=torch.int32, device="cuda")
    view.forward(dev, image, t_final=tfin, last_contrib=last, n_eval=neval, n_blend=nblend)
    out = dict(view=view, image=image, t_final=tfin, last_contrib=last, n_eval=neval,
               n_blend=nblend)
    if backward:
        if dL_dimage is None:
            tgt = torch.as_tensor(np.asarray(target, np.float32)).cuda()
            dL, loss = view.l1_grad(image, tgt)
            out["loss"] = loss
        else:
            dL = torch.as_tensor(np.asarray(dL_dimage, np.float32)).cuda().reshape(shape)
        n = scene.n
        pos = torch.empty(n, dtype=torch.float32, device="cuda")
        col = torch.empty(n, dtype=torch.float32, device="cuda")
        vis = torch.empty(n, dtype=torch.uint8, device="cuda")
        grads = view.backward(dev, dL, pos_stat=pos, col_stat=col, visible=vis)
        out.update(dL=dL, grads=grads, pos_stat=pos, col_stat=col, visible=vis)
    torch.cuda.synchronize()
    host = {}
    for k, v in list(out.items()):
        if isinstance(v, torch.Tensor):
            host[k] = v.cpu()
    host["records"] = view.records().cpu()
    host["tiles_touched"] = view.tiles_touched().cpu()
    host["pair_vals"] = view.pair_vals().cpu()
    host["ranges"] = view.ranges().cpu()
    host["pair_count"] = int(view.state.pair_count)
    host["grid"] = obn.grid(cam.width, cam.height, stride, off_x, off_y, tile)
    host["_view"], host["_dev"], host["_image"] = view, dev, image
    host["bg"] = bg
    if backward:
        host["grad2d"] = view.grad2d().cpu()
        g = out["grads"]
        host["grads"] = {k: getattr(g, k).cpu() for k in ("means", "scales", "quats", "opacities", "sh")}
    return host


def records_to_oracle(rec32: torch.Tensor) -> dict:
    """GPU float32 records -> the oracle's float64 record dict (exact upcast)."""
    r = rec32.to(F64)
    bits = rec32.view(torch.int32)
    flags = bits[:, 11]
    return dict(u=r[:, 0], v=r[:, 1], A=r[:, 2], B=r[:, 3], C=r[:, 4], opacity=r[:, 5],
                rgb=r[:, 6:9].clone(), z=r[:, 9], radius=bits[:, 10].to(torch.int64),
                culled=(flags & 8) != 0, clamp=torch.stack([(flags >> c) & 1 != 0 for c in range(3)], 1),
                fovx=(flags & 16) != 0, fovy=(flags & 32) != 0)


def quat_floor(scene_or_params, cam, g2d, rel=1e-3) -> torch.Tensor:
    """(N, 4) element allowance for the quaternion gradient.

    An element of dL/dq is g_j/|q| - q_hat_j (q_hat . g)/|q|, with g = dL/dq_hat
    (the gradient w.r.t. the unit quaternion, taken here from the oracle at
    the given 2D gradients ``g2d``): the normalisation's projection subtracts
    the radial part, and the two terms can cancel to far below either.  Each
    side computes g to the bar ``rel`` of its own size, so the difference
    carries rel (|g_j| + |q_hat_j| sum_k |q_hat_k g_k|) / |q|: the bar applied
    to the terms before they cancel, propagated through the projection."""
    p = scene_or_params if isinstance(scene_or_params, opre.Params) else opre.params(scene_or_params)
    c = cam if isinstance(cam, opre.Cam) else opre.camera(cam)
    gq = obw.unit_quaternion_gradient(p, c, torch.as_tensor(g2d).to(F64))
    q = p.quats.detach().to(F64)
    qn = torch.linalg.norm(q, dim=1, keepdim=True)
    qh = q / qn
    terms = (gq.abs() + qh.abs() * (qh.abs() * gq.abs()).sum(1, keepdim=True)) / qn
    return rel * torch.nan_to_num(terms, nan=0.0, posinf=0.0, neginf=0.0)


def grad_close(got: torch.Tensor, want: torch.Tensor, rel=1e-3, name="", floor=None, quiet=False):
    """The gradient bar: per tensor ||d|| / ||g|| <= rel, and per element
    |d| <= rel (|g| + rel max|g|).

    ``floor`` (optional, per element, same shape as ``want``) widens the
    element bound by a rounding allowance derived from the magnitude of the
    terms that cancel in that element; the callers that pass one state its
    derivation.  The worst ratio of |d| to the bound is printed either way."""
    got = got.to(F64).flatten()
    want = want.to(F64).flatten()
    d = (got - want).abs()
    gmax = float(want.abs().max()) if want.numel() else 0.0
    if gmax == 0.0:
        assert (float(got.abs().max()) if got.numel() else 0.0) == 0.0, name
        return 0.0
    nrel = float(torch.linalg.norm(got - want) / torch.linalg.norm(want))
    bound = rel * (want.abs() + rel * gmax)
    plain = float((d / bound).max())
    if floor is not None:
        bound = bound + torch.as_tensor(floor, dtype=F64).flatten()
    ratio = d / bound
    worst = float(ratio.max())
    if not quiet:
        extra = f" ({plain:.3f} of the bar without the allowance)" if floor is not None else ""
        say(f"[grad] {name}: norm-rel {nrel:.2e}, worst element {worst:.3f} of its bound{extra}")
    assert nrel <= rel, f"{name}: norm-relative error {nrel:.3e}"
    bad = ratio > 1.0
    assert not bool(bad.any()), (f"{name}: {int(bad.sum())} elements out of bound, worst "
                                 f"{worst:.3e} of the bound")
    return nrel


def l1_matches_oracle(image, dL, loss, target, grid, label):
    """The L1 stage against ``oracle.loss.l1`` fed the HIP image: the sign of
    every element of dL/dimage exactly, its magnitude 1/(3 pixels) within
    the float32 rounding of that reciprocal, the loss (float64 sum of
    float32 residuals) within 1e-6 relative."""
    want_loss, want = ols.l1(image.to(F64), target, grid)
    got = dL.to(F64)
    assert got.shape == want.shape, label
    assert torch.equal(torch.sign(got), torch.sign(want)), f"{label}: a residual sign differs"
    inv = 1.0 / want.numel()
    assert float((got - want).abs().max()) <= 2.0 ** -22 * inv, label
    rel = abs(float(loss) - float(want_loss)) / float(want_loss)
    assert rel <= 1e-6, (label, rel)
    return rel
