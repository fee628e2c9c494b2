"""torch.autograd bindings of the rasterizer: Gaussian parameters in, dilated
image out, with the hand-written backward of libtgs behind ``backward``.

Argument marshalling only -- every stage runs in the HIP library:

* ``rasterize(view, means, scales, quats, opacities, sh)`` -> image
  [3][H_ds][W_ds] of one view (camera + dilation pattern).  The backward
  walks every pixel's list back to front from the final transmittance and
  last blended entry the forward left in the view's workspace (8 bytes per
  pixel), recovering the transmittance in front of every entry by division.
  The records, pair lists and that per-pixel state are reused if the
  workspace still holds them; otherwise (``recompute=True``, or another
  forward ran on the same view in between) the backward re-derives them
  from the saved parameters first (a forward pass without the image).
* ``l1_loss(view, image, target)`` -> scalar L1 loss of the rendered pixels
  against the full-resolution target (Sec. 4.1); its gradient comes from the
  same kernel call.
* ``rasterize_batch(batch, ...)`` -> one image per view of a ``Batch``; the
  backward is one batched call, so the parameter gradients of all views are
  summed on the device.

Gradients are with respect to the arguments as passed: scales after the
exponential, opacities after the sigmoid, raw quaternions.  Densification
statistics of each backward are accumulated into an optional ``Stats``.
"""
from __future__ import annotations

import torch

from . import api

__all__ = ["Stats", "rasterize", "l1_loss", "rasterize_batch"]


class Stats:
    """Running sums of the densification statistics of Sec. 4.3 over backward
    passes: positional-gradient norm, appearance-gradient norm and the number
    of views in which each Gaussian was visible."""

    def __init__(self, n: int, device="cuda"):
        self.pos = torch.zeros(n, dtype=torch.float32, device=device)
        self.col = torch.zeros(n, dtype=torch.float32, device=device)
        self.count = torch.zeros(n, dtype=torch.int32, device=device)
        self._pos = torch.empty_like(self.pos)
        self._col = torch.empty_like(self.col)
        self._vis = torch.empty(n, dtype=torch.uint8, device=device)

    def buffers(self):
        return self._pos, self._col, self._vis

    def accumulate(self):
        self.pos += self._pos
        self.col += self._col
        self.count += self._vis

    def reset(self):
        self.pos.zero_()
        self.col.zero_()
        self.count.zero_()


def _scene(sh_degree, means, scales, quats, opacities, sh):
    c = lambda t: t.detach().contiguous()
    return api.DeviceScene(c(means), c(scales), c(quats), c(opacities), c(sh), int(sh_degree))


class _Rasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, view, sh_degree, stats, recompute, means, scales, quats, opacities, sh):
        dev = _scene(sh_degree, means, scales, quats, opacities, sh)
        image = torch.empty(view.image_shape, dtype=torch.float32, device=means.device)
        view.forward(dev, image)
        ctx.view, ctx.sh_degree, ctx.stats, ctx.recompute = view, sh_degree, stats, recompute
        ctx.generation = view.generation
        ctx.save_for_backward(dev.means, dev.scales, dev.quats, dev.opacities, dev.sh)
        return image

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, dL):
        means, scales, quats, opacities, sh = ctx.saved_tensors
        view = ctx.view
        dev = api.DeviceScene(means, scales, quats, opacities, sh, ctx.sh_degree)
        if ctx.recompute or view.generation != ctx.generation:
            view.preprocess_fwd(dev)
            view.bin_sort(dev)
            view.raster_fwd(None)
        grads = api.DeviceScene(*(torch.empty_like(t) for t in (means, scales, quats, opacities,
                                                                  sh)), ctx.sh_degree)
        bufs = ctx.stats.buffers() if ctx.stats is not None else (None, None, None)
        view.backward(dev, dL.contiguous(), grads, *bufs)
        if ctx.stats is not None:
            ctx.stats.accumulate()
        return (None, None, None, None, grads.means, grads.scales, grads.quats, grads.opacities,
                grads.sh)


def rasterize(view: api.View, means, scales, quats, opacities, sh, sh_degree: int | None = None,
              stats: Stats | None = None, recompute: bool = False):
    """Dilated image of one view; differentiable in all five parameter tensors.

    Shapes: means/scales [3][n], quats [4][n], opacities [n], sh [K][3][n]
    (K >= (degree+1)^2), float32 on the device."""
    deg = int(sh_degree) if sh_degree is not None else int(round(sh.shape[0] ** 0.5)) - 1
    return _Rasterize.apply(view, deg, stats, bool(recompute), means, scales, quats, opacities, sh)


class _L1(torch.autograd.Function):
    @staticmethod
    def forward(ctx, view, image, target):
        dL = torch.empty_like(image)
        loss = torch.empty(1, dtype=torch.float64, device=image.device)
        view.l1_grad(image.contiguous(), target, dL, loss)
        ctx.save_for_backward(dL)
        return loss[0]

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g):
        (dL,) = ctx.saved_tensors
        return None, dL * g.to(dL.dtype), None


def l1_loss(view: api.View, image, target):
    """Mean |image - target| over the rendered pixels and channels (float64
    scalar); target is the full-resolution [3][H][W] float32 image."""
    return _L1.apply(view, image, target)


class _RasterizeBatch(torch.autograd.Function):
    @staticmethod
    def forward(ctx, batch, sh_degree, stats, means, scales, quats, opacities, sh):
        dev = _scene(sh_degree, means, scales, quats, opacities, sh)
        batch.forward(dev)
        ctx.generation = batch.generation
        ctx.batch, ctx.sh_degree, ctx.stats = batch, sh_degree, stats
        images = tuple(t.clone() for t in batch.images)
        ctx.save_for_backward(dev.means, dev.scales, dev.quats, dev.opacities, dev.sh)
        ctx.shapes = [t.shape for t in images]
        return images

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, *dLs):
        means, scales, quats, opacities, sh = ctx.saved_tensors
        b = ctx.batch
        dev = api.DeviceScene(means, scales, quats, opacities, sh, ctx.sh_degree)
        # when a later forward has overwritten the workspaces, rebuild the
        # binning and per-pixel state from the saved parameters (the images
        # it writes into the batch's own buffers are the same)
        if b.generation != ctx.generation:
            b.forward(dev)
        keep = []
        io = b.io
        old = [io[k].dL_dimage for k in range(b.nv)]
        for k in range(b.nv):
            d = dLs[k] if dLs[k] is not None else torch.zeros(ctx.shapes[k], dtype=torch.float32,
                                                              device=means.device)
            d = d.contiguous()
            keep.append(d)
            io[k].dL_dimage = d.data_ptr()
        grads = api.DeviceScene(*(torch.empty_like(t) for t in (means, scales, quats, opacities,
                                                                  sh)), ctx.sh_degree)
        bufs = ctx.stats.buffers() if ctx.stats is not None else (None, None, None)
        try:
            b.backward(dev, grads, *bufs)
        finally:
            for k, dl in enumerate(old):
                io[k].dL_dimage = dl
        if ctx.stats is not None:
            ctx.stats.accumulate()
        return (None, None, None, grads.means, grads.scales, grads.quats, grads.opacities,
                grads.sh)


def rasterize_batch(batch: api.Batch, means, scales, quats, opacities, sh,
                    sh_degree: int | None = None, stats: Stats | None = None):
    """One dilated image per view of ``batch``; the backward sums the
    parameter gradients of all views in one batched call."""
    deg = int(sh_degree) if sh_degree is not None else int(round(sh.shape[0] ** 0.5)) - 1
    return _RasterizeBatch.apply(batch, deg, stats, means, scales, quats, opacities, sh)
