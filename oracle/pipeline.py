"""The oracle's stages chained end to end: preprocess -> bin -> raster -> L1 -> backward.

One iteration of the paper's dilated fitting loop for one view and one offset
(Sec. 4.1, last paragraph: stride d, one offset per iteration), minus the
optimiser.  Used for end-to-end comparisons, finite-difference pins and the
CPU baseline timing.
"""
from __future__ import annotations

import torch

from . import backward as bw
from . import binning as bn
from . import loss as ls
from . import preprocess as pre
from . import raster as rs

F64 = torch.float64


def forward(scene, cam, stride: int = 1, off_x: int = 0, off_y: int = 0, tile: int = 16,
            bg=(0.0, 0.0, 0.0), p: pre.Params | None = None, tiles=None) -> dict:
    c = pre.camera(cam)
    if p is None:
        p = pre.params(scene)
    rec = pre.preprocess(p, c)
    g = bn.grid(c.width, c.height, stride, off_x, off_y, tile)
    bins = bn.bin_gaussians(rec["u"], rec["v"], rec["z"], rec["radius"], rec["culled"], g)
    out = rs.raster_forward(rec, bins["vals"], bins["ranges"], g, bg=bg, tiles=tiles)
    return dict(rec=rec, bins=bins, grid=g, cam=c, params=p, **out)


def forward_backward(scene, cam, target, stride: int = 1, off_x: int = 0, off_y: int = 0,
                     tile: int = 16, bg=(0.0, 0.0, 0.0), dL_dimage=None) -> dict:
    """Forward, L1 loss (or a given upstream gradient), and all gradients."""
    p = pre.params(scene, requires_grad=True)
    f = forward(scene, cam, stride, off_x, off_y, tile, bg, p=p)
    g = f["grid"]
    loss = None
    if dL_dimage is None:
        loss, dL_dimage = ls.l1(f["image"].detach(), target, g)
    g2d = bw.raster_backward(f["rec"], f["bins"]["vals"], f["bins"]["ranges"], g, dL_dimage, bg=bg)
    grads = bw.preprocess_backward(p, f["cam"], g2d)
    pos, col = bw.densification_stats(g2d, f["bins"]["visible"], f["cam"].width, f["cam"].height)
    return dict(f, loss=loss, dL_dimage=dL_dimage, g2d=g2d, grads=grads, pos_stat=pos,
                col_stat=col)


def image_functional(scene, cam, weights, stride=1, off_x=0, off_y=0, tile=16, bg=(0.0, 0.0, 0.0),
                     p: pre.Params | None = None) -> torch.Tensor:
    """<weights, image>, the scalar used by the finite-difference pins."""
    f = forward(scene, cam, stride, off_x, off_y, tile, bg, p=p)
    return (f["image"] * torch.as_tensor(weights, dtype=F64)).sum()
