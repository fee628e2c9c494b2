"""Gradients of the rendered image and the per-Gaussian densification statistics.

The paper trains by backpropagating the photometric loss through the
rasterizer (Sec. 3: densification follows "the accumulated gradient"; Sec. 5.1
uses an optimised backward kernel from prior work without describing it).  The
gradient has a plain definition: the derivative of the forward.  It is obtained
here by reverse-mode differentiation of ``oracle.raster`` and
``oracle.preprocess`` in float64; the skip / stop / clamp decisions are
piecewise-constant, so their derivative is zero, and the alpha clamp at 0.99
passes no gradient where o exp(p) > 0.99.

Two stages, matching the split of the HIP path:
  raster stage:     dL/d(u, v, A, B, C, o, r, g, b) per Gaussian, summed over
                    all rendered pixels (9 values, this column order);
  preprocess stage: chain rule from those 9 values to means, scales,
                    quaternions, opacities and SH coefficients.

Densification statistics (Sec. 4.3, position- and appearance-gradient
thresholds).  Readings: the positional statistic is the norm of the
view-space 2D-mean gradient in normalised device units,
|| (dL/du * W / 2, dL/dv * H / 2) ||, with the full-resolution W, H; the
appearance statistic is the norm of the gradient w.r.t. the blended colour,
|| dL/d(r, g, b) ||.  Both are per view and zero for Gaussians that touch no
tile.
"""
from __future__ import annotations

import torch

from . import preprocess as pre
from . import raster

F64 = torch.float64
G2D_FIELDS = ("u", "v", "A", "B", "C", "opacity")


def raster_backward(rec: dict, vals, ranges, g, dL_dimage, bg=(0.0, 0.0, 0.0), tiles=None,
                    chunk: int = 1024) -> torch.Tensor:
    """(N, 9) float64: dL/d(u, v, A, B, C, o, r, g, b)."""
    leaves = {k: rec[k].detach().to(F64).clone().requires_grad_(True)
              for k in G2D_FIELDS + ("rgb",)}
    out = raster.raster_forward(leaves, vals, ranges, g, bg=bg, tiles=tiles, chunk=chunk)
    s = (out["image"] * torch.as_tensor(dL_dimage, dtype=F64)).sum()
    if s.requires_grad:
        s.backward()
    cols = []
    for k in G2D_FIELDS:
        gr = leaves[k].grad
        cols.append(torch.zeros_like(leaves[k]) if gr is None else gr)
    grgb = leaves["rgb"].grad
    if grgb is None:
        grgb = torch.zeros_like(leaves["rgb"])
    return torch.cat([torch.stack(cols, 1), grgb], 1).detach()


def preprocess_backward(p: pre.Params, cam: pre.Cam, g2d: torch.Tensor) -> dict:
    """Chain rule from the 9 per-Gaussian values to the parameters.

    ``p`` must hold leaf tensors with requires_grad.  Returns gradients shaped
    like the (N, .) parameter tensors.
    """
    rec = pre.preprocess(p, cam)
    g2d = torch.as_tensor(g2d, dtype=F64)
    s = sum((rec[k] * g2d[:, j]).sum() for j, k in enumerate(G2D_FIELDS))
    s = s + (rec["rgb"] * g2d[:, 6:9]).sum()
    grads = torch.autograd.grad(s, [p.means, p.scales, p.quats, p.opacities, p.sh],
                                allow_unused=True)
    names = ("means", "scales", "quats", "opacities", "sh")
    ref = (p.means, p.scales, p.quats, p.opacities, p.sh)
    return {n: (torch.zeros_like(r) if gr is None else gr).detach()
            for n, gr, r in zip(names, grads, ref)}


def unit_quaternion_gradient(p: pre.Params, cam: pre.Cam, g2d: torch.Tensor) -> torch.Tensor:
    """(N, 4): dL/dq_hat, the gradient w.r.t. the unit quaternion q_hat = q/|q|
    before the normalisation removes its radial part.

    The parameter gradient is (I - q_hat q_hat^T) dL/dq_hat / |q|, a difference
    of two terms that can nearly cancel; this returns the terms' source so that
    a comparison can size the rounding such a difference carries."""
    with torch.no_grad():
        qn = p.quats.detach() / torch.linalg.norm(p.quats.detach(), dim=1, keepdim=True)
    unit = pre.Params(p.means.detach(), p.scales.detach(), qn.clone().requires_grad_(True),
                      p.opacities.detach(), p.sh.detach(), p.degree)
    rec = pre.preprocess(unit, cam, unit_quats=True)
    g2d = torch.as_tensor(g2d, dtype=F64)
    s = sum((rec[k] * g2d[:, j]).sum() for j, k in enumerate(G2D_FIELDS))
    s = s + (rec["rgb"] * g2d[:, 6:9]).sum()
    (gq,) = torch.autograd.grad(s, [unit.quats], allow_unused=True)
    return torch.zeros_like(qn) if gq is None else gq.detach()


def densification_stats(g2d: torch.Tensor, visible: torch.Tensor, width: int, height: int):
    """(pos, col) per Gaussian, zero where not visible."""
    g2d = torch.as_tensor(g2d, dtype=F64)
    pos = torch.sqrt((g2d[:, 0] * (0.5 * width)) ** 2 + (g2d[:, 1] * (0.5 * height)) ** 2)
    col = torch.linalg.norm(g2d[:, 6:9], dim=1)
    vis = torch.as_tensor(visible, dtype=torch.bool)
    return torch.where(vis, pos, 0.0), torch.where(vis, col, 0.0)
