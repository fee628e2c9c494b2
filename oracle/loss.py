"""L1 photometric loss on the rendered pixels (supervision of Fig. 2 / Sec. 4.1).

Each downsampled pixel (i, j) is compared with the full-resolution target pixel
it was rendered at, (d i + o_x, d j + o_y) ("supervision from corresponding
high-resolution pixels").  Reading for the normalisation: the mean over the
rendered pixels and the 3 channels, so the average over the d^2 phases of a
full cycle of offsets equals the full-resolution loss.  sign(0) = 0.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64


def gather_target(target, g) -> torch.Tensor:
    """The full-resolution target pixels that the downsampled image supervises."""
    t = torch.as_tensor(np.asarray(target, dtype=np.float64))
    return t[:, g.off_y::g.stride, g.off_x::g.stride][:, :g.h_ds, :g.w_ds]


def l1(image: torch.Tensor, target, g):
    """(loss, dL/dimage) with image planar [3][H_ds][W_ds]."""
    gt = gather_target(target, g)
    diff = image - gt
    n = diff.numel()
    loss = diff.abs().sum() / n
    grad = torch.sign(diff.detach()) / n
    return loss, grad
