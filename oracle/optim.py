"""Adam (Kingma & Ba, 2015, Algorithm 1) in float64: the optimiser of the
fitting loop that follows the backward (Tab. 2 of the paper trains with the
3DGS recipe, whose optimiser is Adam).

Test infrastructure only (see the package header).
"""
from __future__ import annotations

import torch

F64 = torch.float64


def adam_step(p, g, m, v, t: int, lr: float, beta1: float, beta2: float, eps: float):
    """One update at step t (1-based).  Returns the new (p, m, v), float64.

    m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
    p <- p - lr * mhat / (sqrt(vhat) + eps) with mhat = m / (1 - b1^t),
    vhat = v / (1 - b2^t)."""
    p, g, m, v = (torch.as_tensor(x, dtype=F64) for x in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    p = p - lr * mhat / (torch.sqrt(vhat) + eps)
    return p, m, v
