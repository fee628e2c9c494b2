"""Densification selection of Sec. 4.3 from accumulated statistics, written
out plainly (test infrastructure only, see the package header).

A Gaussian seen by at least one view is a candidate when its mean
positional-gradient norm reaches tau_pos, or, in events where the appearance
branch is active, its mean appearance-gradient norm reaches tau_col.  Under a
budget K only the K candidates with the largest score
max(mean_pos / tau_pos, mean_col / tau_col) remain, equal scores in
ascending index.  The decisions are taken in float32, as the kernels take
them (IEEE division).
"""
from __future__ import annotations

import numpy as np


def select(pos_sum, col_sum, count, tau_pos: float, tau_col: float, color_active: bool,
           budget: int = -1):
    """Returns (mask uint8 [n], number selected)."""
    pos = np.asarray(pos_sum, np.float32)
    cnt = np.asarray(count, np.int64)
    n = pos.shape[0]
    tp = np.float32(tau_pos)
    mask = np.zeros(n, np.uint8)
    scores = np.zeros(n, np.float32)
    for i in range(n):
        if cnt[i] <= 0:
            continue
        c = np.float32(cnt[i])
        ap = np.float32(pos[i] / c)
        cand = bool(ap >= tp)
        score = np.float32(ap / tp)
        if color_active:
            ac = np.float32(np.float32(col_sum[i]) / c)
            tc = np.float32(tau_col)
            cand = cand or bool(ac >= tc)
            score = max(score, np.float32(ac / tc))
        mask[i] = 1 if cand else 0
        scores[i] = score
    cands = [i for i in range(n) if mask[i]]
    if budget < 0 or len(cands) <= budget:
        return mask, len(cands)
    # largest score first, ties in ascending index
    order = sorted(cands, key=lambda i: (-float(scores[i]), i))
    keep = np.zeros(n, np.uint8)
    keep[order[:budget]] = 1
    return keep, budget
