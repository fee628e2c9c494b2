"""Densification consumers (Sec. 4.2-4.3, Supp. Alg. 1): the convergence-aware
budget schedule, on the host, and the selection of Gaussians to densify, on
the GPU (``tgs_densify_select``).

Budget (Eq. 7): with N Gaussians at the start of densification and a target
M, the budget at densification progress t in [1, 100] (percent of the
densification window) is

    B(t) = N + (t^a - 1) / (100^a - 1) (M_adaptive - N).

The exponent a follows the convergence of the loss (Eq. 6, Alg. 1): the
loss history is smoothed by an exponential moving average (weight 0.1); after
a warm-up (a = 1) the signed slope of log(ema) against log(step) is fitted
over the whole history (s_hist) and over the most recent window (s_recent);

    eps = s_recent - s_hist,      a = a_base + 0.5 tanh(eps), clipped to [0.1, 2],

where a_base is the moving average of the recent fitted exponents |s_hist|.
A loss that converges more slowly than its power law so far (eps > 0) raises a
and slows the growth of the budget; faster convergence lowers it.  The final
target M_adaptive grows by 10% (at most to 1.5 M) while the recent decline
rate -s_recent exceeds 0.05 and shrinks by 10% (at least to 0.5 M) when the
loss rises faster than that.

Selection (Sec. 4.3): Gaussians whose mean positional-gradient norm reaches
tau_pos, or -- in the 20% of densification events where the appearance branch
is drawn -- whose mean appearance-gradient norm reaches tau_col = 0.01 tau_pos,
keeping at most the budget's remainder, largest normalised score first.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import api

__all__ = ["BudgetSchedule", "Densifier", "COLOR_PROBABILITY", "TAU_COLOR_RATIO"]

COLOR_PROBABILITY = 0.2     # appearance branch drawn in 20% of the events (Sec. 4.3)
TAU_COLOR_RATIO = 0.01      # tau_col = 0.01 tau_pos (Sec. 4.3)


def _slope(steps, values) -> float:
    """Least-squares slope of log(values) against log(steps)."""
    x = np.log(np.asarray(steps, np.float64))
    y = np.log(np.asarray(values, np.float64))
    xm = x - x.mean()
    den = float((xm * xm).sum())
    return float((xm * (y - y.mean())).sum() / den) if den > 0 else 0.0


@dataclasses.dataclass
class BudgetSchedule:
    """Eq. 6-7 and Alg. 1.  ``record`` every iteration's loss; ``budget`` at
    any iteration of the densification window [start, end]."""
    n_init: int
    n_max: int
    start: int
    end: int
    warmup: int = 100
    window: int = 100
    ema_weight: float = 0.1
    lam: float = 0.5
    base_window: int = 5
    rate_threshold: float = 0.05

    def __post_init__(self):
        if not (self.end > self.start and self.n_max >= self.n_init >= 0):
            raise ValueError("need end > start and n_max >= n_init >= 0")
        self.steps: list = []
        self.ema: list = []
        self.bases: list = []
        self.m_adaptive = float(self.n_max)
        self.alpha = 1.0

    def record(self, step: int, loss: float):
        """Add one iteration's loss (step >= 1)."""
        prev = self.ema[-1] if self.ema else loss
        self.steps.append(int(step))
        self.ema.append(self.ema_weight * float(loss) + (1.0 - self.ema_weight) * prev)

    def update(self) -> float:
        """Refit the exponent and the target from the history (Alg. 1)."""
        if len(self.ema) <= self.warmup:
            self.alpha = 1.0
            return self.alpha
        steps, ema = self.steps[self.warmup:], self.ema[self.warmup:]
        s_hist = _slope(steps, ema)
        s_recent = _slope(steps[-self.window:], ema[-self.window:])
        self.bases = (self.bases + [abs(s_hist)])[-self.base_window:]
        base = float(np.mean(self.bases))
        rate = -s_recent
        if rate > self.rate_threshold:
            self.m_adaptive = min(self.m_adaptive * 1.1, 1.5 * self.n_max)
        elif rate < -self.rate_threshold:
            self.m_adaptive = max(self.m_adaptive * 0.9, 0.5 * self.n_max)
        eps = s_recent - s_hist
        self.alpha = min(2.0, max(0.1, base + self.lam * math.tanh(eps)))
        return self.alpha

    def progress(self, step: int) -> float:
        """Densification progress t in [1, 100] (percent of the window)."""
        f = (step - self.start) / (self.end - self.start)
        return 1.0 + 99.0 * min(1.0, max(0.0, f))

    def budget(self, step: int) -> int:
        """B(t) of Eq. 7 at iteration ``step`` with the current exponent."""
        t, a = self.progress(step), self.alpha
        frac = (t - 1.0) / 99.0 if abs(a - 1.0) < 1e-12 else (t ** a - 1.0) / (100.0 ** a - 1.0)
        return int(round(self.n_init + frac * (self.m_adaptive - self.n_init)))


class Densifier:
    """One densification event: the budget's remainder, the appearance-branch
    draw and the GPU selection from accumulated statistics (``autograd.Stats``
    or sums of the batched ``pos_stat`` / ``col_stat`` / ``visible``)."""

    def __init__(self, ctx: api.Context, schedule: BudgetSchedule, tau_pos: float, seed: int = 0):
        self.ctx, self.schedule, self.tau_pos = ctx, schedule, float(tau_pos)
        self.rng = np.random.default_rng(seed)

    def select(self, step: int, n_current: int, pos_sum, col_sum, count):
        """Returns (mask uint8 [n] on the device, number selected, colour branch drawn)."""
        color = bool(self.rng.random() < COLOR_PROBABILITY)
        room = max(0, self.schedule.budget(step) - int(n_current))
        mask, cnt, _ws = api.densify_select(self.ctx, pos_sum, col_sum, count, self.tau_pos,
                                            TAU_COLOR_RATIO * self.tau_pos, color, room)
        return mask, int(cnt.item()), color
