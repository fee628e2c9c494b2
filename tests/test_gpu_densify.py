"""Densification selection kernel against the oracle: masks and counts
bit-exact, with and without the appearance branch and the budget, on
statistics with many exact ties and values at the thresholds."""
import numpy as np
import pytest
import torch

from gpu_helpers import ctx, say
from oracle import densify as oden
from paper_2412_13547_amd import api

pytestmark = pytest.mark.gpu


def _stats(n, seed):
    rng = np.random.default_rng(seed)
    cnt = rng.integers(0, 5, n).astype(np.int32)
    # quantised values produce exact ties and exact threshold hits
    pos = (rng.integers(0, 40, n) * 0.125 * np.maximum(cnt, 1)).astype(np.float32)
    col = (rng.integers(0, 40, n) * 0.00125 * np.maximum(cnt, 1)).astype(np.float32)
    return pos, col, cnt


@pytest.mark.parametrize("n", [0, 1, 777, 5000])
@pytest.mark.parametrize("color", [False, True])
@pytest.mark.parametrize("budget", [-1, 0, 37, 100000])
def test_selection_matches_oracle(n, color, budget):
    pos, col, cnt = _stats(n, 100 + n)
    want, wk = oden.select(pos, col, cnt, 2.5, 0.025, color, budget)
    g = lambda a: torch.as_tensor(a).cuda()
    sel, k, _ws = api.densify_select(ctx(), g(pos), g(col), g(cnt), 2.5, 0.025, color, budget)
    torch.cuda.synchronize()
    assert int(k.item()) == wk
    assert sel.cpu().numpy().tolist() == want.tolist()
    if n == 5000 and budget == 37:
        say(f"[gpu] densify n={n} color={color}: {wk} selected, bit-exact")


def test_densifier_respects_the_budget_remainder():
    from paper_2412_13547_amd.densify import BudgetSchedule, Densifier
    pos, col, cnt = _stats(5000, 7)
    sched = BudgetSchedule(n_init=5000, n_max=5100, start=0, end=100)
    d = Densifier(ctx(), sched, tau_pos=2.5, seed=1)
    g = lambda a: torch.as_tensor(a).cuda()
    room = sched.budget(50) - 5000
    mask, k, color = d.select(50, 5000, g(pos), g(col), g(cnt))
    want, wk = oden.select(pos, col, cnt, 2.5, 0.025, color, room)
    assert k == wk <= room
    assert mask.cpu().numpy().tolist() == want.tolist()
