"""Pins of the oracle's densification selection: thresholds at equality,
the appearance branch, unseen Gaussians, the budget's ordering and ties."""
import numpy as np

from oracle import densify


def test_threshold_is_inclusive_and_uses_the_mean_over_views():
    pos = np.array([2.0, 1.98, 6.0, 0.0], np.float32)
    cnt = np.array([2, 2, 3, 0], np.int32)           # means 1.0, 0.99, 2.0, unseen
    m, k = densify.select(pos, None, cnt, 1.0, 0.01, False)
    assert m.tolist() == [1, 0, 1, 0] and k == 2


def test_appearance_branch_only_when_active():
    pos = np.array([0.5, 0.5, 0.5], np.float32)
    col = np.array([0.02, 0.01, 0.0099], np.float32)
    cnt = np.ones(3, np.int32)
    assert densify.select(pos, col, cnt, 1.0, 0.01, False)[0].tolist() == [0, 0, 0]
    m, k = densify.select(pos, col, cnt, 1.0, 0.01, True)
    assert m.tolist() == [1, 1, 0] and k == 2


def test_budget_keeps_the_largest_scores_ties_by_index():
    pos = np.array([3.0, 5.0, 3.0, 0.5, 5.0, 4.0], np.float32)
    cnt = np.ones(6, np.int32)
    m, k = densify.select(pos, None, cnt, 1.0, 0.01, False, budget=3)
    assert m.tolist() == [0, 1, 0, 0, 1, 1] and k == 3       # 5 (1), 5 (4), 4 (5)
    m, k = densify.select(pos, None, cnt, 1.0, 0.01, False, budget=4)
    assert m.tolist() == [1, 1, 0, 0, 1, 1] and k == 4       # then 3 at index 0 before 2
    m, k = densify.select(pos, None, cnt, 1.0, 0.01, False, budget=0)
    assert m.sum() == 0 and k == 0
    m, k = densify.select(pos, None, cnt, 1.0, 0.01, False, budget=100)
    assert m.tolist() == [1, 1, 1, 0, 1, 1] and k == 5


def test_appearance_score_is_normalised_by_its_own_threshold():
    # position 1.5 tau_pos vs colour 3 tau_col: the colour score ranks first
    pos = np.array([1.5, 0.0], np.float32)
    col = np.array([0.0, 0.03], np.float32)
    cnt = np.ones(2, np.int32)
    m, k = densify.select(pos, col, cnt, 1.0, 0.01, True, budget=1)
    assert m.tolist() == [0, 1] and k == 1
