"""The convergence-aware budget schedule (Eq. 6-7, Alg. 1) against closed
forms: the end points and the linear case of Eq. 7, the warm-up exponent, the
exponent fitted to an exact power law, the 10% steps of the adaptive target
and their clamps, and the direction of the exponent's response."""
import math

import pytest

from paper_2412_13547_amd.densify import BudgetSchedule


def _sched(**kw):
    return BudgetSchedule(n_init=1000, n_max=5000, start=500, end=3000, **kw)


def test_eq7_end_points_and_linear_case():
    s = _sched()
    for a in (0.3, 1.0, 1.7):
        s.alpha = a
        assert s.budget(500) == 1000 and s.budget(3000) == 5000
        assert s.budget(100) == 1000 and s.budget(4000) == 5000       # clamped progress
    s.alpha = 1.0
    # t = 1 + 99 f: linear in the window
    assert s.budget(500 + 1250) == round(1000 + (s.progress(1750) - 1) / 99 * 4000)
    s.alpha = 0.5
    t = s.progress(1000)
    assert s.budget(1000) == round(1000 + (t ** 0.5 - 1) / (100 ** 0.5 - 1) * 4000)


def test_budget_decreases_with_the_exponent_inside_the_window():
    s = _sched()
    vals = []
    for a in (0.2, 0.5, 1.0, 1.5, 2.0):
        s.alpha = a
        vals.append(s.budget(1200))
    assert vals == sorted(vals, reverse=True) and vals[0] > vals[-1]


def test_warm_up_uses_the_linear_schedule():
    s = _sched(warmup=50)
    for k in range(1, 51):
        s.record(k, 1.0 / k)
    assert s.update() == 1.0


def test_exponent_of_an_exact_power_law():
    # loss = 3 k^-0.6: the smoothed history is a power law up to the EMA's lag,
    # whose effect fades; recent and historical slopes agree -> a ~= 0.6
    s = _sched(warmup=100, window=400)
    for k in range(1, 4001):
        s.record(k, 3.0 * k ** -0.6)
    a = s.update()
    assert abs(s.bases[-1] - 0.6) < 0.03
    assert abs(a - 0.6) < 0.03


@pytest.mark.parametrize("k", [1, 3, 6])
def test_target_grows_by_ten_percent_while_the_loss_falls(k):
    s = _sched(warmup=10, window=50)
    for i in range(1, 401):
        s.record(i, i ** -1.0)
    for _ in range(k):
        s.update()
    assert s.m_adaptive == pytest.approx(min(5000 * 1.1 ** k, 7500), rel=1e-12)


def test_target_shrinks_when_the_loss_rises_and_is_clamped():
    s = _sched(warmup=10, window=50)
    for i in range(1, 401):
        s.record(i, 0.01 * i ** 0.5)
    for _ in range(20):
        s.update()
    assert s.m_adaptive == pytest.approx(2500, rel=1e-12)


def test_slower_recent_convergence_raises_the_exponent():
    # a power law that stalls: recent slope ~0 > historical slope -> eps > 0
    s = _sched(warmup=20, window=100)
    for i in range(1, 1001):
        s.record(i, i ** -0.8 if i < 700 else 700 ** -0.8)
    a = s.update()
    base = s.bases[-1]
    assert a > base and a == pytest.approx(min(2.0, max(0.1, base + 0.5 * math.tanh(
        s_recent_minus_hist(s)))), rel=1e-12)


def s_recent_minus_hist(s):
    from paper_2412_13547_amd.densify import _slope
    steps, ema = s.steps[s.warmup:], s.ema[s.warmup:]
    return _slope(steps[-s.window:], ema[-s.window:]) - _slope(steps, ema)
