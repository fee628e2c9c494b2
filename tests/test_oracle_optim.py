"""Pins of the oracle's Adam against closed forms of the update."""
import torch

from oracle import optim

F64 = torch.float64


def test_first_step_from_zero_moments_is_lr_times_sign():
    # mhat = g, vhat = g^2 at t = 1, so the step is lr g / (|g| + eps)
    g = torch.tensor([3.0, -0.5, 1e-3, 0.0], dtype=F64)
    p0 = torch.tensor([1.0, 2.0, -3.0, 4.0], dtype=F64)
    z = torch.zeros(4, dtype=F64)
    lr, eps = 0.01, 1e-8
    p, m, v = optim.adam_step(p0, g, z, z, 1, lr, 0.9, 0.999, eps)
    assert torch.allclose(p, p0 - lr * g / (g.abs() + eps), rtol=0, atol=1e-15)
    assert torch.allclose(m, 0.1 * g, rtol=1e-15) and torch.allclose(v, 0.001 * g * g, rtol=1e-12)


def test_constant_gradient_steps_are_all_equal():
    # with a constant g the bias corrections make mhat = g and vhat = g^2 at
    # every step, so k steps move p by k lr g / (|g| + eps)
    g = torch.tensor([0.2, -4.0], dtype=F64)
    p = torch.tensor([0.0, 1.0], dtype=F64)
    p0 = p.clone()
    m = torch.zeros(2, dtype=F64)
    v = torch.zeros(2, dtype=F64)
    lr, eps = 0.05, 1e-12
    for t in range(1, 26):
        p, m, v = optim.adam_step(p, g, m, v, t, lr, 0.8, 0.95, eps)
    assert torch.allclose(p, p0 - 25 * lr * g / (g.abs() + eps), rtol=0, atol=1e-12)


def test_two_steps_in_exact_arithmetic():
    # b1 = 1/2, b2 = 3/4, g = +1 then -1: m2 = -1/4, v2 = 7/16,
    # mhat2 = -1/3, vhat2 = 1: p2 = p0 - lr/(1+eps) + (lr/3)/(1+eps)
    lr, eps = 0.1, 1e-3
    p, m, v = optim.adam_step(torch.tensor(5.0, dtype=F64), 1.0, 0.0, 0.0, 1, lr, 0.5, 0.75, eps)
    assert float(m) == 0.5 and float(v) == 0.25
    p, m, v = optim.adam_step(p, -1.0, m, v, 2, lr, 0.5, 0.75, eps)
    assert float(m) == -0.25 and float(v) == 0.4375
    assert abs(float(p) - (5.0 - lr / (1 + eps) + (lr / 3) / (1 + eps))) < 1e-15


def test_zero_gradient_only_decays_moments():
    m = torch.tensor([0.3], dtype=F64)
    v = torch.tensor([0.04], dtype=F64)
    p, m2, v2 = optim.adam_step(torch.tensor([1.0], dtype=F64), 0.0, m, v, 3, 0.1, 0.9, 0.99, 1e-8)
    assert torch.allclose(m2, 0.9 * m) and torch.allclose(v2, 0.99 * v)
    mhat = 0.9 * 0.3 / (1 - 0.9 ** 3)
    vhat = 0.99 * 0.04 / (1 - 0.99 ** 3)
    assert abs(float(p) - (1.0 - 0.1 * mhat / (vhat ** 0.5 + 1e-8))) < 1e-14
