"""Fused Adam kernel against the oracle's Adam: every step is taken by both
from the kernel's previous float32 state (teacher forcing), on groups of
ragged sizes, one of them misaligned for vector access; graph replays."""
import numpy as np
import pytest
import torch

from gpu_helpers import ctx, say
from oracle import optim as oopt
from paper_2412_13547_amd import api

pytestmark = pytest.mark.gpu
F64 = torch.float64


def _groups(seed):
    rng = np.random.default_rng(seed)
    sizes = [3 * 1021, 4 * 4096, 1, 0, 16 * 777 + 3]
    base = torch.as_tensor(rng.normal(0, 1, sum(sizes) + 1).astype(np.float32)).cuda()
    params, off = [], 1          # offset 1: the first group starts misaligned
    for s in sizes:
        params.append(base[off:off + s])
        off += s
    return rng, params


def _check_step(adam, grads, t, prev):
    """Moments against the oracle from the previous state, with bounds of a
    few float32 roundings of the terms (b1 m and (1 - b1) g may cancel); the
    parameter against the oracle's update from the kernel's own new moments."""
    f32 = lambda x: float(np.float32(x))     # the kernel receives float32 hyperparameters
    b1, b2, eps = f32(adam.betas[0]), f32(adam.betas[1]), f32(adam.eps)
    for k, g in enumerate(grads):
        p0, m0, v0 = prev[k]
        if p0.numel() == 0:
            continue
        g = g.cpu().to(F64)
        lr = f32(adam.lrs[k])
        _p, m, v = oopt.adam_step(p0, g, m0, v0, t, lr, b1, b2, eps)
        m_new = adam.exp_avg[k].cpu().to(F64)
        v_new = adam.exp_avg_sq[k].cpu().to(F64)
        p_new = adam.params[k].cpu().to(F64)
        ulp = 2.0 ** -24
        assert bool(((m_new - m).abs() <= 4 * ulp * (b1 * m0.abs() + (1 - b1) * g.abs())).all()), (t, k)
        assert bool(((v_new - v).abs() <= 4 * ulp * (b2 * v0 + (1 - b2) * g * g)).all()), (t, k)
        # the update from the kernel's moments, then the subtraction from p
        bc1, bc2 = 1 - b1 ** t, 1 - b2 ** t
        step = lr * (m_new / bc1) / (torch.sqrt(v_new / bc2) + eps)
        want = p0 - step
        assert bool(((p_new - want).abs() <= 12 * ulp * step.abs() + ulp * p0.abs() + 1e-38).all()), (t, k)


def test_adam_matches_oracle_step_by_step():
    rng, params = _groups(3)
    lrs = [1e-3, 1e-2, 0.5, 1e-3, 0.0]
    adam = api.Adam(ctx(), [p.contiguous() for p in params], lrs, betas=(0.9, 0.999), eps=1e-15)
    # the binding needs contiguous tensors: params above are views of one buffer
    for t in range(1, 6):
        prev = [(p.cpu().to(F64), m.cpu().to(F64), v.cpu().to(F64))
                for p, m, v in zip(adam.params, adam.exp_avg, adam.exp_avg_sq)]
        grads = [torch.as_tensor(rng.normal(0, 10.0 ** rng.integers(-3, 2), p.shape).astype(np.float32)).cuda()
                 for p in adam.params]
        adam.step(grads)
        torch.cuda.synchronize()
        assert adam.step_count == t
        _check_step(adam, grads, t, prev)
    say("[gpu] adam: 5 teacher-forced steps within bounds")


def test_adam_graph_replays():
    rng, params = _groups(4)
    ps = [p.clone() for p in params]
    eager = api.Adam(ctx(), [p.clone() for p in ps], [1e-2] * 5)
    graphed = api.Adam(ctx(), [p.clone() for p in ps], [1e-2] * 5)
    grads = [torch.as_tensor(rng.normal(0, 1, p.shape).astype(np.float32)).cuda() for p in ps]
    api.Adam(ctx(), [p.clone() for p in ps], [1e-2] * 5).step(grads)   # kernels loaded
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graphed.step(grads)
    for rep in range(3):
        eager.step(grads)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert graphed.step_count == eager.step_count == rep + 1
        for a, b in zip(eager.params, graphed.params):
            assert torch.equal(a, b), rep
