"""Pins of the oracle's SH basis (colour model of Sec. 3) to a library routine,
to orthonormality under an exact quadrature and to hand-evaluated values."""
import math

import numpy as np
import pytest
import torch
from scipy.special import sph_harm_y

from oracle import sh


def _dirs(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _scipy_real(d, degree):
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    cols = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                cols.append(y.real)
            elif m > 0:
                cols.append(math.sqrt(2.0) * y.real)
            else:
                cols.append(math.sqrt(2.0) * y.imag)
    return np.stack(cols, 1)


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_basis_matches_scipy_complex_harmonics(degree):
    d = _dirs(500, degree)
    ours = sh.basis(torch.as_tensor(d), degree).numpy()
    ref = _scipy_real(d, degree)
    np.testing.assert_allclose(ours, ref, rtol=0, atol=1e-13)


def test_orthonormal_under_exact_quadrature():
    # Gauss-Legendre in cos(theta) (exact to polynomial degree 15) times a
    # uniform phi rule (exact for trigonometric degree < 16): products of two
    # degree <= 3 functions are integrated exactly.
    x, w = np.polynomial.legendre.leggauss(8)
    phis = np.arange(16) * (2 * math.pi / 16)
    ct, ph = np.meshgrid(x, phis, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(16, 2 * math.pi / 16)[None, :]).reshape(-1)
    Y = sh.basis(torch.as_tensor(d), 3).numpy()
    gram = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_hand_values():
    k1 = math.sqrt(3 / (4 * math.pi))
    y = sh.basis(torch.tensor([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]], dtype=torch.float64), 1)
    # m = -1, 0, 1  ->  -k1 y, k1 z, -k1 x  (Condon-Shortley phase kept)
    np.testing.assert_allclose(y[:, 0].numpy(), [1 / (2 * math.sqrt(math.pi))] * 3, atol=1e-15)
    np.testing.assert_allclose(y[0, 1:].numpy(), [0, 0, -k1], atol=1e-15)
    np.testing.assert_allclose(y[1, 1:].numpy(), [-k1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(y[2, 1:].numpy(), [0, k1, 0], atol=1e-15)


def test_degree_zero_is_constant():
    d = _dirs(50, 7)
    y = sh.basis(torch.as_tensor(d), 0).numpy()
    np.testing.assert_allclose(y, 0.5 / math.sqrt(math.pi), atol=1e-15)
