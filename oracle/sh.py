"""Real spherical-harmonic basis used for the view-dependent colour (Sec. 3).

The paper says each Gaussian carries SH coefficients for a view-dependent
colour but does not fix the basis.  Reading used here: the real orthonormal
basis built from the complex harmonics Y_l^m that include the Condon-Shortley
phase (the convention of ``scipy.special.sph_harm_y``):

    Y_{l,0}  = Y_l^0
    Y_{l,m}  = sqrt(2) * Re Y_l^m       for m > 0
    Y_{l,-m} = sqrt(2) * Im Y_l^m       for m > 0

ordered m = -l..l within each degree, degrees 0..3 (16 functions).  Written in
Cartesian form with the unit direction (x, y, z):

    Y_l^m = (-1)^m N_lm sin^m(theta) e^{i m phi} d^m P_l / dz^m (z)
    sin^m(theta) e^{i m phi} = (x + i y)^m,   N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
"""
from __future__ import annotations

import math

import numpy as np
import torch
from numpy.polynomial import legendre as npleg


def _norm(l: int, m: int) -> float:
    return math.sqrt((2 * l + 1) / (4.0 * math.pi) * math.factorial(l - m) / math.factorial(l + m))


def _legendre_deriv_power_coeffs(l: int, m: int) -> np.ndarray:
    """Power-series coefficients (low to high) of d^m P_l / dz^m."""
    c = np.zeros(l + 1)
    c[l] = 1.0
    d = npleg.legder(c, m) if m > 0 else c
    return npleg.leg2poly(d)


def _polyval(coeffs: np.ndarray, z: torch.Tensor) -> torch.Tensor:
    out = torch.zeros_like(z)
    for c in coeffs[::-1]:
        out = out * z + float(c)
    return out


def basis(dirs: torch.Tensor, degree: int) -> torch.Tensor:
    """Evaluate the (degree+1)^2 real SH functions at unit directions.

    dirs: (N, 3) float64 unit vectors.  Returns (N, (degree+1)^2).
    """
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    cols = []
    for l in range(degree + 1):
        # powers (x + i y)^m for m = 0..l
        re = [torch.ones_like(x)]
        im = [torch.zeros_like(x)]
        for _ in range(l):
            r0, i0 = re[-1], im[-1]
            re.append(r0 * x - i0 * y)
            im.append(r0 * y + i0 * x)
        row = {}
        for m in range(0, l + 1):
            p = _polyval(_legendre_deriv_power_coeffs(l, m), z)
            k = _norm(l, m) * (-1.0) ** m
            if m == 0:
                row[0] = k * p
            else:
                row[m] = math.sqrt(2.0) * k * re[m] * p
                row[-m] = math.sqrt(2.0) * k * im[m] * p
        cols.extend(row[m] for m in range(-l, l + 1))
    return torch.stack(cols, dim=1)
