"""Per-Gaussian preprocess: view transform, 3D covariance, EWA projection, colour.

Follows Sec. 3 (Eq. 1: the Gaussian with covariance R S S^T R^T; projection to
a 2D splat) and Sec. 4.1 (the 2D covariance uses the ORIGINAL, full-resolution
focal length even when rendering dilated; a low-pass term keeps every splat at
least one pixel wide; a 3-sigma radius r in full-resolution pixels).

Readings where the paper defers to prior work or is silent:
  * near plane: a Gaussian with camera-space depth t_z <= 0.2 is culled, as is
    one with any non-finite parameter;
  * EWA Jacobian of the perspective map, evaluated at the camera-space centre
    whose x/z and y/z are first clamped to +-1.3 * (W / 2 f) and +-1.3 * (H / 2 f)
    (derivatives of the clamped expression are the true ones: zero outside);
  * low-pass: +0.3 px^2 on both diagonal entries, in full-resolution pixels;
  * radius r = ceil(3 * sqrt(lambda_max)) with lambda_max the exact larger
    eigenvalue; a Gaussian with a non-positive determinant is culled;
  * colour = sum_k sh_k Y_k(dir) + 0.5, clamped below at 0 per channel, with
    dir the unit vector from the camera centre to the mean (``oracle.sh``);
  * quaternions are (w, x, y, z) and are normalised here; scales and opacity
    arrive already activated.
Pixel (x, y) has its centre at (x, y); u = f_x t_x / t_z + c_x.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import sh as shmod

NEAR_Z = 0.2
LOW_PASS = 0.3
FOV_GUARD = 1.3
F64 = torch.float64


@dataclasses.dataclass
class Cam:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: torch.Tensor  # (3, 3) world -> camera rotation
    t: torch.Tensor  # (3,)
    near: float = NEAR_Z


def camera(cam) -> Cam:
    """Accept any object with width/height/fx/fy/cx/cy/w2c (3x4) attributes."""
    w2c = torch.as_tensor(np.asarray(cam.w2c, dtype=np.float64))
    return Cam(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy),
               float(cam.cx), float(cam.cy), w2c[:, :3].clone(), w2c[:, 3].clone(),
               float(getattr(cam, "near", NEAR_Z)))


@dataclasses.dataclass
class Params:
    means: torch.Tensor      # (N, 3)
    scales: torch.Tensor     # (N, 3)
    quats: torch.Tensor      # (N, 4)
    opacities: torch.Tensor  # (N,)
    sh: torch.Tensor         # (N, K, 3)
    degree: int


def params(scene, requires_grad: bool = False) -> Params:
    """Convert the structure-of-arrays float32 scene to float64 (N, .) tensors."""
    def t(a):
        x = torch.as_tensor(np.asarray(a, dtype=np.float64)).clone()
        return x.requires_grad_(requires_grad)
    return Params(t(scene.means.T), t(scene.scales.T), t(scene.quats.T), t(scene.opacities),
                  t(np.transpose(scene.sh, (2, 0, 1))), int(scene.sh_degree))


def rotation(q: torch.Tensor, normalize: bool = True) -> torch.Tensor:
    """Rotation matrix of the normalised quaternion (w, x, y, z); (N, 4) -> (N, 3, 3).

    ``normalize=False`` takes q as already of unit length (the matrix formula
    applied to q as given), so that a gradient w.r.t. the unit quaternion
    itself, before the normalisation's projection, can be read off."""
    if normalize:
        q = q / torch.linalg.norm(q, dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    rows = [
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ]
    return torch.stack(rows, 1)


def covariance_3d(scales: torch.Tensor, quats: torch.Tensor, normalize: bool = True) -> torch.Tensor:
    """Sigma = R S S^T R^T with S = diag(scales) (Sec. 3)."""
    m = rotation(quats, normalize) * scales[:, None, :]
    return m @ m.transpose(1, 2)


def preprocess(p: Params, cam: Cam, unit_quats: bool = False) -> dict:
    """All per-Gaussian quantities the rasterizer needs, in float64.

    Returns a dict of (N,)-leading tensors: u, v (full-resolution pixel centre),
    z (camera depth), A, B, C (inverse 2D covariance, the conic), a, b, c (2D
    covariance with the low-pass), three_sigma (3 sqrt(lambda_max)), radius
    (int64), rgb (N, 3) after the clamp, rgb_raw, clamp (bool N x 3), culled
    (bool), opacity, and the FoV-guard flags fovx, fovy (True where clamped).
    ``unit_quats=True`` skips the quaternion normalisation (the caller passes
    unit quaternions); the values are the same, only the derivative w.r.t.
    the quaternion keeps its radial part.
    """
    n = p.means.shape[0]
    finite = (torch.isfinite(p.means).all(1) & torch.isfinite(p.scales).all(1)
              & torch.isfinite(p.quats).all(1) & torch.isfinite(p.opacities)
              & torch.isfinite(p.sh.reshape(n, -1)).all(1))
    qn = torch.linalg.norm(torch.where(finite[:, None], p.quats, 1.0), dim=1)
    finite = finite & (qn > 0)
    safe = lambda x, v=0.0: torch.where(finite.reshape(-1, *([1] * (x.dim() - 1))), x, v)
    means = safe(p.means)
    scales = safe(p.scales, 1.0)
    quats = torch.where(finite[:, None], p.quats, torch.tensor([1.0, 0, 0, 0], dtype=F64))

    # view transform
    tcam = means @ cam.R.T + cam.t
    tz_raw = tcam[:, 2]
    culled = ~finite | (tz_raw <= cam.near)
    tz = torch.where(culled, torch.ones_like(tz_raw), tz_raw)
    tx, ty = tcam[:, 0], tcam[:, 1]

    u = cam.fx * tx / tz + cam.cx
    v = cam.fy * ty / tz + cam.cy

    # EWA: Jacobian of the perspective map at the (FoV-guarded) centre
    limx = FOV_GUARD * cam.width / (2.0 * cam.fx)
    limy = FOV_GUARD * cam.height / (2.0 * cam.fy)
    rx, ry = tx / tz, ty / tz
    fovx = (rx < -limx) | (rx > limx)
    fovy = (ry < -limy) | (ry > limy)
    cxr = torch.clamp(rx, -limx, limx)
    cyr = torch.clamp(ry, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([
        torch.stack([cam.fx / tz, zero, -cam.fx * cxr / tz], 1),
        torch.stack([zero, cam.fy / tz, -cam.fy * cyr / tz], 1),
    ], 1)                                        # (N, 2, 3)
    Tm = J @ cam.R                               # (N, 2, 3)
    sigma = covariance_3d(scales, quats, normalize=not unit_quats)
    cov2 = Tm @ sigma @ Tm.transpose(1, 2)
    a = cov2[:, 0, 0] + LOW_PASS
    b = cov2[:, 0, 1]
    c = cov2[:, 1, 1] + LOW_PASS
    det = a * c - b * b
    culled = culled | ~(det > 0)
    det_s = torch.where(culled, torch.ones_like(det), det)
    A, B, C = c / det_s, -b / det_s, a / det_s
    half_diff = 0.5 * (a - c)
    lam = 0.5 * (a + c) + torch.sqrt(half_diff * half_diff + b * b)
    three_sigma = 3.0 * torch.sqrt(torch.clamp(lam, min=0.0))
    radius = torch.ceil(three_sigma.detach()).to(torch.int64)
    culled = culled | (radius <= 0)
    radius = torch.where(culled, torch.zeros_like(radius), radius)

    # view-dependent colour
    campos = -(cam.R.T @ cam.t)
    dvec = means - campos
    dirs = dvec / torch.linalg.norm(dvec, dim=1, keepdim=True)
    k = (p.degree + 1) ** 2
    basis = shmod.basis(dirs, p.degree)                       # (N, k)
    rgb_raw = (safe(p.sh)[:, :k, :] * basis[:, :, None]).sum(1) + 0.5
    clamp = rgb_raw < 0
    rgb = torch.clamp(rgb_raw, min=0.0)

    cz = lambda x: torch.where(culled.reshape(-1, *([1] * (x.dim() - 1))), torch.zeros_like(x), x)
    return dict(u=cz(u), v=cz(v), z=tz_raw.detach().clone(), A=cz(A), B=cz(B), C=cz(C),
                a=cz(a), b=cz(b), c=cz(c), three_sigma=cz(three_sigma), radius=radius,
                rgb=cz(rgb), rgb_raw=cz(rgb_raw), clamp=clamp & ~culled[:, None], culled=culled,
                opacity=cz(p.opacities), fovx=fovx & ~culled, fovy=fovy & ~culled)
