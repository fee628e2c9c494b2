"""Seeded synthetic inputs: Gaussian scenes, pinhole cameras and target images.

This module only draws random numbers and lays them out; it holds none of the
rasterizer's arithmetic.  Both the HIP path and the CPU oracle consume what it
produces, so it imports nothing from either.

Layout (structure of arrays, float32, the order the library expects):
    means      [3][N]        world-space centres
    scales     [3][N]        positive per-axis scales (already exponentiated)
    quats      [4][N]        rotation quaternion (w, x, y, z); need not be unit
    opacities  [N]           in (0, 1) (already passed through a sigmoid)
    sh         [K][3][N]     spherical-harmonic coefficients, K = (D+1)^2

The scene families follow the workloads of the paper's 1K and 4K experiments
(millions of Gaussians, SH degree 3, 1080p to 4K views; Sec. 5.2 and the
4K-resolution table of the supplement).  The real captures and trained models
are not available, so these seeded generators stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

NEAR_Z = 0.2


@dataclasses.dataclass
class Camera:
    """Pinhole camera with OpenCV axes (x right, y down, z forward).

    ``w2c`` is the 3x4 row-major world-to-camera matrix [R | t]; pixel (x, y)
    has its centre at integer coordinates (x, y).
    """
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    w2c: np.ndarray  # (3, 4) float32
    near: float = NEAR_Z

    def campos(self) -> np.ndarray:
        r = self.w2c[:, :3].astype(np.float64)
        t = self.w2c[:, 3].astype(np.float64)
        return -(r.T @ t)


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacities: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[:, idx].copy(), self.scales[:, idx].copy(),
                     self.quats[:, idx].copy(), self.opacities[idx].copy(),
                     self.sh[:, :, idx].copy(), self.sh_degree)

    def copy(self) -> "Scene":
        return Scene(self.means.copy(), self.scales.copy(), self.quats.copy(),
                     self.opacities.copy(), self.sh.copy(), self.sh_degree)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def identity_camera(width: int, height: int, focal: float) -> Camera:
    w2c = np.zeros((3, 4), np.float32)
    w2c[0, 0] = w2c[1, 1] = w2c[2, 2] = 1.0
    return Camera(width, height, float(focal), float(focal),
                  (width - 1) / 2.0, (height - 1) / 2.0, w2c)


def look_at_camera(width: int, height: int, focal: float, eye, target=(0.0, 0.0, 0.0),
                   up=(0.0, 1.0, 0.0)) -> Camera:
    """Camera at ``eye`` looking at ``target``; world ``up`` maps to image-up."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    down = -np.asarray(up, np.float64)
    down = down - fwd * np.dot(down, fwd)
    down /= np.linalg.norm(down)
    right = np.cross(down, fwd)              # x = y cross z keeps det(R) = +1
    rot = np.stack([right, down, fwd])       # rows: camera axes in world frame
    w2c = np.zeros((3, 4), np.float64)
    w2c[:, :3] = rot
    w2c[:, 3] = -rot @ eye
    return Camera(width, height, float(focal), float(focal),
                  (width - 1) / 2.0, (height - 1) / 2.0, w2c.astype(np.float32))


def ring_camera(width: int, height: int, angle: float, radius: float = 4.0) -> Camera:
    """Camera on a circle of ``radius`` in the y = 0 plane, looking at the origin."""
    eye = (radius * math.cos(angle), 0.0, radius * math.sin(angle))
    return look_at_camera(width, height, float(width), eye)


def _common_params(rng: np.random.Generator, n: int):
    log_scales = rng.normal(-3.0, 0.5, size=(3, n))
    quats = rng.normal(0.0, 1.0, size=(4, n))
    quats /= np.linalg.norm(quats, axis=0, keepdims=True)
    opac = 1.0 / (1.0 + np.exp(-rng.normal(0.0, 1.0, size=n)))
    return np.exp(log_scales), quats, opac


def _sh_from_unit_rgb(rgb: np.ndarray) -> np.ndarray:
    # Degree-0 coefficient whose colour (coefficient times the constant
    # degree-0 basis value 1/(2 sqrt(pi)), plus 0.5) equals ``rgb``.
    return ((rgb - 0.5) * (2.0 * math.sqrt(math.pi)))[None]


def tiny_config_scene(seed: int = 0, n: int = 1024) -> tuple[Scene, Camera]:
    """1,024 Gaussians, SH degree 0, camera space = world space, 128x128, f = 128."""
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-1.0, 1.0, size=(2, n))
    z = 4.0 + 2.0 * rng.uniform(-1.0, 1.0, size=n)
    means = np.concatenate([xy, z[None]], axis=0)
    scales, quats, opac = _common_params(rng, n)
    rgb = rng.uniform(0.0, 1.0, size=(3, n))
    sh = _sh_from_unit_rgb(rgb)
    scene = Scene(_f32(means), _f32(scales), _f32(quats), _f32(opac), _f32(sh), 0)
    return scene, identity_camera(128, 128, 128.0)


def cluster_means(rng: np.random.Generator, n: int, n_clusters: int = 64,
                  inner_radius: float = 3.0, sigma: float = 0.2,
                  shell_radius: float = 20.0, shell_fraction: float = 0.2) -> np.ndarray:
    """80% of points from equal-weight isotropic clusters inside a ball, 20% on a shell."""
    n_shell = int(round(shell_fraction * n))
    n_in = n - n_shell
    d = rng.normal(size=(n_clusters, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    centres = d * (inner_radius * rng.uniform(0.0, 1.0, size=(n_clusters, 1)) ** (1.0 / 3.0))
    lab = rng.integers(0, n_clusters, size=n_in)
    pts = centres[lab] + sigma * rng.normal(size=(n_in, 3))
    bad = np.linalg.norm(pts, axis=1) > inner_radius
    while bad.any():
        k = int(bad.sum())
        pts[bad] = centres[lab[bad]] + sigma * rng.normal(size=(k, 3))
        bad = np.linalg.norm(pts, axis=1) > inner_radius
    s = rng.normal(size=(n_shell, 3))
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    pts = np.concatenate([pts, shell_radius * s], axis=0)
    return pts.T


def cluster_scene(seed: int, n: int, sh_degree: int = 3) -> Scene:
    rng = np.random.default_rng(seed)
    means = cluster_means(rng, n)
    scales, quats, opac = _common_params(rng, n)
    k = (sh_degree + 1) ** 2
    sh = np.empty((k, 3, n))
    sh[0] = rng.uniform(-1.0, 1.0, size=(3, n))
    if k > 1:
        sh[1:] = rng.normal(0.0, 0.1, size=(k - 1, 3, n))
    return Scene(_f32(means), _f32(scales), _f32(quats), _f32(opac), _f32(sh), sh_degree)


def ring_angle(seed: int) -> float:
    return float(np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi))


def target_image(width: int, height: int, seed: int) -> np.ndarray:
    """Full-resolution target, planar [3][H][W], U(0, 1)."""
    rng = np.random.default_rng(seed)
    return _f32(rng.uniform(0.0, 1.0, size=(3, height, width)))


# Workload recipes.  Seeds: scene = k, target = 1000 + k, camera = 2000 + k.
WORKLOADS = {
    0: dict(name="tiny-128px-1k-sh0", n=1024, width=128, height=128, sh_degree=0, stride=1),
    1: dict(name="full-1080p-500k-sh3", n=500_000, width=1920, height=1080, sh_degree=3, stride=1),
    2: dict(name="dilated-4k-3m-sh3-d2", n=3_000_000, width=3840, height=2160, sh_degree=3, stride=2),
    3: dict(name="batched-12view-2m-sh3", n=2_000_000, sh_degree=3, views=12),
    4: dict(name="autograd-1440p-1m-sh3-d2", n=1_000_000, width=2560, height=1440, sh_degree=3, stride=2),
}

BATCH_RESOLUTIONS = ((960, 540), (1920, 1080), (2560, 1440), (3840, 2160))
BATCH_STRIDES = (1, 2, 4)


def workload(k: int, n: int | None = None):
    """Return (scene, camera, target) for workload ``k`` (0, 1, 2 or 4).

    ``n`` overrides the Gaussian count (the scene recipe is unchanged).
    """
    w = WORKLOADS[k]
    if k == 0:
        scene, cam = tiny_config_scene(seed=0, n=n or w["n"])
    else:
        scene = cluster_scene(k, n or w["n"], w["sh_degree"])
        cam = ring_camera(w["width"], w["height"], ring_angle(2000 + k))
    tgt = target_image(cam.width, cam.height, 1000 + k)
    return scene, cam, tgt


def batched_views(seed: int = 2003, views: int = 12):
    """Cameras and dilation strides of the multi-view batch (resolution, stride per view)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(views):
        w, h = BATCH_RESOLUTIONS[int(rng.integers(0, len(BATCH_RESOLUTIONS)))]
        stride = BATCH_STRIDES[int(rng.integers(0, len(BATCH_STRIDES)))]
        ang = float(rng.uniform(0.0, 2.0 * math.pi))
        out.append((ring_camera(w, h, ang), stride))
    return out


def phase_offsets(step: int, stride: int) -> tuple[int, int]:
    """Pixel phase of iteration ``step``: cycles (0,0), (1,0), (0,1), (1,1) for stride 2."""
    k = step % (stride * stride)
    return k % stride, k // stride


def small_scene(seed: int, n: int, width: int, height: int, sh_degree: int = 3,
                scale_mean: float = -2.3, depth=(2.0, 5.0), spread: float = 0.6) -> tuple[Scene, Camera]:
    """A small scene in front of a ring camera, sized so every Gaussian covers a few tiles.

    Used by the parity tests at sizes the CPU oracle finishes in seconds.
    """
    rng = np.random.default_rng(seed)
    ang = float(rng.uniform(0.0, 2.0 * math.pi))
    cam = ring_camera(width, height, ang, radius=4.0)
    # points in camera space, then mapped to the world
    z = rng.uniform(depth[0], depth[1], size=n)
    x = rng.uniform(-spread, spread, size=n) * z
    y = rng.uniform(-spread, spread, size=n) * z * height / width
    pc = np.stack([x, y, z])
    r = cam.w2c[:, :3].astype(np.float64)
    t = cam.w2c[:, 3].astype(np.float64)
    means = r.T @ (pc - t[:, None])
    log_scales = rng.normal(scale_mean, 0.5, size=(3, n))
    quats = rng.normal(0.0, 1.0, size=(4, n))
    opac = 1.0 / (1.0 + np.exp(-rng.normal(0.0, 1.0, size=n)))
    k = (sh_degree + 1) ** 2
    sh = np.empty((k, 3, n))
    sh[0] = rng.uniform(-1.0, 1.0, size=(3, n))
    if k > 1:
        sh[1:] = rng.normal(0.0, 0.1, size=(k - 1, 3, n))
    scene = Scene(_f32(means), _f32(np.exp(log_scales)), _f32(quats), _f32(opac), _f32(sh), sh_degree)
    return scene, cam


def small_multiview(seed: int, n: int, sizes, sh_degree: int = 3, spread_angle: float = 0.25):
    """A small scene seen by several ring cameras of the given (width, height).

    The Gaussians are placed in front of the first camera as in ``small_scene``
    (sized from the first entry of ``sizes``); camera k sits ``k *
    spread_angle`` radians further round the ring, so every camera sees most
    of them.  Returns (scene, cameras).
    """
    w0, h0 = sizes[0]
    scene, cam0 = small_scene(seed, n, w0, h0, sh_degree=sh_degree)
    ang0 = float(np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi))
    cams = [cam0] + [ring_camera(w, h, ang0 + k * spread_angle) for k, (w, h) in
                     enumerate(sizes) if k > 0]
    return scene, cams


def sweep_case(seed: int):
    """One tiny random case of the property sweep: (scene, camera, stride,
    off_x, off_y, tile, background).

    1-64 Gaussians, images of 8-64 pixels a side, stride 1-4 with any
    offsets, tile 8, 16 or 32, SH degree 0-3, seen by an identity camera
    (camera space = world space).  Besides generic Gaussians it draws the
    inputs where integer decisions sit close to their thresholds: centres
    placed exactly on rendered pixels, on the boundaries of 8- and 16-pixel
    blocks of the downsampled grid (the pixel rectangles of the rasterizer's
    wavefronts) and half a stride beside them; opacities 0.1 % above and
    below 1/255 and 0.99; needle-shaped Gaussians whose screen covariance is
    close to singular before the low-pass term; very large ones.
    """
    rng = np.random.default_rng(seed)
    w, h = int(rng.integers(8, 65)), int(rng.integers(8, 65))
    d = int(rng.integers(1, 5))
    ox, oy = int(rng.integers(0, d)), int(rng.integers(0, d))
    tile = (8, 16, 32)[int(rng.integers(0, 3))]
    n = int(rng.integers(1, 65))
    deg = int(rng.integers(0, 4))
    f = float(w) * float(rng.uniform(0.6, 1.6))
    cam = identity_camera(w, h, f)
    z = rng.uniform(1.0, 6.0, size=n)
    # pixel-space centres
    u = rng.uniform(-0.25 * w, 1.25 * w, size=n)
    v = rng.uniform(-0.25 * h, 1.25 * h, size=n)
    kind = rng.integers(0, 5, size=n)
    for a, (off, size) in enumerate(((ox, w), (oy, h))):
        coord = u if a == 0 else v
        n_ds = max(1, -(-(size - off) // d))
        blk = rng.choice([1, 8, 16], size=n)
        k = rng.integers(0, n_ds // blk + 1, size=n) * blk
        shift = rng.choice([0.0, -0.5 * d, 0.5 * d, -1e-3, 1e-3], size=n)
        snapped = d * k + off + shift
        coord[kind >= 2] = snapped[kind >= 2]
    means = np.stack([(u - cam.cx) * z / f, (v - cam.cy) * z / f, z])
    # screen sizes from a third of a pixel to about the image
    px = np.exp(rng.uniform(np.log(0.3), np.log(0.6 * max(w, h)), size=(3, n)))
    scales = px * z[None] / f
    needle = rng.uniform(size=n) < 0.15
    scales[1:, needle] = scales[:1, needle] * 1e-5
    quats = rng.normal(0.0, 1.0, size=(4, n))
    opac = 1.0 / (1.0 + np.exp(-rng.normal(0.0, 1.0, size=n)))
    special = rng.integers(0, 6, size=n)
    edge = np.array([1.0 / 255.0 * (1 - 1e-3), 1.0 / 255.0 * (1 + 1e-3),
                     0.99 * (1 - 1e-3), 0.99 * (1 + 1e-3), 1.0])
    pick = (special >= 3) & (kind >= 2)
    opac[pick] = edge[rng.integers(0, len(edge), size=int(pick.sum()))]
    k_sh = (deg + 1) ** 2
    sh = np.empty((k_sh, 3, n))
    sh[0] = rng.uniform(-1.2, 1.2, size=(3, n))
    if k_sh > 1:
        sh[1:] = rng.normal(0.0, 0.2, size=(k_sh - 1, 3, n))
    bg = (0.0, 0.0, 0.0) if rng.uniform() < 0.7 else tuple(float(x) for x in rng.uniform(0, 1, 3))
    scene = Scene(_f32(means), _f32(scales), _f32(quats), _f32(opac), _f32(sh), deg)
    return scene, cam, d, ox, oy, tile, bg
