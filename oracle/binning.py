"""Dilated binning: tile rectangles, (tile | depth) keys, stable sort, tile ranges.

Sec. 4.1: tile-Gaussian pairs are generated on the DOWNSAMPLED image of a
dilation pattern (stride d, offsets o_x, o_y): the splat centre is mapped to
the downsampled plane (Eq. 3), its radius becomes r / d (Eq. 4), and the
occupied tiles of the fixed 16x16 (here: T x T) tile grid follow from the two.
The sort of the pairs into per-tile depth order is the prior-art tile
rasterizer's (Sec. 3, "sorted by depth ... tile-based rasterizer").

Readings:
  * Eq. 3 as printed (p_ds = W_ds p_ndc) has lost the affine part of the NDC
    map and the offsets appear in no equation.  It is read as the exact inverse
    of Eq. 5: u_ds = (u - (d-1)/2) / d, likewise v.  Binning therefore does not
    depend on the offsets.
  * r_ds = r / d is kept real (no rounding); r itself is an integer.
  * Downsampled size: W_ds = ceil((W - o_x) / d), H_ds = ceil((H - o_y) / d);
    tile grid G_x = ceil(W_ds / T), G_y = ceil(H_ds / T).
  * Occupied tiles: every tile whose span of downsampled coordinates,
    [t T, (t + 1) T) per axis, intersects the box
    [u_ds - r_ds, u_ds + r_ds] x [v_ds - r_ds, v_ds + r_ds] (interval
    intersection; a tile may qualify without holding a pixel centre inside
    the box, e.g. u_ds - r_ds = 15.5 with T = 16 includes tile 0):
        x_lo = clamp(floor((u_ds - r_ds) / T), 0, G_x)
        x_hi = clamp(floor((u_ds + r_ds) / T) + 1, 0, G_x)      (exclusive)
    evaluated in IEEE double, in exactly this order of operations.
  * Key = tile_id * 2^32 + (IEEE bits of float32(t_z)); t_z > 0 so the
    integer order is the depth order.  Pairs are emitted per Gaussian in index
    order, tiles in row-major order, and sorted stably, so equal keys keep
    ascending Gaussian index and the sorted list is unique.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

F64 = torch.float64


@dataclasses.dataclass(frozen=True)
class Grid:
    width: int
    height: int
    stride: int
    off_x: int
    off_y: int
    tile: int
    w_ds: int
    h_ds: int
    gx: int
    gy: int

    @property
    def num_tiles(self) -> int:
        return self.gx * self.gy


def grid(width: int, height: int, stride: int = 1, off_x: int = 0, off_y: int = 0,
         tile: int = 16) -> Grid:
    w_ds = -(-(width - off_x) // stride)
    h_ds = -(-(height - off_y) // stride)
    return Grid(width, height, stride, off_x, off_y, tile, w_ds, h_ds,
                -(-w_ds // tile), -(-h_ds // tile))


def tile_rects(u, v, radius, culled, g: Grid):
    """(x_lo, x_hi, y_lo, y_hi) int64 per Gaussian; empty for culled ones."""
    u = torch.as_tensor(u, dtype=F64).detach()
    v = torch.as_tensor(v, dtype=F64).detach()
    r = torch.as_tensor(radius).to(F64)
    d, T = float(g.stride), float(g.tile)
    half = 0.5 * (g.stride - 1)
    ud = (u - half) / d
    vd = (v - half) / d
    rd = r / d
    xlo = torch.floor((ud - rd) / T).clamp(0, g.gx).to(torch.int64)
    xhi = (torch.floor((ud + rd) / T) + 1).clamp(0, g.gx).to(torch.int64)
    ylo = torch.floor((vd - rd) / T).clamp(0, g.gy).to(torch.int64)
    yhi = (torch.floor((vd + rd) / T) + 1).clamp(0, g.gy).to(torch.int64)
    culled = torch.as_tensor(culled, dtype=torch.bool)
    z = torch.zeros_like(xlo)
    xlo, xhi = torch.where(culled, z, xlo), torch.where(culled, z, xhi)
    ylo, yhi = torch.where(culled, z, ylo), torch.where(culled, z, yhi)
    return xlo, xhi, ylo, yhi


def depth_bits(z) -> torch.Tensor:
    """IEEE-754 bits of float32(z), as non-negative int64."""
    z32 = np.asarray(torch.as_tensor(z).detach().numpy(), dtype=np.float32)
    return torch.as_tensor(z32.view(np.uint32).astype(np.int64))


def emit_pairs(rects, zbits: torch.Tensor, g: Grid):
    """Keys (int64) and values (Gaussian index) in emission order."""
    xlo, xhi, ylo, yhi = rects
    n = xlo.shape[0]
    w = (xhi - xlo).clamp(min=0)
    cnt = w * (yhi - ylo).clamp(min=0)
    # pair p belongs to Gaussian idx[p]; k is its position inside that
    # Gaussian's rectangle, walked row by row
    idx = torch.repeat_interleave(torch.arange(n, dtype=torch.int64), cnt)
    start = torch.cumsum(cnt, 0) - cnt
    k = torch.arange(idx.numel(), dtype=torch.int64) - start[idx]
    ty = ylo[idx] + k // w[idx]
    tx = xlo[idx] + k % w[idx]
    keys = (ty * g.gx + tx) * (1 << 32) + zbits[idx]
    return keys, idx


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor):
    sk, perm = torch.sort(keys, stable=True)
    return sk, vals[perm]


def tile_ranges(sorted_keys: torch.Tensor, num_tiles: int) -> torch.Tensor:
    """(num_tiles, 2) int64: [start, end) of each tile's run; [0, 0) when empty."""
    tiles = sorted_keys >> 32
    ranges = torch.zeros(num_tiles, 2, dtype=torch.int64)
    if tiles.numel() == 0:
        return ranges
    counts = torch.bincount(tiles, minlength=num_tiles)
    ends = torch.cumsum(counts, 0)
    starts = ends - counts
    nz = counts > 0
    ranges[nz, 0] = starts[nz]
    ranges[nz, 1] = ends[nz]
    return ranges


def bin_gaussians(u, v, z, radius, culled, g: Grid) -> dict:
    """Rectangles, tiles_touched, sorted keys/values and ranges."""
    rects = tile_rects(u, v, radius, culled, g)
    xlo, xhi, ylo, yhi = rects
    touched = ((xhi - xlo) * (yhi - ylo)).clamp(min=0)
    zb = depth_bits(z)
    keys, vals = emit_pairs(rects, zb, g)
    sk, sv = sort_pairs(keys, vals)
    return dict(rects=torch.stack(rects, 1), tiles_touched=touched, zbits=zb,
                keys=sk, vals=sv, ranges=tile_ranges(sk, g.num_tiles),
                visible=(touched > 0) & ~torch.as_tensor(culled, dtype=torch.bool))


def tile_lists_bruteforce(rects: torch.Tensor, zbits: torch.Tensor, g: Grid):
    """Per tile, the Gaussians whose rectangle contains it, ordered by (depth bits, index)."""
    out = []
    r = rects.tolist()
    zb = zbits.tolist()
    for ty in range(g.gy):
        for tx in range(g.gx):
            members = [i for i, (x0, x1, y0, y1) in enumerate(r)
                       if x0 <= tx < x1 and y0 <= ty < y1]
            members.sort(key=lambda i: (zb[i], i))
            out.append(members)
    return out


def expected_key_bits(g: Grid) -> int:
    """Significant bits of a tile id (at least 1)."""
    return max(1, math.ceil(math.log2(max(2, g.num_tiles))))
