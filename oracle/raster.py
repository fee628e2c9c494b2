"""Front-to-back compositing on the dilated pixel set.

Sec. 3 Eq. 2: C(x') = sum_i c_i s_i prod_{j<i} (1 - s_j), with s_i = o_i G'_i(x')
the per-pixel alpha of the i-th splat in depth order.  (The paper writes the
learned opacity as alpha and the per-pixel value as sigma; here o is the
learned opacity and alpha the per-pixel value.)

Sec. 4.1: pixels are taken from the downsampled image of a dilation pattern
(stride d, offsets o_x, o_y); each downsampled pixel (i, j) is blended at its
full-resolution position, and each tile of the downsampled grid walks the list
its pairs produced (``oracle.binning``).

Readings (the paper defers these to prior work):
  * alpha = min(0.99, o exp(p)), p = -1/2 (A dx^2 + C dy^2) - B dx dy,
    dx = u - X, dy = v - Y; an entry with p > 0 or alpha < 1/255 is skipped;
  * with T' = T (1 - alpha): if T' < 1e-4 the walk stops and that entry is not
    blended; otherwise C += rgb alpha T, T = T';
  * output = C + T_final * background;
  * the pixel rendered for downsampled (i, j) is X = d i + o_x, Y = d j + o_y.
    Eq. 5 maps (i, j) to the centre of its d x d block, which is a pixel only
    for odd d; the offsets of Fig. 2 select which pixel of the block is
    rendered and supervised, so Eq. 5 is used (inverted) only for binning.

Besides the image this returns, per pixel, the final transmittance, the
1-based index of the last blended entry (0 if none), the number of entries
examined until the walk ended (the stop entry included), the numbers of
blended and of clamped (o exp(p) > 0.99) entries, and a flag marking
pixels where one of the floating-point decisions above lies so close to its
threshold that float32 and float64 may legitimately decide differently.
"""
from __future__ import annotations

import math

import torch

F64 = torch.float64
ALPHA_MAX = 0.99
ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4

# relative half-widths of the "too close to call" windows used for flags
FLAG_ALPHA = 2e-4
FLAG_T = 2e-4
FLAG_CLAMP = 2e-4


def pixel_grid(g, t: int):
    """Downsampled (i, j) and full-resolution (X, Y) of the pixels of tile t."""
    ty, tx = divmod(t, g.gx)
    js = torch.arange(ty * g.tile, min((ty + 1) * g.tile, g.h_ds))
    is_ = torch.arange(tx * g.tile, min((tx + 1) * g.tile, g.w_ds))
    jj, ii = torch.meshgrid(js, is_, indexing="ij")
    ii, jj = ii.flatten(), jj.flatten()
    X = (g.stride * ii + g.off_x).to(F64)
    Y = (g.stride * jj + g.off_y).to(F64)
    return ii, jj, X, Y


def raster_forward(rec: dict, vals: torch.Tensor, ranges: torch.Tensor, g, bg=(0.0, 0.0, 0.0),
                   tiles=None, chunk: int = 1024) -> dict:
    """Render the downsampled image of grid ``g``.

    rec: dict with (N,) tensors u, v, A, B, C, opacity and (N, 3) rgb (float64;
    may require grad).  vals/ranges: the sorted pair values and per-tile
    [start, end).  ``tiles`` restricts the work to a subset of tile ids (other
    pixels are left at zero / flagged False).
    """
    u, v, A, B, Cc, o, rgb = (rec["u"], rec["v"], rec["A"], rec["B"], rec["C"],
                              rec["opacity"], rec["rgb"])
    bg = torch.as_tensor(bg, dtype=F64)
    H, W = g.h_ds, g.w_ds
    tile_ids = range(g.num_tiles) if tiles is None else tiles
    pix_idx, colours, tfin = [], [], []
    last_all = torch.zeros(H * W, dtype=torch.int64)
    neval_all = torch.zeros(H * W, dtype=torch.int64)
    nblend_all = torch.zeros(H * W, dtype=torch.int64)
    nclamp_all = torch.zeros(H * W, dtype=torch.int64)
    flag_all = torch.zeros(H * W, dtype=torch.bool)
    for t in tile_ids:
        ii, jj, X, Y = pixel_grid(g, t)
        P = X.numel()
        if P == 0:
            continue
        start, end = int(ranges[t, 0]), int(ranges[t, 1])
        T_run = torch.ones(P, dtype=F64)
        col = torch.zeros(P, 3, dtype=F64)
        alive = torch.ones(P, dtype=torch.bool)
        last = torch.zeros(P, dtype=torch.int64)
        neval = torch.zeros(P, dtype=torch.int64)
        nblend = torch.zeros(P, dtype=torch.int64)
        nclamp = torch.zeros(P, dtype=torch.int64)
        flag = torch.zeros(P, dtype=torch.bool)
        for c0 in range(start, end, chunk):
            if not bool(alive.any()):
                break
            c1 = min(end, c0 + chunk)
            ids = vals[c0:c1]
            L = c1 - c0
            dx = u[ids][None, :] - X[:, None]
            dy = v[ids][None, :] - Y[:, None]
            power = -0.5 * (A[ids] * dx * dx + Cc[ids] * dy * dy) - B[ids] * dx * dy
            raw = o[ids] * torch.exp(power)
            alpha = torch.clamp(raw, max=ALPHA_MAX)
            skip = (power > 0) | (alpha < ALPHA_MIN)
            one_minus = torch.where(skip, torch.ones_like(alpha), 1.0 - alpha)
            # transmittance before / after each entry, multiplied in list order
            Tcum = torch.cumprod(torch.cat([T_run[:, None], one_minus], 1), 1)
            T_before, T_after = Tcum[:, :-1], Tcum[:, 1:]
            stop = ~skip & (T_after < T_MIN)
            any_stop = stop.any(1)
            first = torch.argmax(stop.to(torch.int8), 1)
            lim = torch.where(any_stop, first, torch.full_like(first, L))
            k = torch.arange(L)[None, :]
            live = (k < lim[:, None]) & alive[:, None]
            examined = (k <= lim[:, None]) & (k < L) & alive[:, None]
            blend = live & ~skip
            w = torch.where(blend, alpha * T_before, torch.zeros_like(alpha))
            col = col + w @ rgb[ids]
            # decisions near their thresholds
            near_a = (power <= 0) & ((alpha * 255.0 - 1.0).abs() < FLAG_ALPHA)
            near_t = ~skip & ((T_after / T_MIN - 1.0).abs() < FLAG_T)
            near_c = (raw / ALPHA_MAX - 1.0).abs() < FLAG_CLAMP
            flag = flag | (examined & (near_a | near_t | near_c)).any(1)
            nblend = nblend + blend.sum(1)
            nclamp = nclamp + (blend & (raw > ALPHA_MAX)).sum(1)
            kk = torch.arange(L) + (c0 - start) + 1
            has_blend = blend.any(1)
            last = torch.where(alive & has_blend, (blend * kk[None, :]).max(1).values, last)
            neval = neval + torch.where(alive, torch.where(any_stop, first + 1,
                                                           torch.full_like(first, L)), 0)
            T_end = torch.where(any_stop, T_before.gather(1, first[:, None]).squeeze(1),
                                T_after[:, -1])
            T_run = torch.where(alive, T_end, T_run)
            alive = alive & ~any_stop
        p = jj * W + ii
        pix_idx.append(p)
        colours.append(col + T_run[:, None] * bg[None, :])
        tfin.append(T_run)
        last_all[p] = last
        neval_all[p] = neval
        nblend_all[p] = nblend
        nclamp_all[p] = nclamp
        flag_all[p] = flag
    if pix_idx:
        p = torch.cat(pix_idx)
        image = torch.zeros(H * W, 3, dtype=F64).index_put((p,), torch.cat(colours))
        t_final = torch.zeros(H * W, dtype=F64).index_put((p,), torch.cat(tfin))
    else:
        image = torch.zeros(H * W, 3, dtype=F64)
        t_final = torch.zeros(H * W, dtype=F64)
    return dict(image=image.T.reshape(3, H, W), t_final=t_final.reshape(H, W),
                last_contrib=last_all.reshape(H, W), n_eval=neval_all.reshape(H, W),
                n_blend=nblend_all.reshape(H, W), n_clamp=nclamp_all.reshape(H, W),
                flag=flag_all.reshape(H, W))


def render_pixel_loop(rec: dict, order, member, X: float, Y: float, bg=(0.0, 0.0, 0.0)):
    """The compositing definition for one pixel, as a plain loop.

    ``order`` lists Gaussian indices front to back; ``member(i)`` says whether
    Gaussian i takes part at this pixel.  Returns (rgb, T, last).
    """
    T = 1.0
    C = [0.0, 0.0, 0.0]
    last = 0
    k = 0
    for i in order:
        if not member(i):
            continue
        k += 1
        dx = float(rec["u"][i]) - X
        dy = float(rec["v"][i]) - Y
        p = -0.5 * (float(rec["A"][i]) * dx * dx + float(rec["C"][i]) * dy * dy) \
            - float(rec["B"][i]) * dx * dy
        if p > 0:
            continue
        a = min(ALPHA_MAX, float(rec["opacity"][i]) * math.exp(p))
        if a < ALPHA_MIN:
            continue
        Tn = T * (1.0 - a)
        if Tn < T_MIN:
            break
        for ch in range(3):
            C[ch] += float(rec["rgb"][i, ch]) * a * T
        T = Tn
        last = k
    return [C[ch] + T * bg[ch] for ch in range(3)], T, last
