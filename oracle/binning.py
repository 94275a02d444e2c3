"""Tile binning: (tile, depth) keys, their order and per-tile ranges (oracle; test
infrastructure only).

The paper does not describe the tile rasterizer's sort (it inherits it from the
original 3DGS configuration, Sec. V-A).  Reading: each visible Gaussian g of view v
emits one pair per tile of its tile rect (geometry.py); the key is
(global tile id << 32) | bits(fp32 depth) and the value is g.  Pairs are ordered by
ascending (key, g).  Depths are above the near plane (> 0), so the fp32 bit
patterns order like the depth values.  Tile t's range is the half-open interval of
sorted positions whose key has tile t ([0, 0) for an empty tile).

With cull="ellipse" a pair is listed only if the Gaussian's cutoff region
{d : a dx^2 + 2 b dx dy + c dy^2 <= -2 tau} (exactly the pixels where the cutoff
rule can pass) meets the box spanned by the tile's pixel centres; the other pairs
of the rect contribute nothing to any pixel of their tile.  The test is evaluated
in FP64 on the FP64 centre, conic and cutoff of geometry.py.  The minimum of the
quadratic over the box is 0 when the centre lies inside, else the smallest of its
minima along the four edges (each a clamped 1-D minimiser).
"""
from __future__ import annotations

import numpy as np

from .geometry import tile_layout


def box_min_q(a, b, c, dx0, dx1, dy0, dy1):
    """Minimum of q(dx, dy) = a dx^2 + 2 b dx dy + c dy^2 (positive definite) over
    the box [dx0, dx1] x [dy0, dy1]: 0 if the box holds the origin, else the
    smallest of the minima along the four edges."""
    nbc = -b / c
    nba = -b / a

    def q(dx, dy):
        return ((a * dx) * dx + ((2.0 * b) * dx) * dy) + (c * dy) * dy

    best = np.full(np.shape(dx0), np.inf)
    for dxe in (dx0, dx1):
        best = np.minimum(best, q(dxe, np.clip(nbc * dxe, dy0, dy1)))
    for dye in (dy0, dy1):
        best = np.minimum(best, q(np.clip(nba * dye, dx0, dx1), dye))
    inside = (dx0 <= 0) & (dx1 >= 0) & (dy0 <= 0) & (dy1 >= 0)
    return np.where(inside, 0.0, best)


def ellipse_meets_tile(p, g, tx, ty, W, H, tile):
    """Vectorised cutoff-region / tile-box test for Gaussians g of projection p
    and tiles (tx, ty) (arrays of equal length)."""
    u = p["u"].detach().numpy()[g]
    w = p["w"].detach().numpy()[g]
    a = p["a"].detach().numpy()[g]
    b = p["b"].detach().numpy()[g]
    c = p["c"].detach().numpy()[g]
    L = -2.0 * p["tau"].detach().numpy()[g]
    x0 = tx * tile + 0.5
    x1 = np.minimum(tx * tile + (tile - 0.5), W - 0.5)
    y0 = ty * tile + 0.5
    y1 = np.minimum(ty * tile + (tile - 0.5), H - 0.5)
    return box_min_q(a, b, c, x0 - u, x1 - u, y0 - w, y1 - w) <= L


def bin_pairs(projs, cams, tile: int = 16, cull: str = "ellipse"):
    """Returns dict with keys (uint64 [K]), values (uint32 [K], Gaussian index),
    views (int32 [K]), ranges (int64 [n_tiles, 2]) and counts (int64 [n_tiles]).
    cull: "rect" lists every tile of the rect, "ellipse" only the tiles the
    cutoff region meets."""
    tiles_x, tiles_y, off = tile_layout(cams, tile)
    tiles_all, depth_all, g_all, v_all = [], [], [], []
    for v, p in enumerate(projs):
        touched = p["touched"]
        ids = np.nonzero(touched)[0]
        cnt = touched[ids]
        k = int(cnt.sum())
        if k == 0:
            continue
        rep = np.repeat(ids, cnt)
        start = np.repeat(np.cumsum(cnt) - cnt, cnt)
        local = np.arange(k, dtype=np.int64) - start
        nx = (p["tx1"] - p["tx0"] + 1)[rep]
        tx = p["tx0"][rep] + local % nx
        ty = p["ty0"][rep] + local // nx
        if cull == "ellipse":
            keep = ellipse_meets_tile(p, rep, tx, ty, p["width"], p["height"], tile)
            rep, tx, ty = rep[keep], tx[keep], ty[keep]
            k = int(keep.sum())
            if k == 0:
                continue
        elif cull != "rect":
            raise ValueError(cull)
        tiles_all.append(off[v] + ty * tiles_x[v] + tx)
        depth_all.append(p["depth_bits"][rep].astype(np.uint64))
        g_all.append(rep.astype(np.int64))
        v_all.append(np.full(k, v, np.int32))
    n_tiles = off[-1]
    if not tiles_all:
        return dict(keys=np.zeros(0, np.uint64), values=np.zeros(0, np.uint32), views=np.zeros(0, np.int32),
                    ranges=np.zeros((n_tiles, 2), np.int64), counts=np.zeros(n_tiles, np.int64))
    tl = np.concatenate(tiles_all)
    dp = np.concatenate(depth_all)
    gg = np.concatenate(g_all)
    vv = np.concatenate(v_all)
    order = np.lexsort((gg, dp, tl))
    tl, dp, gg, vv = tl[order], dp[order], gg[order], vv[order]
    keys = (tl.astype(np.uint64) << np.uint64(32)) | dp
    counts = np.bincount(tl, minlength=n_tiles).astype(np.int64)
    ends = np.cumsum(counts)
    starts = ends - counts
    ranges = np.stack([np.where(counts > 0, starts, 0), np.where(counts > 0, ends, 0)], axis=1)
    return dict(keys=keys, values=gg.astype(np.uint32), views=vv, ranges=ranges, counts=counts)
