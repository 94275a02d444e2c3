"""Tile binning: (tile, depth) keys, their order and per-tile ranges (oracle; test
infrastructure only).

The paper does not describe the tile rasterizer's sort (it inherits it from the
original 3DGS configuration, Sec. V-A).  Reading: each visible Gaussian g of view v
emits one pair per tile of its tile rect (geometry.py); the key is
(global tile id << 32) | bits(fp32 depth) and the value is g.  Pairs are ordered by
ascending (key, g).  Depths are above the near plane (> 0), so the fp32 bit
patterns order like the depth values.  Tile t's range is the half-open interval of
sorted positions whose key has tile t ([0, 0) for an empty tile).
"""
from __future__ import annotations

import numpy as np

from .geometry import tile_layout


def bin_pairs(projs, cams, tile: int = 16):
    """Returns dict with keys (uint64 [K]), values (uint32 [K], Gaussian index),
    views (int32 [K]), ranges (int64 [n_tiles, 2]) and counts (int64 [n_tiles])."""
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
