"""Tile-size autotuner for batched multi-view steps.

The rasterizer's results do not depend on the tile edge (the cutoff rule is
per pixel), so the edge is a pure performance choice: small tiles cull more
pairs and waste fewer lanes on splats that cover part of a tile, large tiles
stage each record for more pixels and sort fewer (tile, Gaussian) pairs.  The
autotuner times one forward + backward (preprocess, bin sort, forward, loss,
backward) per candidate edge on the caller's actual field and views, after a
warm-up, with HIP events on the current stream, and keeps the fastest per
workload signature (field size rounded to a power of two, SH degree, the
multiset of view sizes).
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence, Tuple

import torch

from . import gs_reserve_pairs
from .pipeline import Rasterizer

CANDIDATES = (8, 16, 32)


def signature(n: int, sh_degree: int, cams: Sequence[dict], coarse: bool = False) -> Tuple:
    """Workload key: field size rounded up to a power of two, SH degree and (unless
    coarse) the multiset of view sizes."""
    sizes = () if coarse else tuple(sorted((int(c["width"]), int(c["height"])) for c in cams))
    return (int(math.ceil(math.log2(max(n, 1)))), int(sh_degree), sizes)


class Autotuner:
    """coarse: key on field size and SH degree only, timing the first step shape met
    in each bucket (for loops whose batches change from step to step, where timing
    every shape would cost more than it saves)."""

    def __init__(self, candidates: Sequence[int] = CANDIDATES, warmup: int = 1, reps: int = 3,
                 coarse: bool = False):
        self.candidates = tuple(candidates)
        self.warmup = warmup
        self.reps = reps
        self.coarse = coarse
        self.table: Dict[Tuple, int] = {}
        self.timings: Dict[Tuple, Dict[int, float]] = {}

    def time_tile(self, rz: Rasterizer, tile: int, params: torch.Tensor, n: int, sh_degree: int,
                  cams: Sequence[dict], target: torch.Tensor, w_l1: float, w_dssim: float) -> float:
        """Milliseconds of one forward + backward at this tile edge (mean of reps)."""
        rz.set_views(cams, tile)
        color = rz.new_image()
        dl = rz.new_image()
        grad = torch.zeros_like(params)
        loss = torch.zeros(len(cams), dtype=torch.float64, device=rz.device)

        def once():
            rz.preprocess(params, n, sh_degree)
            rz.bin_sort()
            rz.render_fwd(color)
            rz.loss(color, target, w_l1, w_dssim, loss, dl)
            rz.render_bwd(dl, grad)

        for _ in range(self.warmup):
            once()
        stream = torch.cuda.current_stream(rz.device)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(self.reps):
            once()
        t1.record(stream)
        t1.synchronize()
        return t0.elapsed_time(t1) / self.reps

    def choose(self, rz: Rasterizer, params: torch.Tensor, n: int, sh_degree: int, cams: Sequence[dict],
               target: torch.Tensor, w_l1: float = 0.8, w_dssim: float = 0.2) -> int:
        """The fastest tile edge for this workload (timed once per signature)."""
        key = signature(n, sh_degree, cams, self.coarse)
        timed = key not in self.table
        if timed:
            t = {tile: self.time_tile(rz, tile, params, n, sh_degree, cams, target, w_l1, w_dssim)
                 for tile in self.candidates}
            self.timings[key] = t
            self.table[key] = min(t, key=t.get)
        best = self.table[key]
        rz.set_views(cams, best)
        if timed and len(self.candidates) > 1:
            # the smallest edge lists the most pairs and left the pair buffers sized
            # for it: size them for the chosen edge (with the library's 25% slack)
            rz.preprocess(params, n, sh_degree)
            k = rz.bin_sort(count=True)
            gs_reserve_pairs(rz.ctx, max(1, k + k // 4 + 1024))
        return best

    def last_timings(self, n: int, sh_degree: int, cams: Sequence[dict]) -> Optional[Dict[int, float]]:
        return self.timings.get(signature(n, sh_degree, cams, self.coarse))
