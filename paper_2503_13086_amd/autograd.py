"""torch.autograd.Function over the hand-written forward and backward kernels.

`rasterize(params, n, sh_degree, cams, ...)` returns the concatenated image
(layout of include/gs.h) and, on backward, the gradient of every Gaussian
parameter from gs_render_bwd.  The per-pixel forward state the backward needs
(sorted pair lists, final transmittance, last blended position) lives in the
library context between the two calls:

  mode="store"      keep one context per call (its pair lists stay allocated until
                    backward runs); fastest, peak memory grows with every forward
                    that is waiting for its backward.
  mode="recompute"  all calls share one context; if another forward has reused it
                    when backward runs, backward first re-runs preprocess, sort and
                    forward for its own inputs (the contributor lists are
                    recomputed rather than stored), so only one set of lists is
                    alive at a time.
"""
from __future__ import annotations

import weakref
from typing import Optional, Sequence

import torch

from .pipeline import Rasterizer

_shared: dict = {}
_live: "weakref.WeakSet[Rasterizer]" = weakref.WeakSet()


def context_bytes() -> int:
    """Device memory held right now by the library contexts of this module (the
    per-call contexts of mode "store" that await their backward, and the shared
    contexts of mode "recompute")."""
    return sum(rz.memory_bytes() for rz in list(_live) if rz.ctx)


def _shared_rasterizer(device: int) -> Rasterizer:
    rz = _shared.get(device)
    if rz is None:
        rz = Rasterizer(device)
        rz.generation = 0
        _shared[device] = rz
        _live.add(rz)
    return rz


def _forward_state(rz: Rasterizer, params, n, sh_degree, cams):
    rz.preprocess(params, n, sh_degree, cams)
    rz.bin_sort()
    color = rz.render_fwd()
    rz.generation = getattr(rz, "generation", 0) + 1
    return color


class GSRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, n: int, sh_degree: int, cams, mode: str, device: int):
        if not params.is_cuda or params.dtype != torch.float32 or not params.is_contiguous():
            raise ValueError("params must be a contiguous float32 CUDA tensor [n_params, stride]")
        p = params.detach()
        if mode == "store":
            rz = Rasterizer(device)
            _live.add(rz)
        elif mode == "recompute":
            rz = _shared_rasterizer(device)
        else:
            raise ValueError(f"unknown mode {mode}")
        color = _forward_state(rz, p, n, sh_degree, cams)
        ctx.rz, ctx.mode, ctx.gen = rz, mode, rz.generation
        ctx.meta = (n, sh_degree, list(cams))
        ctx.save_for_backward(params)
        return color

    @staticmethod
    def backward(ctx, dL_dcolor):
        (params,) = ctx.saved_tensors
        rz = ctx.rz
        n, sh_degree, cams = ctx.meta
        if ctx.mode == "recompute" and rz.generation != ctx.gen:
            _forward_state(rz, params.detach(), n, sh_degree, cams)
        grad = torch.zeros_like(params)
        rz.params = params.detach()
        rz.render_bwd(dL_dcolor.contiguous(), grad)
        if ctx.mode == "store":
            rz.close()
            ctx.rz = None
        return grad, None, None, None, None, None


def rasterize(params: torch.Tensor, n: int, sh_degree: int, cams: Sequence[dict], mode: str = "store",
              device: Optional[int] = None) -> torch.Tensor:
    """Differentiable render of all views; returns the concatenated image."""
    dev = params.device.index if device is None else device
    return GSRasterize.apply(params, n, sh_degree, list(cams), mode, 0 if dev is None else dev)
