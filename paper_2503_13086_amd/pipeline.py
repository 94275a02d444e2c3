"""Device-buffer plumbing around the C ABI, using torch for allocation and streams.

`Rasterizer` owns one library context and the torch tensors a training step needs
(image, dL/dimage, gradients, Adam moments); every computation is one of the
gs_* calls of the binding.  Buffer dtypes and sizes follow include/gs.h.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import (gs_memory_bytes, gs_load_balance, gs_create, gs_destroy, gs_layout, gs_preprocess, gs_bin_sort, gs_render_fwd, gs_loss,
               gs_render_bwd, gs_adam_step, gs_render_bwd_adam, gs_buffer_size, gs_copy_buffer, gs_profile_enable,
               gs_sync_status,
               gs_profile_read,
               KERNEL_NAMES, GS_BUF_RECORDS, GS_BUF_DEPTH, GS_BUF_TOUCHED, GS_BUF_TILE_RECT, GS_BUF_KEYS,
               GS_BUF_VALUES, GS_BUF_RANGES, GS_BUF_T_FINAL, GS_BUF_N_CONTRIB, GS_BUF_LAST, GS_BUF_GRAD2D,
               GS_BUF_PAIR_VIEW, GS_BUF_ALPHA_SUM, GS_BUF_EVALS, GS_BUF_PAIRS_EFF)

_BUF_DTYPES = {GS_BUF_RECORDS: torch.uint8, GS_BUF_DEPTH: torch.int32, GS_BUF_TOUCHED: torch.int32,
               GS_BUF_TILE_RECT: torch.int16, GS_BUF_KEYS: torch.int64, GS_BUF_VALUES: torch.int32,
               GS_BUF_RANGES: torch.int32, GS_BUF_T_FINAL: torch.float32, GS_BUF_N_CONTRIB: torch.int32,
               GS_BUF_LAST: torch.int32, GS_BUF_GRAD2D: torch.float32, GS_BUF_PAIR_VIEW: torch.int32,
               GS_BUF_ALPHA_SUM: torch.float32, GS_BUF_EVALS: torch.int32, GS_BUF_PAIRS_EFF: torch.int32}

# 3DGS-lineage per-group learning rates (position is the per-view Eq. 6-8 rate's eta^0):
# mean, log-scale, rotation, opacity, SH DC, SH rest
DEFAULT_LR = (1.6e-4, 5e-3, 1e-3, 2.5e-2, 2.5e-3, 1.25e-4)


def n_params(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


class Rasterizer:
    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        self.ctx = gs_create(device)
        self.cams = None
        self.pix_off = None
        self.K = None
        self.tile = 16

    def close(self):
        if self.ctx:
            torch.cuda.synchronize(self.device)
            gs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- geometry of the batch of views ----
    def set_views(self, cams: Sequence[dict], tile: Optional[int] = None):
        """Views of the next steps; tile: 8, 16 or 32 (default: keep the current edge)."""
        self.cams = list(cams)
        if tile is not None:
            self.tile = tile
        self.pix_off, self.tile_off = gs_layout(self.cams, self.tile)
        self.P = self.pix_off[-1]

    def image_views(self, flat: torch.Tensor):
        """Split a concatenated image buffer into per-view [3, H, W] views."""
        out = []
        for v, c in enumerate(self.cams):
            a, b = 3 * self.pix_off[v], 3 * self.pix_off[v + 1]
            out.append(flat[a:b].view(3, c["height"], c["width"]))
        return out

    def new_image(self, fill: Optional[float] = None) -> torch.Tensor:
        t = torch.empty(3 * self.P, dtype=torch.float32, device=self.device)
        if fill is not None:
            t.fill_(fill)
        return t

    def pack_images(self, imgs) -> torch.Tensor:
        flat = [torch.as_tensor(np.ascontiguousarray(im), dtype=torch.float32).reshape(-1) for im in imgs]
        return torch.cat(flat).to(self.device)

    # ---- the hot path ----
    def preprocess(self, params: torch.Tensor, n: int, sh_degree: int, cams=None, stream=None):
        if cams is not None:
            self.set_views(cams)
        self.params, self.n, self.sh_degree = params, n, sh_degree
        self.stride = params.shape[1]
        gs_preprocess(self.ctx, params, n, self.stride, sh_degree, self.cams, self.tile, stream)

    def bin_sort(self, stream=None, count: bool = True) -> Optional[int]:
        """K when count is True (waits for the device); count False keeps K on the
        device (check the step with sync_status)."""
        self.K = gs_bin_sort(self.ctx, stream, count)
        return self.K

    def sync_status(self, stream=None):
        gs_sync_status(self.ctx, stream)

    def render_fwd(self, color: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if color is None:
            color = self.new_image()
        gs_render_fwd(self.ctx, color, stream)
        return color

    def loss(self, color, target, w_l1=1.0, w_dssim=0.0, loss_out=None, dL_dcolor=None, stream=None):
        if dL_dcolor is None:
            dL_dcolor = self.new_image()
        if loss_out is None:
            loss_out = torch.zeros(len(self.cams), dtype=torch.float64, device=self.device)
        gs_loss(self.ctx, color, target, w_l1, w_dssim, loss_out, dL_dcolor, stream)
        return loss_out, dL_dcolor

    def load_balance(self, w_load: float, loss_out=None, stream=None):
        """Eq. 9 term on the last forward; its gradient joins the next render_bwd."""
        gs_load_balance(self.ctx, w_load, loss_out, stream)
        return loss_out

    def render_bwd(self, dL_dcolor, grad: Optional[torch.Tensor] = None, accumulate=False, stream=None):
        if grad is None:
            grad = torch.zeros_like(self.params)
        gs_render_bwd(self.ctx, self.params, dL_dcolor, grad, accumulate, stream)
        return grad

    def adam_step(self, grad, m, v, step, lr_group=DEFAULT_LR, view_lr_scale=None, group_mask=1, beta1=0.9,
                  beta2=0.999, eps=1e-15, stream=None):
        gs_adam_step(self.ctx, self.params, grad, m, v, step, self.n, self.stride, self.sh_degree, lr_group,
                     view_lr_scale, group_mask, beta1, beta2, eps, stream)

    def render_bwd_adam(self, dL_dcolor, m, v, step, lr_group=DEFAULT_LR, view_lr_scale=None, group_mask=1,
                        grad: Optional[torch.Tensor] = None, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
        """render_bwd + adam_step in one pass (the parameters of the last preprocess
        are updated in place); the gradient is written to `grad` when given."""
        gs_render_bwd_adam(self.ctx, self.params, dL_dcolor, grad, m, v, step, lr_group, view_lr_scale, group_mask,
                           beta1, beta2, eps, stream)

    # ---- inspection ----
    def buffer(self, which: int, stream=None) -> torch.Tensor:
        nbytes = gs_buffer_size(self.ctx, which)
        dt = _BUF_DTYPES[which]
        esz = torch.empty(0, dtype=dt).element_size()
        out = torch.empty(nbytes // esz, dtype=dt, device=self.device)
        if nbytes:
            gs_copy_buffer(self.ctx, which, out, nbytes, stream)
        return out

    def memory_bytes(self) -> int:
        """Device memory held by the library context's own buffers."""
        return gs_memory_bytes(self.ctx)

    def profile(self, enable=True):
        gs_profile_enable(self.ctx, enable)

    def profile_read(self):
        res = {}
        for k, name in enumerate(KERNEL_NAMES):
            n, ms = gs_profile_read(self.ctx, k)
            res[name] = (n, ms)
        return res


def params_to_device(params_np: np.ndarray, device=0) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(params_np), dtype=torch.float32).to(torch.device("cuda", device))
