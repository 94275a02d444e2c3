"""Gradient of a loss w.r.t. every Gaussian parameter (oracle; test infrastructure
only).

Given dL/dcolor for each view (the upstream gradient of the rendered images), the
parameter gradient is the exact derivative of the forward definition
(geometry.py + composite.py), summed over views, taken by reverse-mode automatic
differentiation in FP64.  Conventions of that derivative (Sec. IV-E asks only that
gradients accumulate per Gaussian; the rest is the 3DGS backward):
  * discrete choices (which pairs pass the cutoff, the order, the stopping point,
    the tile rect) are held fixed;
  * a capped alpha (o exp(power) > ALPHA_MAX) and a colour clamped at 0 have zero
    derivative; the off-axis Jacobian clamp passes derivative only through depth.
Pixels whose upstream gradient is zero in all channels contribute nothing and are
not evaluated.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np
import torch

from .composite import ordered_visible, select, blend
from .geometry import params_f64, project_view

F64 = torch.float64
_LEAF_KEYS = ("u", "w", "a", "b", "c", "o", "rgb")


def param_grads(params32: np.ndarray, n: int, sh_degree: int, cams: List[dict], dL_dcolor: List[np.ndarray],
                tile: int = 16, max_elems: int = 4_000_000, pixel_masks: Optional[List[np.ndarray]] = None,
                dL_dalpha_sum: Optional[List[np.ndarray]] = None):
    """dL/dparams as FP64 numpy [n_params, n] for upstream images dL_dcolor[v]
    ([3, H, W], any float type) and, optionally, upstream gradients of the soft
    per-pixel count dL_dalpha_sum[v] ([H, W]; the load-balancing term).
    pixel_masks[v] ([H, W] bool) optionally limits the pixels evaluated (pixels
    outside it must have zero upstream gradient)."""
    P = params_f64(params32, n, requires_grad=True)
    for v, cam in enumerate(cams):
        proj = project_view(P, cam, sh_degree, tile)
        ids = ordered_visible(proj)
        sel = select(proj, ids, requires_grad=True)
        leaves = {k: sel[k].detach().clone().requires_grad_(True) for k in _LEAF_KEYS}
        q = {k: sel[k].detach() for k in sel}
        g = np.asarray(dL_dcolor[v], np.float64)
        gA = None if dL_dalpha_sum is None else np.asarray(dL_dalpha_sum[v], np.float64)
        active = np.any(g != 0, axis=0)
        if gA is not None:
            active |= gA != 0
        if pixel_masks is not None:
            active &= pixel_masks[v]
        py, px = np.nonzero(active)
        if len(px) and len(ids):
            bg = torch.as_tensor(np.asarray(proj["bg"], np.float64))
            chunk = max(1, min(1024, max_elems // len(ids)))
            gq = dict(leaves)
            gq["tau"] = q["tau"]
            for s in range(0, len(px), chunk):
                r = blend(q, px[s:s + chunk], py[s:s + chunk], margins=False, grad_q=gq)
                out = r["C"] + r["T_final"][None, :] * bg[:, None]
                up = torch.as_tensor(g[:, py[s:s + chunk], px[s:s + chunk]])
                obj = (out * up).sum()
                if gA is not None:
                    obj = obj + (r["alpha_sum"] * torch.as_tensor(gA[py[s:s + chunk], px[s:s + chunk]])).sum()
                obj.backward()
            outs, grads = [], []
            for k in _LEAF_KEYS:
                if leaves[k].grad is not None:
                    outs.append(sel[k])
                    grads.append(leaves[k].grad)
            if outs:
                torch.autograd.backward(outs, grads)
    if P.grad is None:
        return np.zeros((P.shape[0], n))
    return P.grad.detach().numpy().copy()
