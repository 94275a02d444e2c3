"""Per-pixel front-to-back alpha blending, Eq. 2 (oracle; test infrastructure only).

For pixel p = (i, j) with centre (i + 1/2, j + 1/2), walk the visible Gaussians of
the view in ascending (fp32 depth, index) order.  For each Gaussian with screen
centre (u, w), conic (a, b, c), opacity o, cutoff tau and colour rgb:

  d = (u - i - 1/2, w - j - 1/2),  power = -(a dx^2 + c dy^2)/2 - b dx dy
  skip if power > 0 or power < tau                       (cutoff, see geometry.py)
  alpha = min(ALPHA_MAX, o exp(power)),  T' = T (1 - alpha)
  stop (without blending) if T' < T_MIN
  C += rgb alpha T,  T = T'
  output C + T bg, final transmittance T, number of blended Gaussians.

With the cutoffs switched off (tau = -inf, ALPHA_MAX = 1, T_MIN = 0) this is Eq. 2
exactly.  The walk is evaluated for many pixels at once: the transmittance before
Gaussian k is the running product of (1 - alpha) over the Gaussians before it
(skipped Gaussians contribute a factor of exactly 1), which is the same sequence of
FP64 multiplications as the sequential walk.  Columns (Gaussians) that pass the
cutoff for no pixel of the current pixel batch contribute exactly 0 colour and a
factor of exactly 1, so they are dropped before the products; this changes no bit
of the result.

The oracle also reports, per pixel, how close each discrete decision came to its
threshold (relative margins; the stop test's margin is divided by the running
product's accumulated sensitivity), so a test can set aside pixels where an fp32
evaluation may legitimately decide the other way.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np
import torch

from .constants import ALPHA_MAX, T_MIN

F64 = torch.float64
_FIELDS = ("u", "w", "a", "b", "c", "o")


def _first_true(mask: torch.Tensor) -> torch.Tensor:
    """Column index of the first True per row (0 for rows with none or no columns)."""
    if mask.shape[1] == 0:
        return torch.zeros(mask.shape[0], dtype=torch.long)
    return mask.to(torch.int8).argmax(1)


def ordered_visible(proj) -> np.ndarray:
    """Indices of visible Gaussians in ascending (fp32 depth bits, index) order."""
    vis = np.nonzero(proj["visible"])[0]
    order = np.lexsort((vis, proj["depth_bits"][vis]))
    return vis[order]


def select(proj, ids: np.ndarray, requires_grad=False) -> Dict[str, torch.Tensor]:
    """Per-Gaussian FP64 quantities restricted to `ids` (in that order)."""
    idx = torch.as_tensor(ids, dtype=torch.long)
    q = {k: proj[k].index_select(0, idx) for k in _FIELDS}
    q["rgb"] = proj["rgb"].index_select(1, idx)
    q["tau"] = proj["tau"].detach().index_select(0, idx)
    if requires_grad:
        return q
    return {k: v.detach() for k, v in q.items()}


def blend(q, px: np.ndarray, py: np.ndarray, *, cutoffs=True, alpha_max=ALPHA_MAX, t_min=T_MIN,
          margins=True, grad_q: Optional[Dict[str, torch.Tensor]] = None):
    """Blend one batch of pixels of one view.  q: selected quantities (detached);
    grad_q: the same quantities carrying autograd history, or None.

    Returns dict with C [3, n] (differentiable through grad_q when given), T_final
    [n], n_contrib [n], last (position in the ordered list of the last blended
    Gaussian, -1 if none), alpha_sum [n] (sum of the blended alphas, differentiable
    like C), blended_any (positions in the ordered list of the Gaussians that at
    least one of the pixels blends) and, if margins, m_cut / m_sign / m_cap / m_T [n]."""
    n = len(px)
    G = q["u"].shape[0]
    pxc = torch.as_tensor(np.asarray(px, np.float64) + 0.5)
    pyc = torch.as_tensor(np.asarray(py, np.float64) + 0.5)
    out = {}
    with torch.no_grad():
        dx = q["u"][None, :] - pxc[:, None]
        dy = q["w"][None, :] - pyc[:, None]
        a, b, c = q["a"][None, :], q["b"][None, :], q["c"][None, :]
        power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        if cutoffs:
            passed = (power <= 0) & (power >= q["tau"][None, :])
        else:
            passed = torch.ones_like(power, dtype=torch.bool)
        cols = torch.nonzero(passed.any(0)).flatten()
        ps = passed[:, cols]
        pw = power[:, cols]
        og = q["o"][cols][None, :] * torch.exp(pw)
        alpha = torch.where(ps, torch.clamp(og, max=alpha_max), torch.zeros_like(og))
        T_incl = torch.cumprod(1.0 - alpha, dim=1)
        stop = ps & (T_incl < t_min)
        nc = cols.numel()
        has_stop = stop.any(1)
        kstar = torch.where(has_stop, _first_true(stop), torch.full((n,), nc, dtype=torch.long))
        kidx = torch.arange(nc)
        blended = ps & (kidx[None, :] < kstar[:, None])
        out["n_contrib"] = blended.sum(1).numpy().astype(np.int64)
        out["blended_any"] = cols[blended.any(0)].numpy() if nc else np.zeros(0, np.int64)
        # Gaussians that pass the cutoff test before the walk ends (the stopping one
        # included): the pixel's work count
        out["n_eval"] = (ps & (kidx[None, :] <= kstar[:, None])).sum(1).numpy().astype(np.int64)
        lastk = torch.where(blended.any(1), nc - 1 - _first_true(blended.flip(1)),
                            torch.full((n,), -1, dtype=torch.long))
        if nc:
            out["last"] = torch.where(lastk >= 0, cols[lastk.clamp(min=0)], torch.full((n,), -1, dtype=torch.long)).numpy()
        else:
            out["last"] = np.full(n, -1, np.int64)
        if margins:
            inf = torch.tensor(float("inf"), dtype=F64)
            # decisions that matter: every pair up to and including the stopping one
            stop_col = torch.where(has_stop, cols[kstar.clamp(max=max(nc - 1, 0))] if nc else kstar,
                                   torch.full((n,), G, dtype=torch.long))
            upto = torch.arange(G)[None, :] <= stop_col[:, None]
            s_abs = 0.5 * (a.abs() * dx * dx + c.abs() * dy * dy) + (b * dx * dy).abs()
            m_cut = (power - q["tau"][None, :]).abs() / (q["tau"][None, :].abs() + s_abs)
            m_sign = torch.where(s_abs > 0, power.abs() / torch.where(s_abs > 0, s_abs, torch.ones_like(s_abs)), inf)
            out["m_cut"] = torch.where(upto, m_cut, inf).amin(1).numpy() if G else np.full(n, np.inf)
            out["m_sign"] = torch.where(upto, m_sign, inf).amin(1).numpy() if G else np.full(n, np.inf)
            upto_c = ps & (kidx[None, :] <= kstar[:, None])
            m_cap = (og - alpha_max).abs() / alpha_max
            # the stop test compares a running product: its distance to the threshold is
            # measured in units of the product's accumulated relative sensitivity
            # sum_k (1 + alpha_k / (1 - alpha_k)) (one unit per factor, amplified where
            # 1 - alpha is small)
            sens = torch.cumsum(torch.where(ps, 1.0 + alpha / (1.0 - alpha), torch.zeros_like(alpha)), dim=1)
            m_T = ((T_incl - t_min).abs() / (t_min * sens.clamp(min=1.0)) if t_min > 0
                   else torch.full_like(T_incl, float("inf")))
            out["m_cap"] = torch.where(upto_c, m_cap, inf).amin(1).numpy() if nc else np.full(n, np.inf)
            out["m_T"] = torch.where(upto_c, m_T, inf).amin(1).numpy() if nc else np.full(n, np.inf)

    src = grad_q if grad_q is not None else q
    u, w = src["u"][cols], src["w"][cols]
    a2, b2, c2, o2 = src["a"][cols], src["b"][cols], src["c"][cols], src["o"][cols]
    rgb = src["rgb"][:, cols]
    dx2 = u[None, :] - pxc[:, None]
    dy2 = w[None, :] - pyc[:, None]
    power2 = -0.5 * (a2[None, :] * dx2 * dx2 + c2[None, :] * dy2 * dy2) - b2[None, :] * dx2 * dy2
    alpha2 = torch.clamp(o2[None, :] * torch.exp(power2), max=alpha_max)
    alpha2 = torch.where(ps, alpha2, torch.zeros_like(alpha2))
    Ti = torch.cumprod(1.0 - alpha2, dim=1)
    ones = torch.ones((n, 1), dtype=F64)
    Te = torch.cat([ones, Ti[:, :-1]], dim=1) if nc else Ti
    wgt = torch.where(blended, alpha2 * Te, torch.zeros_like(alpha2))
    C = torch.stack([(wgt * rgb[ch][None, :]).sum(1) for ch in range(3)])
    Tall = torch.cat([ones, Ti], dim=1)                          # Tall[:, k] = T before column k
    T_final = Tall.gather(1, kstar[:, None]).squeeze(1)
    out["C"] = C
    out["T_final"] = T_final
    # soft per-pixel Gaussian count of the load-balancing term (loss.py): the sum of
    # the alphas of the blended Gaussians
    out["alpha_sum"] = torch.where(blended, alpha2, torch.zeros_like(alpha2)).sum(1)
    return out


def composite_pixels(proj, px, py, *, cutoffs=True, alpha_max=ALPHA_MAX, t_min=T_MIN, margins=True,
                     max_elems=4_000_000):
    """Blend arbitrary pixels (int arrays px, py) of one view; no autograd.
    Returns color [3, n] (background added), T_final, n_contrib, last_g (index of
    the last blended Gaussian, -1 if none), alpha_sum and margins."""
    ids = ordered_visible(proj)
    q = select(proj, ids)
    px = np.asarray(px, np.int64)
    py = np.asarray(py, np.int64)
    n = len(px)
    chunk = max(1, min(1024, max_elems // max(1, len(ids))))
    keys = ["m_cut", "m_sign", "m_cap", "m_T"] if margins else []
    acc = {k: [] for k in ["C", "T_final", "n_contrib", "n_eval", "last", "alpha_sum"] + keys}
    for s in range(0, n, chunk):
        r = blend(q, px[s:s + chunk], py[s:s + chunk], cutoffs=cutoffs, alpha_max=alpha_max,
                  t_min=t_min, margins=margins)
        for k in acc:
            acc[k].append(r[k].numpy() if isinstance(r[k], torch.Tensor) else r[k])
    res = {k: (np.concatenate(v, axis=-1) if v else np.zeros(0)) for k, v in acc.items()}
    bg = np.asarray(proj["bg"], np.float64)
    color = res.pop("C").reshape(3, n) + res["T_final"][None, :] * bg[:, None]
    last = res.pop("last")
    res["last_g"] = np.where(last >= 0, ids[np.clip(last, 0, max(len(ids) - 1, 0))] if len(ids) else -1, -1)
    res["color"] = color
    if margins:
        res["margin"] = np.minimum.reduce([res["m_cut"], res["m_sign"], res["m_cap"], res["m_T"]])
    return res


def render_view(proj, **kw):
    """Whole image of one view: color [3, H, W], T_final, n_contrib, last_g and
    margins as [H, W] arrays."""
    W, H = proj["width"], proj["height"]
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    r = composite_pixels(proj, ii.ravel(), jj.ravel(), **kw)
    out = {}
    for k, v in r.items():
        out[k] = v.reshape(3, H, W) if k == "color" else v.reshape(H, W)
    return out


def render_views(projs, **kw):
    return [render_view(p, **kw) for p in projs]


def tile_blended_counts(proj, tile: int = 16) -> np.ndarray:
    """[tiles_y, tiles_x] for the view: per tile, the number of Gaussians that at
    least one pixel of the tile blends (O9's cutoff, cap and stop rules).  These
    are the (tile, Gaussian) pairs whose per-tile partial gradients the backward
    adds into each Gaussian's sum (the splat-level accumulation of Sec. IV-E)."""
    ids = ordered_visible(proj)
    q = select(proj, ids)
    W, H = proj["width"], proj["height"]
    tx_n, ty_n = -(-W // tile), -(-H // tile)
    out = np.zeros((ty_n, tx_n), np.int64)
    for ty in range(ty_n):
        for tx in range(tx_n):
            jj, ii = np.meshgrid(np.arange(ty * tile, min((ty + 1) * tile, H)),
                                 np.arange(tx * tile, min((tx + 1) * tile, W)), indexing="ij")
            r = blend(q, ii.ravel(), jj.ravel(), margins=False)
            out[ty, tx] = len(r["blended_any"])
    return out
