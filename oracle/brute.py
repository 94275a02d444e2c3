"""Scalar pure-Python per-pixel compositing (oracle; test infrastructure only).

A second, loop-by-loop evaluation of Eq. 2 with the cutoff, cap and stopping rule
(see composite.py), used on tiny scenes to pin the vectorised compositing: one
pixel at a time, one Gaussian at a time, in ascending (fp32 depth, index) order,
with plain Python floats.
"""
from __future__ import annotations

import math

import numpy as np

from .constants import ALPHA_MAX, T_MIN


def render_pixel(proj, i: int, j: int):
    """Returns (colour [3] with background, T_final, n_blended, last_g, alpha_sum,
    n_eval): alpha_sum is the sum of the alphas of the blended Gaussians (the soft
    per-pixel Gaussian count of the load-balancing term, see loss.py); n_eval counts
    the Gaussians that pass the cutoff test before the walk ends, the one that
    stops it included."""
    vis = [g for g in range(len(proj["visible"])) if proj["visible"][g]]
    vis.sort(key=lambda g: (int(proj["depth_bits"][g]), g))
    u, w = proj["u"].detach().numpy(), proj["w"].detach().numpy()
    a, b, c = proj["a"].detach().numpy(), proj["b"].detach().numpy(), proj["c"].detach().numpy()
    o, tau = proj["o"].detach().numpy(), proj["tau"].detach().numpy()
    rgb = proj["rgb"].detach().numpy()
    T = 1.0
    C = [0.0, 0.0, 0.0]
    nb, last = 0, -1
    asum = 0.0
    ne = 0
    for g in vis:
        dx = float(u[g]) - (i + 0.5)
        dy = float(w[g]) - (j + 0.5)
        power = -0.5 * (float(a[g]) * dx * dx + float(c[g]) * dy * dy) - float(b[g]) * dx * dy
        if power > 0.0 or power < float(tau[g]):
            continue
        ne += 1
        alpha = min(ALPHA_MAX, float(o[g]) * math.exp(power))
        Tn = T * (1.0 - alpha)
        if Tn < T_MIN:
            break
        for ch in range(3):
            C[ch] += float(rgb[ch, g]) * alpha * T
        T = Tn
        nb += 1
        last = g
        asum += alpha
    bg = proj["bg"]
    return [C[ch] + T * bg[ch] for ch in range(3)], T, nb, last, asum, ne


def render_image(proj):
    W, H = proj["width"], proj["height"]
    col = np.zeros((3, H, W))
    Tf = np.zeros((H, W))
    nc = np.zeros((H, W), np.int64)
    lg = np.zeros((H, W), np.int64)
    asum = np.zeros((H, W))
    ne = np.zeros((H, W), np.int64)
    for j in range(H):
        for i in range(W):
            cc, t, n, l, a, e = render_pixel(proj, i, j)
            ne[j, i] = e
            col[:, j, i] = cc
            Tf[j, i] = t
            nc[j, i] = n
            lg[j, i] = l
            asum[j, i] = a
    return dict(color=col, T_final=Tf, n_contrib=nc, last_g=lg, alpha_sum=asum, n_eval=ne)


def blended_ids(proj, i: int, j: int):
    """The Gaussians pixel (i, j) blends, in blending order (same walk as
    render_pixel)."""
    vis = [g for g in range(len(proj["visible"])) if proj["visible"][g]]
    vis.sort(key=lambda g: (int(proj["depth_bits"][g]), g))
    u, w = proj["u"].detach().numpy(), proj["w"].detach().numpy()
    a, b, c = proj["a"].detach().numpy(), proj["b"].detach().numpy(), proj["c"].detach().numpy()
    o, tau = proj["o"].detach().numpy(), proj["tau"].detach().numpy()
    T = 1.0
    ids = []
    for g in vis:
        dx = float(u[g]) - (i + 0.5)
        dy = float(w[g]) - (j + 0.5)
        power = -0.5 * (float(a[g]) * dx * dx + float(c[g]) * dy * dy) - float(b[g]) * dx * dy
        if power > 0.0 or power < float(tau[g]):
            continue
        alpha = min(ALPHA_MAX, float(o[g]) * math.exp(power))
        Tn = T * (1.0 - alpha)
        if Tn < T_MIN:
            break
        T = Tn
        ids.append(g)
    return ids
