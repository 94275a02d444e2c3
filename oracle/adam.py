"""Adam step with a learning rate per view (oracle; test infrastructure only).

The optimizer is the original 3DGS one (Sec. V-A): Adam with beta1 = 0.9,
beta2 = 0.999, eps = 1e-15, applied densely to every parameter of every Gaussian,
with a step counter per Gaussian (Gaussians appended later start at step 0).
Sec. IV-D replaces the global position learning-rate decay by a learning rate per
image (Eq. 6-8).  Reading for a step over several views: each parameter group g
has a base rate lr_group[g]; for the groups in `group_mask` the rate of Gaussian i
is multiplied by the mean of view_scale[v] over the views v in which i is visible
(over all views when it is visible in none).  With one view and
view_scale = eta_j / eta^0 this is the scalar of Eq. 6-8.

Parameter groups by row (see the layout in the input generator):
  0 mean (rows 0-2), 1 log-scale (3-5), 2 rotation (6-9), 3 opacity (10),
  4 SH DC (11-13), 5 SH rest (14..).
"""
from __future__ import annotations

import numpy as np

GROUP_MEAN, GROUP_SCALE, GROUP_ROT, GROUP_OPACITY, GROUP_SH_DC, GROUP_SH_REST = range(6)


def row_groups(n_rows: int) -> np.ndarray:
    g = np.full(n_rows, GROUP_SH_REST, np.int64)
    g[0:3] = GROUP_MEAN
    g[3:6] = GROUP_SCALE
    g[6:10] = GROUP_ROT
    g[10] = GROUP_OPACITY
    g[11:14] = GROUP_SH_DC
    return g


def view_factor(view_scale, visible):
    """Per-Gaussian multiplier: mean of view_scale over the views that see it.
    visible: bool [V, n]."""
    vs = np.asarray(view_scale, np.float64)
    vis = np.asarray(visible, bool)
    cnt = vis.sum(0)
    s = (vs[:, None] * vis).sum(0)
    return np.where(cnt > 0, s / np.maximum(cnt, 1), vs.mean())


def adam_step(params, grads, m, v, step, lr_group, view_scale=None, visible=None, group_mask=1,
              beta1=0.9, beta2=0.999, eps=1e-15):
    """One dense Adam step in FP64.  params/grads/m/v: [n_rows, n]; step: [n]
    (uint).  Returns new (params, m, v, step) as FP64 / int64 arrays."""
    p = np.asarray(params, np.float64)
    g = np.asarray(grads, np.float64)
    m = np.asarray(m, np.float64)
    v = np.asarray(v, np.float64)
    k = np.asarray(step, np.int64) + 1
    b1, b2 = float(np.float32(beta1)), float(np.float32(beta2))
    e = float(np.float32(eps))
    m_new = b1 * m + (1.0 - b1) * g
    v_new = b2 * v + (1.0 - b2) * g * g
    bc1 = 1.0 - b1 ** k
    bc2 = 1.0 - b2 ** k
    groups = row_groups(p.shape[0])
    lr = np.asarray(lr_group, np.float64)[groups][:, None] * np.ones((1, p.shape[1]))
    if view_scale is not None and len(view_scale) > 0:
        f = view_factor(view_scale, visible)
        for r in range(p.shape[0]):
            if (group_mask >> groups[r]) & 1:
                lr[r] = lr[r] * f
    upd = (m_new / bc1[None, :]) / (np.sqrt(v_new / bc2[None, :]) + e)
    return p - lr * upd, m_new, v_new, k
