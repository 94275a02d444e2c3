"""Host-side scalars of the progressive schedule (oracle; test infrastructure only).

Sec. IV-C: hierarchical image weights (Eq. 3-4) and the local iteration budget
(Eq. 5).  Sec. IV-D: the per-image learning rate (Eq. 6-8).  Readings where the
paper is silent or garbled are stated per function.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np


def lr_current(trained_iters: float, eta0: float, etaf: float, t_a: float) -> float:
    """Eq. 6-7: log-linear interpolation between eta0 and etaf, with progress
    t = T_j / T_a capped at 1.  (The subscript of t in Eq. 6 is read as the image
    index j.)"""
    t = 1.0 if trained_iters > t_a else trained_iters / t_a
    return math.exp(math.log(eta0) * (1.0 - t) + math.log(etaf) * t)


def lr_neighbourhood(j: int, lr_c: Sequence[float], overlap: np.ndarray) -> float:
    """Eq. 8: mean of image j's own rate and its overlapping images' rates, each
    neighbour weighted by its overlap M[i, j]; the overlapping set is every i != j
    with M[i, j] > 0 and the denominator counts them plus one."""
    M = np.asarray(overlap, np.float64)
    nb = [i for i in range(len(lr_c)) if i != j and M[i, j] > 0]
    return (lr_c[j] + sum(M[i, j] * lr_c[i] for i in nb)) / (len(nb) + 1)


def hierarchical_weights(overlap: np.ndarray, new: int) -> Dict[int, float]:
    """Eq. 3-4: the new image gets weight 1; images overlapping it (layer 2) get
    M[i, new]; an image first reached in layer k gets the mean over layer k-1 of
    weight * overlap.  Layers are breadth-first layers of the overlap graph (an
    edge where M > 0).  Images never reached get no weight."""
    M = np.asarray(overlap, np.float64)
    n = M.shape[0]
    w = {new: 1.0}
    prev = [new]
    seen = {new}
    while prev:
        nxt = [i for i in range(n) if i not in seen and any(M[j, i] > 0 for j in prev)]
        for i in nxt:
            w[i] = sum(w[j] * M[j, i] for j in prev) / len(prev)
        seen.update(nxt)
        prev = nxt
    return w


def local_budget(weights: Dict[int, float], n_m: int, t_i: int) -> Dict[int, int]:
    """Eq. 5: the top N_m images by weight share T_I / 2 iterations in proportion to
    1 - exp(-w).  Rounded to integers by largest remainder so the shares sum to
    exactly T_I / 2."""
    top = sorted(weights, key=lambda i: (-weights[i], i))[:n_m]
    raw = {i: (1.0 - math.exp(-weights[i])) for i in top}
    tot = sum(raw.values())
    half = t_i // 2
    if tot <= 0:
        return {i: 0 for i in top}
    share = {i: raw[i] / (2.0 * tot) * t_i for i in top}
    base = {i: int(math.floor(share[i])) for i in top}
    rem = half - sum(base.values())
    for i in sorted(top, key=lambda i: (-(share[i] - base[i]), i))[:rem]:
        base[i] += 1
    return base


def iteration_plan(weights: Dict[int, float], n: int, n_m: int, t_i: int, u: Sequence[float]) -> List[int]:
    """Sec. IV-C: the image trained by each of the T_I iterations after an arrival.

    Local half: the Eq. 5 shares of the key images (local_budget), spent round
    robin over the key images in weight order (ties by index) while a share lasts.
    Semi-global half (T_I minus the local count): the remaining images are spread
    evenly -- ordered by the uniform draws u (ties by index) and taken cyclically,
    so counts differ by at most one and, with more images than iterations, the
    ones trained are a draw without replacement.  With no remaining image the
    semi-global half covers every image.  (The paper fixes neither the visiting
    order nor the rounding; these are readings.)"""
    share = local_budget(weights, n_m, t_i) if weights else {}
    keys = sorted(share, key=lambda i: (-weights[i], i))
    left = dict(share)
    local: List[int] = []
    while any(left[i] > 0 for i in keys):
        for i in keys:
            if left[i] > 0:
                local.append(i)
                left[i] -= 1
    rest = [i for i in range(n) if i not in share] or list(range(n))
    rest.sort(key=lambda i: (u[i], i))
    semi = [rest[k % len(rest)] for k in range(t_i - len(local))]
    return local + semi
