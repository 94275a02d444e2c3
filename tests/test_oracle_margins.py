"""Pins of the oracle's per-pixel decision margins (composite.blend: m_cut, m_T).

A margin says how close a pixel's discrete decisions came to their thresholds; the
parity tests set aside pixels whose margin is below what fp32 evaluation can
resolve.  What fixes a margin is its meaning: moving the inputs of one decision by
a relative amount eps can change a pixel's outcome (its blend count or last blended
Gaussian) only where that decision's margin is at most about eps.  Each test
perturbs one input of the projected splats by a seeded relative amount of at most
eps, renders again, and requires

  * every pixel whose outcome changed to have the margin below the bound derived
    in the test's docstring, and
  * the margin not to flag much more than that: a stated fraction of the pixels
    at most lies below the bound (a margin that flags everything would hide every
    mistake).

Cap and exponent-sign margins (m_cap, m_sign) move no blend count (the cap is
continuous in the colour and a positive-definite conic never gives a positive
exponent), so they are pinned by closed forms of a single splat instead."""
import math

import numpy as np
import torch

import scenegen
from oracle import geometry, composite
from oracle.constants import ALPHA_MAX, T_MIN

EPS = 2e-4


def _scene():
    # dense field: most pixels stop blending, many pairs lie near the cutoff
    sc = scenegen.small_scene(61, 2500, 0, [(64, 56)], log_scale_mean=-2.3)
    return geometry.project_view(geometry.params_f64(sc.params, sc.n), sc.cams[0], 0)


def _perturbed(pr, key, trial):
    """Trial 0 and 1 scale every splat's value by 1 + eps and 1 - eps (moves that
    add up along a pixel's list), later trials by independent seeded factors in
    [1 - eps, 1 + eps]."""
    out = dict(pr)
    x = pr[key].detach()
    if trial < 2:
        f = np.full(x.shape[0], 1.0 + (EPS if trial == 0 else -EPS))
    else:
        f = 1.0 + EPS * np.random.default_rng(trial).uniform(-1.0, 1.0, size=x.shape[0])
    out[key] = x * torch.as_tensor(f)
    return out


def _changed(r0, r1):
    return (r0["n_contrib"] != r1["n_contrib"]) | (r0["last_g"] != r1["last_g"])


def test_cutoff_margin_flags_every_cutoff_flip():
    """Cutoff taus moved by a relative eps: the exponents are unchanged, so a pair's
    cutoff test p >= tau changes only where |p - tau| <= eps |tau|, and then
    m_cut = |p - tau| / (|tau| + s) <= eps (s >= 0 the magnitude of the exponent's
    terms).  The first decision that differs lies at or before the pixel's stop,
    which is where the margin looks."""
    pr = _scene()
    r0 = composite.render_view(pr)
    flips = 0
    for trial in range(3):
        r1 = composite.render_view(_perturbed(pr, "tau", trial))
        ch = _changed(r0, r1)
        flips += int(ch.sum())
        assert (r0["m_cut"][ch] <= EPS * (1 + 1e-9)).all(), r0["m_cut"][ch].max()
    assert flips >= 10, f"only {flips} outcome changes: the test no longer probes the margin"
    assert (r0["m_cut"] <= EPS).mean() <= 0.1


def test_stop_margin_flags_every_stop_flip():
    """Opacities moved by a relative eps (cutoffs held): exponents and cutoff tests
    are unchanged, each alpha = min(0.99, o e^p) moves by at most eps alpha, so the
    running product T moves by at most a relative eps * sum alpha/(1 - alpha)
    (first order), which is at most eps times the sensitivity sum the margin divides
    by.  A stop test T < 1e-4 can therefore change only where
    m_T = |T - 1e-4| / (1e-4 sens) <= eps T / 1e-4, and T is within a few eps of
    1e-4 there: the bound used is 1.5 eps."""
    pr = _scene()
    r0 = composite.render_view(pr)
    assert (r0["n_contrib"] > 0).mean() > 0.5 and (r0["T_final"] < 2e-3).mean() > 0.2
    flips = 0
    for trial in range(3):
        r1 = composite.render_view(_perturbed(pr, "o", trial))
        ch = _changed(r0, r1)
        flips += int(ch.sum())
        assert (r0["m_T"][ch] <= 1.5 * EPS).all(), r0["m_T"][ch].max()
    assert flips >= 10, f"only {flips} outcome changes: the test no longer probes the margin"
    # the bound is a worst case (it also covers the product's own rounding, one unit
    # per factor), so it flags more pixels than any one perturbation flips
    assert (r0["m_T"] <= 1.5 * EPS).mean() <= 0.25


def _one_splat(a, b, c, o, tau, u=10.3, w=7.6):
    t = lambda v: torch.tensor([v], dtype=torch.float64)
    return dict(visible=np.array([True]), depth_bits=np.array([0x40000000], np.uint32), u=t(u), w=t(w),
                a=t(a), b=t(b), c=t(c), o=t(o), tau=t(tau), rgb=torch.ones((3, 1), dtype=torch.float64),
                bg=[0.0, 0.0, 0.0])


def test_cap_and_sign_margins_single_splat():
    """One splat, pixels around its centre.  The cap margin is the relative distance
    of o e^p to 0.99 on the pixels it passes; the exponent-sign margin, |p| over
    the magnitude of its terms, is 1 wherever the conic's cross term has the sign
    of the diagonal ones (no cancellation) and drops below 1 where it cancels them
    (the exponent is then smaller than its terms)."""
    a, b, c, o = 0.02, 0.008, 0.03, 0.995
    pr = _one_splat(a, b, c, o, -4.5)
    ii, jj = np.meshgrid(np.arange(21), np.arange(16), indexing="xy")
    r = composite.composite_pixels(pr, ii.ravel(), jj.ravel())
    dx = 10.3 - ii.ravel() - 0.5
    dy = 7.6 - jj.ravel() - 0.5
    q = a * dx * dx + 2 * b * dx * dy + c * dy * dy            # > 0: the conic is positive definite
    g = o * np.exp(-0.5 * q)
    passed = (-0.5 * q >= -4.5)
    # passing pixels are the first (and only) decision: the cap margin is exact
    assert np.allclose(r["m_cap"][passed], np.abs(g[passed] - ALPHA_MAX) / ALPHA_MAX, rtol=1e-12)
    assert np.isinf(r["m_cap"][~passed]).all()
    # some pixels are capped (o e^p above 0.99) and some not
    assert (g[passed] > ALPHA_MAX).any() and (g[passed] < ALPHA_MAX).any()
    same = dx * dy >= 0                                       # cross term adds to the diagonal terms
    assert np.allclose(r["m_sign"][same & (q > 0)], 1.0, rtol=1e-12)
    assert (r["m_sign"][~same] < 1.0).all()
    # cutoff margin: distance of p to tau relative to |tau| plus the terms' magnitude
    s_abs = 0.5 * (a * dx * dx + c * dy * dy) + np.abs(b * dx * dy)
    assert np.allclose(r["m_cut"], np.abs(-0.5 * q + 4.5) / (4.5 + s_abs), rtol=1e-12)
    # the stop margin of a lone splat: T = 1 - alpha, sensitivity 1 + alpha/(1 - alpha)
    al = np.minimum(ALPHA_MAX, g)
    m_t = np.abs((1 - al) - T_MIN) / (T_MIN * (1 + al / (1 - al)))
    assert np.allclose(r["m_T"][passed], m_t[passed], rtol=1e-10)
    assert math.isinf(composite.composite_pixels(_one_splat(a, b, c, o, -0.01), [0], [0])["m_cap"][0])


def test_cutoff_margin_covers_the_stopping_splat():
    """The stop test and the cutoff test of the splat that stops a pixel are both
    decisions: four splats on pixel (0, 0), front to back: an opaque one (alpha
    0.99), one that leaves T just above 1e-4, one sitting 1e-8 inside its cutoff
    whose alpha would take T below 1e-4 (so the walk stops there), and a faint one
    behind it that blends only if the third is skipped.  Moving the third's cutoff
    by 1e-8 changes the blend count, so m_cut must be that small."""
    t = lambda v: torch.tensor(v, dtype=torch.float64)
    a1 = float(np.float32(ALPHA_MAX))
    T1 = 1.0 - a1
    o2 = 1.0 - 1.005e-4 / T1                 # T = 1.005e-4 after the second
    d3 = math.sqrt(9.0 * (1.0 - 1e-8))        # exponent -4.5 (1 - 1e-8) at unit variance
    o4 = 0.0045                               # alpha above 1/255, T stays above 1e-4
    pr = dict(visible=np.ones(4, bool), depth_bits=np.arange(1, 5, dtype=np.uint32),
              u=t([0.5, 0.5, 0.5 + d3, 0.5]), w=t([0.5] * 4), a=t([1.0] * 4), b=t([0.0] * 4), c=t([1.0] * 4),
              o=t([0.995, o2, 0.9, o4]), tau=t([-4.5, -4.5, -4.5, -math.log(255 * o4)]),
              rgb=torch.ones((3, 4), dtype=torch.float64), bg=[0.0, 0.0, 0.0])
    r = composite.composite_pixels(pr, [0], [0])
    assert r["n_contrib"][0] == 2 and r["last_g"][0] == 1      # stopped at the third
    skip3 = dict(pr, tau=t([-4.5, -4.5, -4.49, -math.log(255 * o4)]))
    assert composite.composite_pixels(skip3, [0], [0])["n_contrib"][0] == 3   # the fourth blends instead
    assert r["m_cut"][0] <= 1e-8
