"""Pins of the oracle's colour and compositing: SH orthonormality by quadrature and
agreement with scipy's complex harmonics, closed-form single-Gaussian footprints,
two-Gaussian ordering, blending invariants, Eq. 2 with the cutoffs switched off,
and a scalar brute-force renderer on tiny scenes."""
import math

import numpy as np
import pytest
import torch
from scipy.special import sph_harm_y

import scenegen
from oracle import geometry, composite, brute
from oracle.sh import sh_basis
from oracle.constants import KAPPA, ALPHA_MAX, T_MIN


def test_sh_orthonormal_by_quadrature():
    ct, wt = np.polynomial.legendre.leggauss(24)             # exact for polynomials in cos(theta) up to degree 47
    nphi = 32
    phi = 2 * np.pi * np.arange(nphi) / nphi
    CT, PH = np.meshgrid(ct, phi, indexing="ij")
    ST = np.sqrt(1 - CT ** 2)
    x, y, z = ST * np.cos(PH), ST * np.sin(PH), CT
    Y = sh_basis(x.ravel(), y.ravel(), z.ravel(), 3)          # [16, npts]
    w = (np.repeat(wt, nphi) * (2 * np.pi / nphi))
    G = (Y * w[None]) @ Y.T
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_sh_matches_scipy_real_form():
    """Real form of scipy's Condon-Shortley-phased harmonics: sqrt(2) Re Y_l^m for
    m > 0, Y_l^0, sqrt(2) Im Y_l^|m| for m < 0, ordered k = l^2 + l + m."""
    rng = np.random.default_rng(0)
    d = rng.normal(size=(3, 500))
    d /= np.linalg.norm(d, axis=0)
    theta = np.arccos(d[2])
    phi = np.arctan2(d[1], d[0])
    Y = sh_basis(d[0], d[1], d[2], 3)
    k = 0
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), theta, phi)
            ref = c.real if m == 0 else (math.sqrt(2) * (c.real if m > 0 else c.imag))
            assert np.abs(Y[k] - ref).max() < 1e-13, (l, m)
            k += 1


def test_sh_degree0_colour():
    sc = scenegen.small_scene(3, 50, 0, [(32, 32)])
    pr = geometry.project_view(geometry.params_f64(sc.params, sc.n), sc.cams[0], 0)
    c0 = 0.5 / math.sqrt(math.pi)
    ref = np.maximum(c0 * sc.params[11:14, :sc.n].astype(np.float64) + 0.5, 0)
    assert np.abs(pr["rgb"].numpy() - ref).max() < 1e-14


def _single(o_logit, ls, z=2.0, f=64.0, W=48, H=40, cx=23.7, cy=19.2, colour=(0.9, 0.4, 0.1)):
    P = np.zeros((14, 1), np.float32)
    P[2, 0] = z                      # on the optical axis; the principal point sets its pixel position
    P[3:6, 0] = ls
    P[6, 0] = 1.0
    P[10, 0] = o_logit
    c0 = 0.5 / math.sqrt(math.pi)
    P[11:14, 0] = (np.array(colour) - 0.5) / c0
    cam = scenegen.camera(np.eye(3), np.zeros(3), f, f, cx, cy, W, H)
    return P, cam


@pytest.mark.parametrize("o_logit,ls", [(3.0, -3.0), (-2.5, -2.5), (0.0, -3.5), (5.0, -2.0)])
def test_single_isotropic_gaussian_closed_form(o_logit, ls):
    P, cam = _single(o_logit, ls)
    pr = geometry.project_view(geometry.params_f64(P, 1), cam, 0)
    r = composite.render_view(pr)
    z = float(P[2, 0])
    s = math.exp(float(np.float32(ls)))
    sig2 = (64.0 * s / z) ** 2 + KAPPA
    o = 1 / (1 + math.exp(-float(np.float32(o_logit))))
    u, w = pr["u"].item(), pr["w"].item()
    col = pr["rgb"][:, 0].numpy()
    for j in range(cam["height"]):
        for i in range(cam["width"]):
            d2 = (u - i - 0.5) ** 2 + (w - j - 0.5) ** 2
            g = o * math.exp(-d2 / (2 * sig2))
            inside = d2 <= 9 * sig2 and g >= 1 / 255
            a = min(ALPHA_MAX, g) if inside else 0.0
            assert np.allclose(r["color"][:, j, i], col * a, rtol=1e-12, atol=1e-14)
            assert abs(r["T_final"][j, i] - (1 - a)) < 1e-14
            assert abs(r["alpha_sum"][j, i] - a) < 1e-14


def test_two_gaussians_depth_order():
    cam = scenegen.camera(np.eye(3), np.zeros(3), 64.0, 64.0, 16.0, 16.0, 32, 32)
    P = np.zeros((14, 2), np.float32)
    P[6] = 1.0
    P[3:6] = -2.0
    P[10] = [1.0, 0.5]
    c0 = 0.5 / math.sqrt(math.pi)
    P[11:14, 0] = (np.array([1.0, 0.0, 0.0]) - 0.5) / c0
    P[11:14, 1] = (np.array([0.0, 0.0, 1.0]) - 0.5) / c0
    # (equal depths: the lower index is in front)
    for z0, z1 in [(2.0, 3.0), (3.0, 2.0), (2.5, 2.5)]:
        Q = P.copy()
        Q[2] = [z0, z1]
        Q[0] = [0.01 * z0, -0.02 * z1]
        pr = geometry.project_view(geometry.params_f64(Q, 2), cam, 0)
        r = composite.render_view(pr)
        first, second = (0, 1) if z0 <= z1 else (1, 0)
        assert (z0 != z1) or pr["depth_bits"][0] == pr["depth_bits"][1]
        for (j, i) in [(16, 16), (15, 17), (18, 14)]:
            al = []
            for g in range(2):
                dx = pr["u"][g].item() - i - 0.5
                dy = pr["w"][g].item() - j - 0.5
                pw = -0.5 * (pr["a"][g].item() * dx * dx + pr["c"][g].item() * dy * dy) - pr["b"][g].item() * dx * dy
                al.append(min(ALPHA_MAX, pr["o"][g].item() * math.exp(pw)) if pw >= pr["tau"][g].item() else 0.0)
            c = pr["rgb"].numpy()
            ref = c[:, first] * al[first] + c[:, second] * al[second] * (1 - al[first])
            assert np.allclose(r["color"][:, j, i], ref, rtol=1e-12, atol=1e-15)


def test_blending_invariants():
    sc = scenegen.small_scene(21, 400, 2, [(40, 36)], log_scale_mean=-2.0)
    pr = geometry.project_view(geometry.params_f64(sc.params, sc.n), sc.cams[0], 2)
    r = composite.render_view(pr)
    assert r["T_final"].min() >= T_MIN and r["T_final"].max() <= 1.0
    assert (r["n_contrib"] > 3).mean() > 0.3
    # unit colours: C = sum alpha_k T_k = 1 - T_final (telescoping)
    pr1 = dict(pr)
    pr1["rgb"] = torch.ones_like(pr["rgb"])
    r1 = composite.render_view(pr1)
    assert np.abs(r1["color"] - (1 - r["T_final"])[None]).max() < 1e-13
    # soft count: sum alpha >= 1 - prod(1 - alpha) = 1 - T_final, each blended alpha <= 0.99
    assert (r["alpha_sum"] >= 1 - r["T_final"] - 1e-13).all()
    assert (r["alpha_sum"] <= ALPHA_MAX * r["n_contrib"] + 1e-13).all()
    # 0 <= C <= max colour * (1 - T_final) with a black background
    cmax = pr["rgb"].numpy()[:, pr["visible"]].max()
    assert r["color"].min() >= 0 and (r["color"] <= cmax * (1 - r["T_final"])[None] + 1e-13).all()
    # transmittance never increases along the list: check via truncated lists
    ids = composite.ordered_visible(pr)
    prev = np.ones((36, 40))
    for cut in [len(ids) // 4, len(ids) // 2, len(ids)]:
        pc = dict(pr)
        vis = np.zeros_like(pr["visible"])
        vis[ids[:cut]] = True
        pc["visible"] = vis
        rc = composite.render_view(pc)
        assert (rc["T_final"] <= prev + 1e-15).all() or (rc["n_contrib"] < r["n_contrib"]).any()
        prev = rc["T_final"]


def test_cutoffs_off_is_eq2():
    sc = scenegen.small_scene(22, 25, 1, [(16, 12)], log_scale_mean=-1.8)
    pr = geometry.project_view(geometry.params_f64(sc.params, sc.n), sc.cams[0], 1)
    jj, ii = np.meshgrid(np.arange(12), np.arange(16), indexing="ij")
    r = composite.composite_pixels(pr, ii.ravel(), jj.ravel(), cutoffs=False, alpha_max=1.0, t_min=0.0, margins=False)
    ids = composite.ordered_visible(pr)
    c = pr["rgb"].numpy()
    for p in range(ii.size):
        i, j = ii.ravel()[p], jj.ravel()[p]
        a = []
        for g in ids:
            dx = pr["u"][g].item() - i - 0.5
            dy = pr["w"][g].item() - j - 0.5
            pw = -0.5 * (pr["a"][g].item() * dx * dx + pr["c"][g].item() * dy * dy) - pr["b"][g].item() * dx * dy
            a.append(pr["o"][g].item() * math.exp(pw))
        a = np.array(a)
        ref = sum(c[:, g] * a[k] * np.prod(1 - a[:k]) for k, g in enumerate(ids))
        assert np.allclose(r["color"][:, p], ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("seed,deg,size", [(31, 0, (32, 32)), (32, 3, (29, 23)), (33, 1, (17, 40))])
def test_vectorised_equals_scalar_brute_force(seed, deg, size):
    sc = scenegen.small_scene(seed, 64, deg, [size], log_scale_mean=-2.2, bg=(0.2, 0.5, 0.1))
    pr = geometry.project_view(geometry.params_f64(sc.params, sc.n), sc.cams[0], deg)
    rv = composite.render_view(pr)
    rb = brute.render_image(pr)
    assert np.abs(rv["color"] - rb["color"]).max() < 1e-14
    assert np.abs(rv["T_final"] - rb["T_final"]).max() < 1e-15
    assert (rv["n_contrib"] == rb["n_contrib"]).all()
    assert (rv["n_eval"] == rb["n_eval"]).all()
    assert (rv["last_g"] == rb["last_g"]).all()
    assert np.abs(rv["alpha_sum"] - rb["alpha_sum"]).max() < 1e-13
    assert rv["n_contrib"].max() >= 4


@pytest.mark.parametrize("seed,deg,size,tile", [(31, 0, (32, 32), 16), (32, 3, (29, 23), 8), (33, 1, (17, 40), 16)])
def test_tile_blended_counts_equal_brute_force_union(seed, deg, size, tile):
    """Per tile, the Gaussians some pixel blends: the vectorised count equals the
    size of the union of the scalar walk's blended lists over the tile's pixels,
    and every blended (pixel, Gaussian) belongs to exactly one tile's count."""
    sc = scenegen.small_scene(seed, 64, deg, [size], log_scale_mean=-2.2)
    pr = geometry.project_view(geometry.params_f64(sc.params, sc.n), sc.cams[0], deg)
    got = composite.tile_blended_counts(pr, tile)
    W, H = size
    want = np.zeros_like(got)
    for ty in range(got.shape[0]):
        for tx in range(got.shape[1]):
            u = set()
            for j in range(ty * tile, min((ty + 1) * tile, H)):
                for i in range(tx * tile, min((tx + 1) * tile, W)):
                    u.update(brute.blended_ids(pr, i, j))
            want[ty, tx] = len(u)
    assert np.array_equal(got, want)
    assert got.sum() > got.size        # tiles share Gaussians: several per tile on average



def test_soft_count_stops_with_the_walk():
    """Four opaque Gaussians stacked on the axis: at the centre pixel the first
    blends (alpha capped at fl32(0.99), T = 1 - fl32(0.99) after it) and the second
    stops the walk ((1 - fl32(0.99))^2 < fl32(1e-4)), so the soft count is one
    capped alpha although all four pass the cutoff; the scalar walk agrees
    everywhere."""
    cam = scenegen.camera(np.eye(3), np.zeros(3), 64.0, 64.0, 8.0, 8.0, 16, 16)
    P = np.zeros((14, 4), np.float32)
    P[2] = [2.0, 2.5, 3.0, 3.5]
    P[3:6] = -1.0
    P[6] = 1.0
    P[10] = 8.0
    pr = geometry.project_view(geometry.params_f64(P, 4), cam, 0)
    r = composite.render_view(pr)
    assert (1 - ALPHA_MAX) ** 2 < T_MIN
    assert r["n_contrib"][8, 8] == 1
    assert r["n_eval"][8, 8] == 2          # the blended one and the one that stops the walk
    assert abs(r["alpha_sum"][8, 8] - ALPHA_MAX) < 1e-15
    rb = brute.render_image(pr)
    assert np.abs(r["alpha_sum"] - rb["alpha_sum"]).max() < 1e-13
