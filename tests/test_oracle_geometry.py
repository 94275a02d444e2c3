"""Pins of the oracle's per-Gaussian geometry against things other than itself:
library routines (scipy rotations, numpy eigen-decompositions and matrix products),
closed forms, finite differences of the pinhole map, Monte Carlo projection of
samples, and brute-force tile enumeration."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation
from scipy.special import expit

import scenegen
from oracle import geometry, binning
from oracle.constants import KAPPA, JAC_CLAMP, CUTOFF_FLOOR


def _P(params32, n):
    return geometry.params_f64(params32, n)


def test_rotation_matches_scipy_and_is_orthonormal():
    rng = np.random.default_rng(0)
    q = rng.normal(size=(4, 200))
    P = np.zeros((11 + 3, 200), np.float32)
    P[6:10] = q
    _, qn, _ = geometry.activations(torch.as_tensor(P.astype(np.float64)))
    R = np.array([[e.numpy() for e in row] for row in geometry.rotation(qn)])  # [3, 3, n]
    qq = P[6:10].astype(np.float64)
    ref = Rotation.from_quat(np.stack([qq[1], qq[2], qq[3], qq[0]], 1)).as_matrix()  # scalar-last
    assert np.abs(np.moveaxis(R, 2, 0) - ref).max() < 1e-13
    Rm = np.moveaxis(R, 2, 0)
    assert np.abs(Rm @ np.swapaxes(Rm, 1, 2) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(Rm) - 1).max() < 1e-13


def test_opacity_is_logistic():
    x = np.linspace(-12, 12, 101).astype(np.float32)
    P = np.zeros((14, x.size), np.float32)
    P[6] = 1.0
    P[10] = x
    _, _, o = geometry.activations(torch.as_tensor(P.astype(np.float64)))
    assert np.abs(o.numpy() - expit(x.astype(np.float64))).max() < 1e-15


def test_covariance_eigen_and_matrix_route():
    rng = np.random.default_rng(1)
    n = 100
    P = scenegen.make_field(rng, n, 0, log_scale_mean=-1.0, log_scale_std=1.0)
    s, q, _ = geometry.activations(_P(P, n))
    Sig = np.array([[e.numpy() for e in row] for row in geometry.covariance3d(s, q)])
    Sig = np.moveaxis(Sig, 2, 0)
    sv = np.exp(P[3:6].astype(np.float64)).T
    R = Rotation.from_quat(np.stack([P[7], P[8], P[9], P[6]], 1).astype(np.float64)).as_matrix()
    ref = R @ (sv[:, :, None] ** 2 * np.eye(3)) @ np.swapaxes(R, 1, 2)
    assert np.abs(Sig - ref).max() / np.abs(ref).max() < 1e-13
    ev = np.linalg.eigvalsh(Sig)
    assert np.allclose(ev, np.sort(sv ** 2, 1), rtol=1e-10, atol=0)
    # identity quaternion gives diag(s^2)
    P2 = P.copy()
    P2[6:10] = 0
    P2[6] = 1
    s2, q2, _ = geometry.activations(_P(P2, n))
    Sig2 = geometry.covariance3d(s2, q2)
    for k in range(3):
        for l in range(3):
            exp_ = (np.exp(P2[3 + k].astype(np.float64)) ** 2) if k == l else 0.0
            assert np.allclose(Sig2[k][l].numpy(), exp_, rtol=1e-15, atol=0)


def _cam_general():
    R, t = scenegen.look_at((1.5, -0.7, -4.0), (0.2, 0.1, 0.3))
    return scenegen.camera(R, t, 310.0, 290.0, 101.5, 77.25, 203, 151)


def test_projection_matches_camera_matrix():
    rng = np.random.default_rng(2)
    n = 300
    P = scenegen.make_field(rng, n, 0, half_extent=1.0)
    cam = _cam_general()
    pr = geometry.project_view(_P(P, n), cam, 0)
    K = np.array([[cam["fx"], 0, cam["cx"]], [0, cam["fy"], cam["cy"]], [0, 0, 1]], np.float64)
    X = P[0:3, :n].astype(np.float64)
    xc = cam["R"].astype(np.float64) @ X + cam["t"].astype(np.float64)[:, None]
    h = K @ xc
    assert np.allclose(pr["u"].numpy(), h[0] / h[2], rtol=0, atol=1e-9)
    assert np.allclose(pr["w"].numpy(), h[1] / h[2], rtol=0, atol=1e-9)
    assert np.allclose(pr["tz"].numpy(), xc[2], rtol=1e-15, atol=1e-15)
    # a point on the optical axis lands on the principal point
    P2 = P[:, :1].copy()
    Rinv = cam["R"].astype(np.float64).T
    P2[0:3, 0] = (Rinv @ (np.array([0, 0, 3.0]) - cam["t"].astype(np.float64))).astype(np.float32)
    pr2 = geometry.project_view(_P(P2, 1), cam, 0)
    assert abs(pr2["u"].item() - float(cam["cx"])) < 1e-5 and abs(pr2["w"].item() - float(cam["cy"])) < 1e-5


def test_isotropic_on_axis_closed_form():
    # Sigma' = ((f s / z)^2 + kappa) I for an isotropic Gaussian on the optical axis
    cam = scenegen.camera(np.eye(3), np.zeros(3), 200.0, 200.0, 64.0, 48.0, 128, 96)
    for z, ls in [(2.0, -3.0), (5.0, -1.5), (1.0, -4.0)]:
        P = np.zeros((14, 1), np.float32)
        P[2, 0] = z
        P[3:6, 0] = ls
        P[6, 0] = 1.0
        pr = geometry.project_view(_P(P, 1), cam, 0)
        s = math.exp(float(np.float32(ls)))
        ref = (200.0 * s / z) ** 2 + KAPPA
        assert abs(pr["S00"].item() - ref) <= 1e-14 * ref
        assert abs(pr["S11"].item() - ref) <= 1e-14 * ref
        assert pr["S01"].item() == 0.0
        assert abs(pr["r"].item() - 3 * math.sqrt(ref)) <= 1e-14 * ref


def _pinhole_map(cam, X):
    return np.array([cam["fx"] * X[0] / X[2] + cam["cx"], cam["fy"] * X[1] / X[2] + cam["cy"]], np.float64)


def _fd_jacobian(cam, X, h=1e-6):
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h * max(1.0, abs(X[k]))
        J[:, k] = (_pinhole_map(cam, X + e) - _pinhole_map(cam, X - e)) / (2 * e[k])
    return J


@pytest.mark.parametrize("offaxis", [False, True])
def test_ewa_equals_fd_jacobian_route(offaxis):
    """Sigma' - kappa I = J W Sigma W^T J^T, with J the finite-difference Jacobian of
    the pinhole map at the camera point (moved onto the clamp boundary when it lies
    beyond 1.3x the half field of view)."""
    rng = np.random.default_rng(3 + offaxis)
    cam = _cam_general()
    n = 40
    P = scenegen.make_field(rng, n, 0, half_extent=0.8, log_scale_mean=-2.0)
    Rw = cam["R"].astype(np.float64)
    tw = cam["t"].astype(np.float64)
    if offaxis:
        # push the points sideways in camera space, far beyond the field of view
        Xc = Rw @ P[0:3, :n].astype(np.float64) + tw[:, None]
        Xc[0] += 3.0 * Xc[2]
        P[0:3, :n] = (Rw.T @ (Xc - tw[:, None])).astype(np.float32)
    pr = geometry.project_view(_P(P, n), cam, 0)
    s, q, _ = geometry.activations(_P(P, n))
    Sig = np.moveaxis(np.array([[e.numpy() for e in row] for row in geometry.covariance3d(s, q)]), 2, 0)
    limx = JAC_CLAMP * 0.5 * cam["width"] / cam["fx"]
    limy = JAC_CLAMP * 0.5 * cam["height"] / cam["fy"]
    n_clamped = 0
    for g in range(n):
        X = Rw @ P[0:3, g].astype(np.float64) + tw
        if X[2] <= 0.2:
            continue
        Xe = X.copy()
        if abs(X[0] / X[2]) > limx or abs(X[1] / X[2]) > limy:
            n_clamped += 1
        Xe[0] = X[2] * np.clip(X[0] / X[2], -limx, limx)
        Xe[1] = X[2] * np.clip(X[1] / X[2], -limy, limy)
        J = _fd_jacobian(cam, Xe)
        ref = J @ Rw @ Sig[g] @ Rw.T @ J.T
        got = np.array([[pr["S00"][g].item() - KAPPA, pr["S01"][g].item()],
                        [pr["S01"][g].item(), pr["S11"][g].item() - KAPPA]])
        assert np.abs(got - ref).max() <= 1e-7 * np.abs(ref).max()
    if offaxis:
        assert n_clamped > 0


def test_ewa_monte_carlo():
    """Projected samples of a small 3D Gaussian have (to first order) the 2D
    covariance J W Sigma W^T J^T."""
    rng = np.random.default_rng(5)
    cam = _cam_general()
    P = scenegen.make_field(rng, 3, 0, half_extent=0.3, log_scale_mean=-4.0, log_scale_std=0.3)
    pr = geometry.project_view(_P(P, 3), cam, 0)
    s, q, _ = geometry.activations(_P(P, 3))
    Sig = np.moveaxis(np.array([[e.numpy() for e in row] for row in geometry.covariance3d(s, q)]), 2, 0)
    Rw, tw = cam["R"].astype(np.float64), cam["t"].astype(np.float64)
    for g in range(3):
        X = rng.multivariate_normal(P[0:3, g].astype(np.float64), Sig[g], size=400_000)
        Xc = X @ Rw.T + tw
        uv = np.stack([cam["fx"] * Xc[:, 0] / Xc[:, 2] + cam["cx"], cam["fy"] * Xc[:, 1] / Xc[:, 2] + cam["cy"]])
        emp = np.cov(uv)
        ref = np.array([[pr["S00"][g].item() - KAPPA, pr["S01"][g].item()],
                        [pr["S01"][g].item(), pr["S11"][g].item() - KAPPA]])
        scale = math.sqrt(ref[0, 0] * ref[1, 1])
        assert np.abs(emp - ref).max() <= 0.02 * scale


def test_conic_and_extent():
    rng = np.random.default_rng(6)
    n = 200
    P = scenegen.make_field(rng, n, 0, half_extent=1.0, log_scale_mean=-2.5, log_scale_std=1.0)
    cam = scenegen.camera(np.eye(3), [0, 0, 3.0], 150.0, 150.0, 64, 64, 128, 128)
    pr = geometry.project_view(_P(P, n), cam, 0)
    for g in range(n):
        S = np.array([[pr["S00"][g].item(), pr["S01"][g].item()], [pr["S01"][g].item(), pr["S11"][g].item()]])
        A = np.array([[pr["a"][g].item(), pr["b"][g].item()], [pr["b"][g].item(), pr["c"][g].item()]])
        assert np.abs(A @ S - np.eye(2)).max() < 1e-12
        lam = np.linalg.eigvalsh(S).max()
        assert abs(pr["lam"][g].item() - lam) <= 1e-12 * lam
        assert abs(pr["r"][g].item() - 3 * math.sqrt(lam)) <= 1e-12 * math.sqrt(lam)


def test_cutoff_exponent():
    rho = np.linspace(-9, 6, 61).astype(np.float32)
    P = np.zeros((14, rho.size), np.float32)
    P[2] = 3.0
    P[6] = 1.0
    P[10] = rho
    cam = scenegen.camera(np.eye(3), np.zeros(3), 100, 100, 32, 32, 64, 64)
    pr = geometry.project_view(_P(P, rho.size), cam, 0)
    o = expit(rho.astype(np.float64))
    tau = pr["tau"].numpy()
    for k in range(rho.size):
        if o[k] * math.exp(CUTOFF_FLOOR) < 1 / 255:
            assert abs(o[k] * math.exp(tau[k]) - 1 / 255) < 1e-15     # alpha threshold binds
        else:
            assert tau[k] == CUTOFF_FLOOR                              # 3-sigma ellipse binds


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_tile_rect_brute_force(tile):
    """Tiles touched == tiles holding at least one pixel centre of the square
    [u-r, u+r] x [w-r, w+r] inside the image (scalar enumeration)."""
    sc = scenegen.small_scene(11, 150, 0, [(77, 45)], log_scale_mean=-2.2, half_extent=1.4, depth=2.5)
    pr = geometry.project_view(_P(sc.params, sc.n), sc.cams[0], 0, tile)
    W, H = 77, 45
    u, w, r = pr["u"].numpy(), pr["w"].numpy(), pr["r"].numpy()
    for g in range(sc.n):
        tiles = set()
        if pr["tz"][g].item() > 0.2:
            for j in range(H):
                if abs((j + 0.5) - w[g]) > r[g]:
                    continue
                for i in range(W):
                    if abs((i + 0.5) - u[g]) <= r[g]:
                        tiles.add((i // tile, j // tile))
        assert pr["touched"][g] == len(tiles)
        if tiles:
            assert pr["visible"][g]
            assert tiles == {(tx, ty) for tx in range(pr["tx0"][g], pr["tx1"][g] + 1)
                             for ty in range(pr["ty0"][g], pr["ty1"][g] + 1)}


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_tile_layout_brute_force(tile):
    # ragged views: the tiles of a view are the distinct (x // tile, y // tile) of
    # its pixels, numbered row by row after the tiles of the views before it
    sizes = [(100, 37), (64, 64), (17, 129), (1, 1), (33, 8)]
    cams = [{"width": w, "height": h} for w, h in sizes]
    tx, ty, off = geometry.tile_layout(cams, tile)
    assert off[0] == 0 and len(off) == len(sizes) + 1
    for v, (w, h) in enumerate(sizes):
        cols = {x // tile for x in range(w)}
        rows = {y // tile for y in range(h)}
        assert (tx[v], ty[v]) == (len(cols), len(rows))
        ids = {off[v] + (y // tile) * tx[v] + x // tile for y in range(h) for x in range(w)}
        assert ids == set(range(off[v], off[v + 1]))


def test_binning_sorted_and_ranges():
    sc = scenegen.small_scene(12, 120, 1, [(40, 29), (33, 50)], log_scale_mean=-2.4)
    projs = geometry.project_views(sc.params, sc.n, 1, sc.cams, 16)
    b = binning.bin_pairs(projs, sc.cams, 16, cull="rect")
    tiles_x, tiles_y, off = geometry.tile_layout(sc.cams, 16)
    tup = []
    for v, pr in enumerate(projs):
        for g in range(sc.n):
            if not pr["visible"][g]:
                continue
            for ty in range(pr["ty0"][g], pr["ty1"][g] + 1):
                for tx in range(pr["tx0"][g], pr["tx1"][g] + 1):
                    tup.append((off[v] + ty * tiles_x[v] + tx, int(pr["depth_bits"][g]), g))
    tup.sort()
    assert len(tup) == len(b["keys"]) == sum(int(p["touched"].sum()) for p in projs)
    for k, (t, d, g) in enumerate(tup):
        assert int(b["keys"][k]) == (t << 32) | d and int(b["values"][k]) == g
    for t in range(off[-1]):
        ks = [k for k, x in enumerate(tup) if x[0] == t]
        if ks:
            assert tuple(b["ranges"][t]) == (ks[0], ks[-1] + 1)
        else:
            assert tuple(b["ranges"][t]) == (0, 0)


def test_view_dependent_colour_independent_route():
    """Colour = max(0, sum_k f_k Y_k(dir) + 1/2) with dir the unit vector from the
    camera centre (solved from R c + t = 0) to the mean, Y_k from scipy's complex
    harmonics in real form."""
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(9)
    n = 80
    P = scenegen.make_field(rng, n, 3, half_extent=1.0, sh_rest_std=0.5)
    cam = _cam_general()
    pr = geometry.project_view(_P(P, n), cam, 3)
    c = np.linalg.solve(cam["R"].astype(np.float64), -cam["t"].astype(np.float64))
    d = P[0:3, :n].astype(np.float64) - c[:, None]
    d /= np.linalg.norm(d, axis=0)
    theta, phi = np.arccos(np.clip(d[2], -1, 1)), np.arctan2(d[1], d[0])
    Y = []
    for l in range(4):
        for m in range(-l, l + 1):
            z = sph_harm_y(l, abs(m), theta, phi)
            Y.append(z.real if m == 0 else math.sqrt(2) * (z.real if m > 0 else z.imag))
    Y = np.array(Y)
    f = P[11:, :n].astype(np.float64).reshape(16, 3, n)
    ref = np.maximum(np.einsum("kcn,kn->cn", f, Y) + 0.5, 0.0)
    # the fp32 camera rotation is orthonormal to ~1e-7 only, so -R^T t and the
    # solved centre differ at that level
    assert np.abs(pr["rgb"].numpy() - ref).max() < 1e-5
    assert (ref == 0).any() and (ref > 0).any()


def test_box_min_matches_dense_sampling():
    """Closed-form minimum of a positive-definite quadratic over a box against a
    dense grid over the box (the grid can only be above it, and not by much)."""
    rng = np.random.default_rng(13)
    for _ in range(300):
        Lm = rng.normal(size=(2, 2))
        A = Lm @ Lm.T + 0.05 * np.eye(2)
        a, b, c = A[0, 0], A[0, 1], A[1, 1]
        dx0, dy0 = rng.uniform(-6, 4, 2)
        dx1, dy1 = dx0 + rng.uniform(0.1, 5), dy0 + rng.uniform(0.1, 5)
        qm = float(binning.box_min_q(np.float64(a), np.float64(b), np.float64(c), np.float64(dx0),
                                     np.float64(dx1), np.float64(dy0), np.float64(dy1)))
        X, Y = np.meshgrid(np.linspace(dx0, dx1, 201), np.linspace(dy0, dy1, 201))
        grid = a * X * X + 2 * b * X * Y + c * Y * Y
        assert grid.min() >= qm - 1e-12 * max(1.0, abs(qm))
        step = max(dx1 - dx0, dy1 - dy0) / 200
        gmax = 2 * max(abs(a) + abs(b), abs(b) + abs(c)) * (max(abs(dx0), abs(dx1), abs(dy0), abs(dy1)) + 1)
        assert grid.min() - qm <= gmax * step


@pytest.mark.parametrize("tile", [16, 8])
def test_ellipse_culling_box_is_the_hull_of_pixel_centres(tile):
    """A pair is kept exactly when the cutoff ellipse meets the rectangle spanned by
    the centres of the tile's pixels that lie inside the image (the box found here by
    listing those pixels; its minimum of the quadratic form by box_min_q, pinned by
    dense sampling).  Ragged image sides make the last row and column of tiles
    partial."""
    W, H = 90, 70
    sc = scenegen.small_scene(15, 400, 0, [(W, H)], log_scale_mean=-1.8, half_extent=1.6, depth=2.5)
    p = geometry.project_views(sc.params, sc.n, 0, sc.cams, tile)[0]
    full = binning.bin_pairs([p], sc.cams, tile, cull="rect")
    kept = binning.bin_pairs([p], sc.cams, tile, cull="ellipse")
    tiles_x = (W + tile - 1) // tile
    kset = set(zip((kept["keys"] >> np.uint64(32)).astype(np.int64).tolist(), kept["values"].tolist()))
    u, w = p["u"].numpy(), p["w"].numpy()
    a, b, c, tau = (p[k].numpy() for k in ("a", "b", "c", "tau"))
    want = set()
    for key, g in zip(full["keys"], full["values"]):
        t, g = int(key >> np.uint64(32)), int(g)
        tx, ty = t % tiles_x, t // tiles_x
        xs = [x + 0.5 for x in range(tx * tile, (tx + 1) * tile) if x < W]
        ys = [y + 0.5 for y in range(ty * tile, (ty + 1) * tile) if y < H]
        q = binning.box_min_q(np.array([a[g]]), np.array([b[g]]), np.array([c[g]]), np.array([min(xs) - u[g]]),
                              np.array([max(xs) - u[g]]), np.array([min(ys) - w[g]]), np.array([max(ys) - w[g]]))
        if q[0] <= -2.0 * tau[g]:
            want.add((t, g))
    assert kset == want
    assert len(want) < len(full["keys"])


@pytest.mark.parametrize("tile", [16, 8])
def test_ellipse_culling_keeps_every_contributing_tile(tile):
    """Every (Gaussian, tile) pair with a pixel centre that passes the cutoff is
    kept; the culled pairs hold none; culling removes a real share of the rect."""
    sc = scenegen.small_scene(14, 300, 0, [(90, 70)], log_scale_mean=-2.0, half_extent=1.2, depth=2.5)
    p = geometry.project_views(sc.params, sc.n, 0, sc.cams, tile)[0]
    full = binning.bin_pairs([p], sc.cams, tile, cull="rect")
    kept = binning.bin_pairs([p], sc.cams, tile, cull="ellipse")
    tiles_x = (90 + tile - 1) // tile
    kset = set(zip((kept["keys"] >> np.uint64(32)).astype(np.int64).tolist(), kept["values"].tolist()))
    u, w = p["u"].numpy(), p["w"].numpy()
    a, b, c, tau = (p[k].numpy() for k in ("a", "b", "c", "tau"))
    n_contrib_pairs = 0
    for key, g in zip(full["keys"], full["values"]):
        t = int(key >> np.uint64(32))
        tx, ty = t % tiles_x, t // tiles_x
        xs = np.arange(tx * tile, min((tx + 1) * tile, 90)) + 0.5
        ys = np.arange(ty * tile, min((ty + 1) * tile, 70)) + 0.5
        X, Y = np.meshgrid(xs - u[g], ys - w[g])
        power = -0.5 * (a[g] * X * X + c[g] * Y * Y) - b[g] * X * Y
        margin = (power - tau[g]) / (abs(tau[g]) + np.abs(power) + 1e-12)
        if (margin > 1e-6).any():
            n_contrib_pairs += 1
            assert (t, int(g)) in kset
        if (t, int(g)) not in kset:
            assert (margin < 1e-6).all()
    assert len(kept["keys"]) < 0.9 * len(full["keys"])
    assert n_contrib_pairs > 0.5 * len(kept["keys"])
