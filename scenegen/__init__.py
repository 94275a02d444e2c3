"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and builds cameras; it contains none of the
rasterizer's arithmetic (no projection, covariance, colour or compositing).  The
scenes stand in for the paper's datasets (Sec. V-A), which are not available:
field sizes mimic the model sizes of Table I (about 0.5M to 3.4M Gaussians) and the
image sizes match the resolutions of the evaluated scenes.

Parameter layout (one fp32 array of shape [n_params, stride], planar, column g is
Gaussian g):
  rows 0..2   mean (x, y, z), world units
  rows 3..5   log-scale per axis
  rows 6..9   rotation quaternion (w, x, y, z), not necessarily normalised
  row  10     opacity logit
  rows 11..   SH coefficients, coefficient k and channel c at row 11 + 3*k + c,
              k < (sh_degree+1)^2
Cameras are dicts with R (3x3, world->camera, x right / y down / z forward),
t (3,), fx, fy, cx, cy, width, height, bg (3,), all fp32 except the integer size.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# DC normalisation of the degree-0 SH basis function, 1/(2*sqrt(pi)); used only to
# draw DC coefficients so that the rendered base colour is uniform in [0, 1].
_DC_NORM = 0.5 / math.sqrt(math.pi)

RESOLUTIONS_C3 = [(1600, 1067), (1296, 864), (979, 546)]


def n_params(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


@dataclass
class Scene:
    params: np.ndarray          # fp32 [n_params, stride]
    n: int
    sh_degree: int
    cams: List[dict]
    targets: List[np.ndarray]   # fp32 [3, H, W] per view
    w_l1: float = 1.0
    w_dssim: float = 0.0
    iters: Optional[np.ndarray] = None   # per-view trained-iteration counters
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def stride(self) -> int:
        return self.params.shape[1]


def make_field(rng: np.random.Generator, n: int, sh_degree: int, *, center=(0.0, 0.0, 0.0),
               half_extent=1.0, log_scale_mean=-3.5, log_scale_std=0.5, sh_rest_std=0.1,
               stride: Optional[int] = None) -> np.ndarray:
    """Random Gaussian field; draws in a fixed order so a seed fixes every value."""
    stride = n if stride is None else stride
    assert stride >= n
    k = (sh_degree + 1) ** 2
    P = np.zeros((n_params(sh_degree), stride), np.float32)
    mean = rng.uniform(-half_extent, half_extent, size=(3, n)) + np.asarray(center, np.float64)[:, None]
    P[0:3, :n] = mean
    P[3:6, :n] = rng.normal(log_scale_mean, log_scale_std, size=(3, n))
    q = rng.normal(0.0, 1.0, size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    P[6:10, :n] = q
    P[10, :n] = rng.normal(0.0, 1.0, size=n)
    dc = (rng.uniform(0.0, 1.0, size=(3, n)) - 0.5) / _DC_NORM
    P[11:14, :n] = dc
    if k > 1:
        P[14:14 + 3 * (k - 1), :n] = rng.normal(0.0, sh_rest_std, size=(3 * (k - 1), n))
    return P


def camera(R, t, fx, fy, cx, cy, width, height, bg=(0.0, 0.0, 0.0)) -> dict:
    return dict(R=np.asarray(R, np.float32).reshape(3, 3), t=np.asarray(t, np.float32).reshape(3),
                fx=np.float32(fx), fy=np.float32(fy), cx=np.float32(cx), cy=np.float32(cy),
                width=int(width), height=int(height), bg=np.asarray(bg, np.float32).reshape(3))


def look_at(eye, target, up=(0.0, -1.0, 0.0)):
    """World->camera (R, t) for a camera at `eye` looking at `target`; camera y points
    along -up (image rows grow downwards)."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    down = -np.asarray(up, np.float64)
    down = down - down.dot(f) * f
    down /= np.linalg.norm(down)
    right = np.cross(down, f)
    R = np.stack([right, down, f])
    t = -R @ eye
    return R.astype(np.float32), t.astype(np.float32)


def pinhole(R, t, width, height, focal_frac=0.75, bg=(0.0, 0.0, 0.0)) -> dict:
    f = focal_frac * width
    return camera(R, t, f, f, width / 2.0, height / 2.0, width, height, bg)


def targets_for(rng: np.random.Generator, cams) -> List[np.ndarray]:
    return [rng.uniform(0.0, 1.0, size=(3, c["height"], c["width"])).astype(np.float32) for c in cams]


def scale_law(n: int) -> float:
    """Mean log-scale for the 20 m box scenes: ln(0.35 * (8000/n)^(1/3))."""
    return math.log(0.35 * (8000.0 / n) ** (1.0 / 3.0))


def random_walk(rng: np.random.Generator, n_poses=64, radius=25.0, step_deg=3.0, jitter=1.0):
    """Camera path on a sphere around the origin; each step perturbs azimuth and
    elevation by N(0, step_deg) and looks at the origin plus N(0, jitter) metres."""
    az, el = 0.0, 0.0
    poses = []
    for _ in range(n_poses):
        az += math.radians(rng.normal(0.0, step_deg))
        el = float(np.clip(el + math.radians(rng.normal(0.0, step_deg)), -1.2, 1.2))
        eye = radius * np.array([math.cos(el) * math.sin(az), -math.sin(el), -math.cos(el) * math.cos(az)])
        tgt = rng.normal(0.0, jitter, size=3)
        poses.append(look_at(eye, tgt))
    return poses


def in_frustum(points: np.ndarray, R, t, width, height, focal_frac=0.75, z_min=0.2) -> np.ndarray:
    """Boolean mask of world points (3, n) inside a pinhole frustum (scene selection
    geometry only)."""
    pc = np.asarray(R, np.float64) @ points + np.asarray(t, np.float64)[:, None]
    z = pc[2]
    f = focal_frac * width
    with np.errstate(divide="ignore", invalid="ignore"):
        ok = (z > z_min) & (np.abs(pc[0] / z) < width / (2 * f)) & (np.abs(pc[1] / z) < height / (2 * f))
    return ok


def rank_by_overlap(points, poses, new_idx, k, width=1296, height=864):
    """Indices of the k poses whose frustum shares the largest fraction of the new
    pose's visible points."""
    Rn, tn = poses[new_idx]
    vn = in_frustum(points, Rn, tn, width, height)
    denom = max(1, int(vn.sum()))
    scores = []
    for i, (R, t) in enumerate(poses):
        if i == new_idx:
            continue
        scores.append((-(in_frustum(points, R, t, width, height) & vn).sum() / denom, i))
    scores.sort()
    return [i for _, i in scores[:k]]


# ----------------------------------------------------------------------------------
# Workloads.  C1..C4 follow the configurations the benchmark is quoted on; the small
# scenes are parity cases that the oracle finishes in seconds.
# ----------------------------------------------------------------------------------

def config1(seed=1, n=10_000, target_seed=101) -> Scene:
    """10k Gaussians, SH degree 0, one 128x128 camera at the origin, L1 loss."""
    rng = np.random.default_rng(seed)
    P = make_field(rng, n, 0, center=(0, 0, 3.0), half_extent=1.0, log_scale_mean=-3.5)
    cam = camera(np.eye(3), np.zeros(3), 128, 128, 64, 64, 128, 128)
    tg = targets_for(np.random.default_rng(target_seed), [cam])
    return Scene(P, n, 0, [cam], tg, 1.0, 0.0, name="c1_10k_128x128_sh0")


def config2(seed=2, n=300_000) -> Scene:
    """300k Gaussians in a 20 m box, SH degree 3, one 1296x864 camera at (0,0,-25)
    looking at the origin; loss 0.8 L1 + 0.2 D-SSIM."""
    rng = np.random.default_rng(seed)
    P = make_field(rng, n, 3, half_extent=10.0, log_scale_mean=scale_law(n))
    R, t = look_at((0, 0, -25.0), (0, 0, 0))
    cam = pinhole(R, t, 1296, 864)
    tg = targets_for(rng, [cam])
    return Scene(P, n, 3, [cam], tg, 0.8, 0.2, name="c2_300k_1296x864_sh3")


def config3(seed=3, n=1_000_000, n_views=9, n_poses=64) -> Scene:
    """1M Gaussians, SH degree 3, the newest pose of a 64-pose random walk plus its 8
    neighbours ranked by frustum overlap, resolutions cycling 1600x1067, 1296x864,
    979x546; per-view trained-iteration counters U{0..30000}."""
    rng = np.random.default_rng(seed)
    P = make_field(rng, n, 3, half_extent=10.0, log_scale_mean=scale_law(n))
    poses = random_walk(rng, n_poses)
    new = n_poses - 1
    sample = P[0:3, : min(n, 200_000)].astype(np.float64)
    nb = rank_by_overlap(sample, poses, new, n_views - 1)
    order = [new] + nb
    cams = []
    for vi, pi in enumerate(order):
        W, H = RESOLUTIONS_C3[vi % 3]
        cams.append(pinhole(poses[pi][0], poses[pi][1], W, H))
    tg = targets_for(rng, cams)
    iters = rng.integers(0, 30001, size=n_views)
    return Scene(P, n, 3, cams, tg, 0.8, 0.2, iters=iters, name="c3_1M_9views_sh3",
                 extra=dict(pose_order=order))


def config4(seed=4, n=3_000_000) -> Scene:
    """3M Gaussians, SH degree 3, one 1920x1080 view (f=1440)."""
    rng = np.random.default_rng(seed)
    P = make_field(rng, n, 3, half_extent=10.0, log_scale_mean=scale_law(n))
    R, t = look_at((0, 0, -25.0), (0, 0, 0))
    cam = pinhole(R, t, 1920, 1080)
    tg = targets_for(rng, [cam])
    return Scene(P, n, 3, [cam], tg, 0.8, 0.2, name="c4_3M_1920x1080_sh3")


def small_scene(seed: int, n: int, sh_degree: int, sizes, *, log_scale_mean=-2.6, half_extent=1.0,
                depth=3.0, focal_frac=0.9, bg=(0.0, 0.0, 0.0), w_l1=1.0, w_dssim=0.0, stride=None,
                spread_deg=8.0) -> Scene:
    """Parity-sized scene: a cube of Gaussians at `depth` in front of the cameras,
    one camera per entry of `sizes` (width, height), each slightly rotated about the
    cube centre so views differ."""
    rng = np.random.default_rng(seed)
    P = make_field(rng, n, sh_degree, center=(0, 0, 0), half_extent=half_extent,
                   log_scale_mean=log_scale_mean, stride=stride)
    cams = []
    for vi, (W, H) in enumerate(sizes):
        az = math.radians(spread_deg * vi * (1 if vi % 2 else -1))
        eye = depth * np.array([math.sin(az), 0.0, -math.cos(az)])
        R, t = look_at(eye, (0, 0, 0))
        cams.append(pinhole(R, t, W, H, focal_frac, bg))
    tg = targets_for(rng, cams)
    return Scene(P, n, sh_degree, cams, tg, w_l1, w_dssim, name=f"small_s{seed}_n{n}_d{sh_degree}")


def opaque_scene(seed: int, n: int, sh_degree: int, sizes, *, frac=0.2, logit_range=(6.0, 9.0),
                 opaque_log_scale=-1.6, **kw) -> Scene:
    """small_scene with a fraction `frac` of nearly opaque Gaussians: their opacity
    logits are drawn from U(logit_range), so o > 0.9975 and their alpha reaches the
    0.99 cap within about a seventh of a standard deviation of their centre; their
    log-scales are drawn around opaque_log_scale (several pixels across), so that
    region holds pixel centres (a pixel behind two of them stops at the third)."""
    sc = small_scene(seed, n, sh_degree, sizes, **kw)
    rng = np.random.default_rng(seed + 7919)
    pick = rng.choice(n, int(frac * n), replace=False)
    sc.params[10, pick] = rng.uniform(logit_range[0], logit_range[1], size=len(pick))
    sc.params[3:6, pick] = rng.normal(opaque_log_scale, 0.3, size=(3, len(pick)))
    sc.name = f"opaque_s{seed}_n{n}_d{sh_degree}"
    return sc


def edge_scene(seed: int, n_inner: int, n_edge: int, sh_degree: int, sizes, *, edge_log_scale=-1.0,
               depth_range=(2.5, 3.5), beyond=(1.35, 1.65), **kw) -> Scene:
    """small_scene plus n_edge large Gaussians placed, for the first camera, just
    outside 1.3x its half field of view in x or in y (the direction tangent is
    `beyond` times the half field of view) at depths in depth_range, with log-scales
    around edge_log_scale, so their footprints still reach into the image."""
    sc = small_scene(seed, n_inner, sh_degree, sizes, **kw)
    rng = np.random.default_rng(seed + 104729)
    cam = sc.cams[0]
    hx = 0.5 * cam["width"] / float(cam["fx"])
    hy = 0.5 * cam["height"] / float(cam["fy"])
    E = make_field(rng, n_edge, sh_degree, log_scale_mean=edge_log_scale, log_scale_std=0.25)
    z = rng.uniform(depth_range[0], depth_range[1], n_edge)
    side = rng.integers(0, 4, n_edge)                      # +x, -x, +y, -y
    out = rng.uniform(beyond[0], beyond[1], n_edge)
    sx = np.where(side < 2, out * hx * np.where(side == 0, 1.0, -1.0), rng.uniform(-hx, hx, n_edge))
    sy = np.where(side >= 2, out * hy * np.where(side == 2, 1.0, -1.0), rng.uniform(-hy, hy, n_edge))
    xc = np.stack([sx * z, sy * z, z])                      # camera coordinates
    R = np.asarray(cam["R"], np.float64)
    t = np.asarray(cam["t"], np.float64)
    E[0:3] = R.T @ (xc - t[:, None])                        # world = R^T (x_cam - t)
    E[10] = rng.normal(1.0, 1.0, n_edge)
    sc.params = np.concatenate([sc.params[:, :n_inner], E], axis=1)
    sc.n = n_inner + n_edge
    sc.name = f"edge_s{seed}_n{n_inner}+{n_edge}_d{sh_degree}"
    return sc


def upstream_grads(seed: int, cams, scale=1e-3) -> List[np.ndarray]:
    """Seeded synthetic dL/dcolor images (fp32 [3, H, W] per view)."""
    rng = np.random.default_rng(seed)
    return [(rng.normal(0.0, scale, size=(3, c["height"], c["width"]))).astype(np.float32) for c in cams]


def _axis_angle(a, b) -> float:
    ca = float(np.clip(np.dot(np.asarray(a[0], np.float64)[2], np.asarray(b[0], np.float64)[2]), -1.0, 1.0))
    return math.degrees(math.acos(ca))


@dataclass
class Arrival:
    """One image of an on-the-fly stream: when it arrives, its camera, the Gaussians
    appended to the field for it, and its overlap degree with each earlier image."""
    time: float
    cam: dict
    block: np.ndarray
    overlap: np.ndarray
    target_seed: int

    def target(self) -> np.ndarray:
        rng = np.random.default_rng(self.target_seed)
        return rng.uniform(0.0, 1.0, size=(3, self.cam["height"], self.cam["width"])).astype(np.float32)


@dataclass
class Stream:
    initial: np.ndarray
    sh_degree: int
    arrivals: List[Arrival]
    name: str = "stream"


def serving_stream(seed=5, n_arrivals=200, n0=50_000, add=(5_000, 20_000), size=(1296, 864), sh_degree=3,
                   mean_interarrival=2.0, n_landmarks=20_000, block_half_extent=3.0, match_deg=20.0) -> Stream:
    """Images arriving along a random-walk camera path at Poisson times
    (exponential gaps of mean `mean_interarrival` seconds, the first at 0).  The
    field starts with n0 Gaussians in the 20 m box (scale law at n0); each arrival
    appends U{add} Gaussians in a cube around a point on its optical axis 0.9 of
    the way to the look-at point (scale law at 2.5M).  The overlap degree of two
    images (the stand-in for the matched feature points an online SfM reports) is
    the fraction of the new image's visible landmarks (uniform points in the box)
    that the earlier image also sees, tapered linearly to 0 as the angle between
    the two optical axes grows to match_deg (feature matching fails across large
    viewpoint changes)."""
    rng = np.random.default_rng(seed)
    W, H = size
    initial = make_field(rng, n0, sh_degree, half_extent=10.0, log_scale_mean=scale_law(n0))
    poses = random_walk(rng, n_arrivals)
    gaps = rng.exponential(mean_interarrival, size=n_arrivals)
    gaps[0] = 0.0
    times = np.cumsum(gaps)
    marks = rng.uniform(-10.0, 10.0, size=(3, n_landmarks))
    vis = [in_frustum(marks, R, t, W, H) for (R, t) in poses]
    arrivals = []
    for i, (R, t) in enumerate(poses):
        R64 = np.asarray(R, np.float64)
        eye = -R64.T @ np.asarray(t, np.float64)
        centre = eye + 0.9 * np.linalg.norm(eye) * R64[2]
        k = int(rng.integers(add[0], add[1] + 1))
        block = make_field(rng, k, sh_degree, center=centre, half_extent=block_half_extent,
                           log_scale_mean=scale_law(2_500_000))
        nv = max(1, int(vis[i].sum()))
        ov = np.array([(vis[i] & vis[j]).sum() / nv * max(0.0, 1.0 - _axis_angle(poses[i], poses[j]) / match_deg)
                       for j in range(i)], np.float64)
        arrivals.append(Arrival(float(times[i]), pinhole(R, t, W, H), block, ov, int(rng.integers(0, 2**63 - 1))))
    return Stream(initial, sh_degree, arrivals, name=f"stream_{n_arrivals}x{W}x{H}_n0_{n0}")
