"""Per-view geometry of every Gaussian, in FP64 (oracle; test infrastructure only).

Follows Eq. 1 (Sec. III): a Gaussian centred at X0 with covariance
Sigma = R S S^T R^T.  The projection to the image (EWA splatting), the extent,
the cutoff and the tile rect are not written out in the paper; they follow the
original 3DGS configuration (Sec. V-A, implementation details); each reading is
stated at the function that takes it (pixel centres at half-integers, near plane
0.2, Jacobian clamp 1.3x the half field of view, dilation 0.3 px^2, extent
3 sqrt(lambda_max), cutoff tau = max(-4.5, -ln(255 o))).

Every decision quantity (camera depth, screen position, 2D covariance and its
largest eigenvalue) is evaluated in FP64 from the fp32 inputs in a fixed operation
order: left-to-right sums of products, written out term by term below.  Products of
two fp32 numbers are exact in FP64, so depth and screen position are reproducible
by any IEEE FP64 evaluation in the same order.
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np
import torch

from .constants import (KAPPA, Z_NEAR, JAC_CLAMP, EXTENT_SIGMAS, CUTOFF_FLOOR, ALPHA_MIN_INV,
                        SH_OFFSET)
from .sh import sh_basis

F64 = torch.float64


def n_sh(sh_degree: int) -> int:
    return (sh_degree + 1) ** 2


def as_f64(x) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(F64)
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


def activations(P: torch.Tensor):
    """Scale s = exp(log-scale), unit quaternion q/|q|, opacity = sigmoid(logit)."""
    s = [torch.exp(P[3 + i]) for i in range(3)]
    qw, qx, qy, qz = P[6], P[7], P[8], P[9]
    qn = torch.sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz)
    q = (qw / qn, qx / qn, qy / qn, qz / qn)
    o = 1.0 / (1.0 + torch.exp(-P[10]))
    return s, q, o


def rotation(q):
    """Rotation matrix of the unit quaternion (w, x, y, z), as nested rows."""
    w, x, y, z = q
    return [[1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)],
            [2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)],
            [2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)]]


def covariance3d(s, q):
    """Eq. 1: Sigma = R S S^T R^T with M = R S, i.e. Sigma_kl = sum_j M_kj M_lj."""
    R = rotation(q)
    M = [[R[k][j] * s[j] for j in range(3)] for k in range(3)]
    return [[(M[k][0] * M[l][0] + M[k][1] * M[l][1]) + M[k][2] * M[l][2] for l in range(3)]
            for k in range(3)]


def _cam_floats(cam):
    R = [[float(np.float32(cam["R"][i][j])) for j in range(3)] for i in range(3)]
    t = [float(np.float32(cam["t"][i])) for i in range(3)]
    return R, t


def camera_center(cam):
    """o_v = -R^T t."""
    R, t = _cam_floats(cam)
    return [-((R[0][k] * t[0] + R[1][k] * t[1]) + R[2][k] * t[2]) for k in range(3)]


def tile_layout(cams, tile: int):
    """Tiles per row/column of each view and the global tile offset of each view
    (views are numbered consecutively; tile (tx, ty) of view v has global id
    tile_off[v] + ty * tiles_x[v] + tx)."""
    tiles_x = [(c["width"] + tile - 1) // tile for c in cams]
    tiles_y = [(c["height"] + tile - 1) // tile for c in cams]
    off = [0]
    for a, b in zip(tiles_x, tiles_y):
        off.append(off[-1] + a * b)
    return tiles_x, tiles_y, off


def project_view(P: torch.Tensor, cam: dict, sh_degree: int, tile: int = 16) -> Dict[str, object]:
    """Everything one view needs from each Gaussian.

    P: FP64 tensor [n_params, N] (may require grad).  Returns a dict with FP64
    tensors u, w (pixel-space centre), a, b, c (conic), o (opacity), tau (cutoff),
    rgb [3, N] (clamped colour), tz (depth), lam (largest eigenvalue), r (extent)
    and numpy arrays visible, depth_bits (fp32 bit pattern of tz), pixel rect
    i0, i1, j0, j1, tile rect tx0, tx1, ty0, ty1 and touched (number of tiles).
    """
    R, t = _cam_floats(cam)
    fx, fy = float(np.float32(cam["fx"])), float(np.float32(cam["fy"]))
    cx, cy = float(np.float32(cam["cx"])), float(np.float32(cam["cy"]))
    W, H = int(cam["width"]), int(cam["height"])

    mx, my, mz = P[0], P[1], P[2]
    s, q, o = activations(P)
    Sig = covariance3d(s, q)

    # camera transform x_cam = R_v mu + t_v
    tx = ((R[0][0] * mx + R[0][1] * my) + R[0][2] * mz) + t[0]
    ty = ((R[1][0] * mx + R[1][1] * my) + R[1][2] * mz) + t[1]
    tz = ((R[2][0] * mx + R[2][1] * my) + R[2][2] * mz) + t[2]
    in_front = (tz > Z_NEAR).detach().numpy()
    # guard the divisions for culled Gaussians; their values are never used
    tzs = torch.where(tz > Z_NEAR, tz, torch.ones_like(tz))

    # pinhole projection, pixel (i, j) has its centre at (i + 1/2, j + 1/2)
    u = (fx * tx) / tzs + cx
    w = (fy * ty) / tzs + cy

    # EWA: Jacobian of the projection at the camera point, clamped off axis
    limx = (JAC_CLAMP * (0.5 * W)) / fx
    limy = (JAC_CLAMP * (0.5 * H)) / fy
    txc = tzs * torch.clamp(tx / tzs, -limx, limx)
    tyc = tzs * torch.clamp(ty / tzs, -limy, limy)
    J00 = fx / tzs
    J02 = -(fx * txc) / (tzs * tzs)
    J11 = fy / tzs
    J12 = -(fy * tyc) / (tzs * tzs)
    # T = J W (W = R_v); row 0 has J01 = 0, row 1 has J10 = 0
    T0 = [J00 * R[0][k] + J02 * R[2][k] for k in range(3)]
    T1 = [J11 * R[1][k] + J12 * R[2][k] for k in range(3)]
    U0 = [(T0[0] * Sig[0][l] + T0[1] * Sig[1][l]) + T0[2] * Sig[2][l] for l in range(3)]
    U1 = [(T1[0] * Sig[0][l] + T1[1] * Sig[1][l]) + T1[2] * Sig[2][l] for l in range(3)]
    S00 = ((U0[0] * T0[0] + U0[1] * T0[1]) + U0[2] * T0[2]) + KAPPA
    S01 = (U0[0] * T1[0] + U0[1] * T1[1]) + U0[2] * T1[2]
    S11 = ((U1[0] * T1[0] + U1[1] * T1[1]) + U1[2] * T1[2]) + KAPPA

    # conic = inverse of the 2D covariance
    det = S00 * S11 - S01 * S01
    det_ok = (det > 0).detach().numpy()
    dets = torch.where(det > 0, det, torch.ones_like(det))
    a = S11 / dets
    b = -S01 / dets
    c = S00 / dets

    # extent: 3 sqrt(largest eigenvalue); cutoff exponent
    lam = 0.5 * (S00 + S11) + torch.sqrt(0.25 * ((S00 - S11) * (S00 - S11)) + S01 * S01)
    r = EXTENT_SIGMAS * torch.sqrt(lam)
    tau = torch.clamp(-torch.log(ALPHA_MIN_INV * o), min=CUTOFF_FLOOR)

    # pixel rect: pixel centres within [u - r, u + r] x [w - r, w + r], inside the image
    with torch.no_grad():
        un, wn, rn = u.detach().numpy(), w.detach().numpy(), r.detach().numpy()
        with np.errstate(invalid="ignore", over="ignore"):
            xlo, xhi = np.ceil((un - rn) - 0.5), np.floor((un + rn) - 0.5)
            ylo, yhi = np.ceil((wn - rn) - 0.5), np.floor((wn + rn) - 0.5)
            i0 = np.nan_to_num(np.clip(xlo, 0, W), nan=W).astype(np.int64)
            i1 = np.nan_to_num(np.clip(xhi, -1, W - 1), nan=-1).astype(np.int64)
            j0 = np.nan_to_num(np.clip(ylo, 0, H), nan=H).astype(np.int64)
            j1 = np.nan_to_num(np.clip(yhi, -1, H - 1), nan=-1).astype(np.int64)
        visible = in_front & det_ok & (i0 <= i1) & (j0 <= j1)
        tx0, tx1, ty0, ty1 = i0 // tile, i1 // tile, j0 // tile, j1 // tile
        touched = np.where(visible, (tx1 - tx0 + 1) * (ty1 - ty0 + 1), 0).astype(np.int64)
        depth_bits = tz.detach().to(torch.float32).numpy().view(np.uint32).copy()

    # view-dependent colour: SH evaluated at the unit direction from the camera centre
    oc = camera_center(cam)
    dx_, dy_, dz_ = mx - oc[0], my - oc[1], mz - oc[2]
    dn = torch.sqrt((dx_ * dx_ + dy_ * dy_) + dz_ * dz_)
    Y = sh_basis(dx_ / dn, dy_ / dn, dz_ / dn, sh_degree)          # [K, N]
    K = n_sh(sh_degree)
    raw = []
    for ch in range(3):
        acc = SH_OFFSET + 0.0 * mx
        for k in range(K):
            acc = acc + P[11 + 3 * k + ch] * Y[k]
        raw.append(acc)
    raw = torch.stack(raw)
    rgb = torch.clamp(raw, min=0.0)

    return dict(u=u, w=w, a=a, b=b, c=c, o=o, tau=tau, rgb=rgb, rgb_raw=raw, tz=tz, lam=lam, r=r,
                S00=S00, S01=S01, S11=S11, visible=visible, depth_bits=depth_bits,
                i0=i0, i1=i1, j0=j0, j1=j1, tx0=tx0, tx1=tx1, ty0=ty0, ty1=ty1, touched=touched,
                width=W, height=H, bg=[float(np.float32(x)) for x in cam["bg"]])


def params_f64(params32: np.ndarray, n: int, requires_grad: bool = False) -> torch.Tensor:
    P = torch.as_tensor(np.ascontiguousarray(params32[:, :n]).astype(np.float64))
    if requires_grad:
        P.requires_grad_(True)
    return P


def project_views(params32: np.ndarray, n: int, sh_degree: int, cams: List[dict], tile: int = 16):
    with torch.no_grad():
        P = params_f64(params32, n)
        return [project_view(P, c, sh_degree, tile) for c in cams]
