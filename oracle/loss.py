"""Image losses and their gradient w.r.t. the rendered image (oracle; test
infrastructure only).

Eq. 10 combines an L1 term, an SSIM term and the load-balancing term of Eq. 9.  The SSIM term follows the original 3DGS
configuration (Sec. V-A): per channel, windowed statistics under a normalised
11x11 Gaussian window with sigma 1.5 and zero padding outside the image, constants
C1 = 0.01^2 and C2 = 0.03^2, averaged over pixels and channels; D-SSIM = 1 - SSIM.
Loss of a view = w_l1 * mean|x - y| + w_dssim * (1 - SSIM(x, y)); a batch of views
sums the per-view losses.  The gradient is taken by reverse-mode automatic
differentiation of this definition in FP64.
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

F64 = torch.float64
C1 = 0.01 ** 2
C2 = 0.03 ** 2
WIN = 11
SIGMA = 1.5


def gaussian_window_1d(size=WIN, sigma=SIGMA) -> torch.Tensor:
    x = torch.arange(size, dtype=F64) - (size // 2)
    g = torch.exp(-(x * x) / (2.0 * sigma * sigma))
    return g / g.sum()


def blur(img: torch.Tensor) -> torch.Tensor:
    """Windowed mean of each channel of img [C, H, W] with zero padding."""
    g = gaussian_window_1d()
    w2 = (g[:, None] * g[None, :])[None, None].expand(img.shape[0], 1, WIN, WIN).contiguous()
    return F.conv2d(img[None], w2, padding=WIN // 2, groups=img.shape[0])[0]


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def image_loss(x: torch.Tensor, y: torch.Tensor, w_l1: float, w_dssim: float) -> torch.Tensor:
    """Loss of one view; x, y FP64 [3, H, W]."""
    val = w_l1 * (x - y).abs().mean()
    if w_dssim != 0.0:
        val = val + w_dssim * (1.0 - ssim_map(x, y).mean())
    return val


def image_loss_and_grad(x32, y32, w_l1: float, w_dssim: float):
    """Loss value (float) and dL/dx (FP64 numpy [3, H, W]) of one view, from fp32 or
    FP64 images promoted to FP64."""
    x = torch.as_tensor(np.asarray(x32, np.float64)).clone().requires_grad_(True)
    y = torch.as_tensor(np.asarray(y32, np.float64))
    val = image_loss(x, y, w_l1, w_dssim)
    val.backward()
    return float(val.detach()), x.grad.numpy()


def load_balance_loss_and_grad(G):
    """Eq. 9: L_load = std over the pixels of one image of G_p, the number of
    Gaussians associated with pixel p.  Readings: a count has no derivative, so
    G_p is the soft count sum_k alpha_k over the Gaussians blended at p (it grows
    by up to 0.99 per blended Gaussian and moves every blended Gaussian's alpha);
    std is the population standard deviation over all pixels of the image; its
    derivative at std = 0 is taken as 0.  Returns (value, dL/dG) for G [H, W]."""
    g = torch.as_tensor(np.asarray(G, np.float64)).clone().requires_grad_(True)
    var = ((g - g.mean()) ** 2).mean()
    if float(var.detach()) == 0.0:
        return 0.0, np.zeros(g.shape)
    val = torch.sqrt(var)
    val.backward()
    return float(val.detach()), g.grad.numpy()
