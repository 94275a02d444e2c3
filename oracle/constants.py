"""Rasterizer constants (oracle side).

The paper fixes none of these (Sec. III gives Eq. 1-2 only; Sec. V-A says the other
settings follow the original 3DGS configuration).  Each is the fp32 value of the
3DGS-lineage constant, promoted to FP64, so that the oracle and an fp32 device
implementation start from the same number.
"""
import numpy as np


def _f32(x: float) -> float:
    return float(np.float32(x))


KAPPA = _f32(0.3)         # low-pass dilation added to both diagonal entries of the 2D covariance (px^2)
Z_NEAR = _f32(0.2)        # camera-space depth at or below which a Gaussian is culled
ALPHA_MAX = _f32(0.99)    # cap on a single splat's alpha
T_MIN = _f32(1e-4)        # transmittance below which a pixel stops blending
JAC_CLAMP = _f32(1.3)     # off-axis clamp of the projection Jacobian, in units of the half field of view
EXTENT_SIGMAS = 3.0       # screen extent radius = 3 * sqrt(largest 2D eigenvalue)
CUTOFF_FLOOR = -4.5       # -(3^2)/2: the 3-sigma ellipse in the exponent of Eq. 1
ALPHA_MIN_INV = 255.0     # a splat contributes only when its alpha >= 1/255
SH_OFFSET = 0.5           # added to the SH colour before clamping at 0
