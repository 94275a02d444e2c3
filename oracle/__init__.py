"""Oracle: a plain, slow, FP64 CPU definition of the rasterizer hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute
this package; only the tests, the smoke check and the benchmark's CPU-baseline leg
use it.  It shares no code with the HIP implementation (the only shared module is
the seeded input generator, which holds none of the method's arithmetic).

What it computes (Gaussian On-the-Fly Splatting, Sec. III and Sec. IV-E; the
remaining conventions follow the original 3DGS configuration, as Sec. V-A states):

  geometry.py   Eq. 1 covariance, camera transform, EWA projection, conic, extent,
                cutoff and pixel/tile rect of each Gaussian in each view
  sh.py         view-dependent colour from real spherical harmonics
  composite.py  Eq. 2 front-to-back alpha blending per pixel
  binning.py    (tile, depth, index) keys, their sort and per-tile ranges
  loss.py       L1 and D-SSIM image losses (Eq. 10 terms) and dL/dimage
  grad.py       gradients of the loss w.r.t. every Gaussian parameter
  adam.py       the Adam step with a learning rate per view (Eq. 6-8 feed it)
  schedule.py   Eq. 3-8 host scalars (hierarchical weights, iteration budget,
                per-image learning rate)
  brute.py      scalar pure-Python compositing for tiny scenes (a pin for composite)

Every function states the passage it follows and the reading it takes where the
paper is silent.
"""
from . import constants  # noqa: F401
from .geometry import project_view, project_views, tile_layout  # noqa: F401
from .sh import sh_basis  # noqa: F401
from .composite import composite_pixels, render_view, render_views  # noqa: F401
from .binning import bin_pairs  # noqa: F401
from .loss import image_loss, image_loss_and_grad  # noqa: F401
from .grad import param_grads  # noqa: F401
from .adam import adam_step  # noqa: F401
from . import schedule  # noqa: F401
