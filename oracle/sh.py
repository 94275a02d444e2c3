"""Real spherical-harmonic basis up to degree 3 (oracle; test infrastructure only).

Sec. III says the colour of each Gaussian comes from spherical harmonics; the basis
(order, normalisation, signs) follows the original 3DGS configuration (Sec. V-A).
That basis is the real form of the Condon-Shortley-phased complex harmonics Y_l^m:

  m > 0:  sqrt(2) Re Y_l^m,   m = 0:  Y_l^0,   m < 0:  sqrt(2) Im Y_l^|m|,

ordered k = l^2 + l + m.  It is evaluated here from its general closed form on the
unit sphere, not from per-term polynomials:

  Y_l^m = N_lm (-1)^m [d^m P_l / dz^m](z) (x + i y)^m,
  N_lm  = sqrt((2l+1)/(4 pi) * (l-m)! / (l+m)!),

with the Legendre polynomial P_l taken from numpy's Legendre series.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


@lru_cache(maxsize=None)
def _terms(degree: int):
    out = []
    for l in range(degree + 1):
        pl = npleg.leg2poly([0] * l + [1])           # power-series coefficients of P_l(z)
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            deriv = nppoly.polyder(pl, am) if am else pl
            coef = norm * ((-1) ** am) * (math.sqrt(2.0) if m != 0 else 1.0)
            out.append((m, coef, tuple(float(v) for v in np.atleast_1d(deriv))))
    return tuple(out)


def _horner(coeffs, z):
    acc = 0.0 * z + coeffs[-1]
    for cf in reversed(coeffs[:-1]):
        acc = acc * z + cf
    return acc


def sh_basis(x, y, z, degree: int):
    """Basis values Y_k(x, y, z) for k < (degree+1)^2 at unit directions; x, y, z may
    be numpy arrays or torch tensors (differentiable).  Returns a list (torch) or an
    array (numpy) with the k axis first."""
    vals = []
    for m, coef, deriv in _terms(degree):
        pz = _horner(deriv, z)
        if m == 0:
            vals.append(coef * pz)
            continue
        re, im = 1.0 + 0.0 * x, 0.0 * x
        for _ in range(abs(m)):
            re, im = re * x - im * y, re * y + im * x
        vals.append(coef * pz * (re if m > 0 else im))
    if isinstance(x, np.ndarray):
        return np.stack(vals)
    return vals
