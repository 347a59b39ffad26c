"""The four operators of the path, written as their definitions (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4 closes with E_s^* X = W^{-1}(D (W X)) with W the fast wavelet transform
and D the level-weight diagonal.  With W orthogonal (periodic boundary) and
D_tau the diagonal holding 2^{-tau s (m-i)} on the detail bands of level i and
1 on the approximation:

  es_adjoint(x)       = D_s W x          pixels -> packed coefficients
  es_apply(c)         = W^T D_s c        packed coefficients -> pixels
  matern_cov_apply(x) = W^T D_{2s} W x   = es_apply(es_adjoint(x)): the paper's
                                           pixel-space E_s^* (Sec. 4) and, up to
                                           the constant of Prop. 3.2 that
                                           Remark 3.3 drops, the Matern covariance
                                           with s = nu + d/2
  matern_sample(xi)   = W^T D_s W xi     symmetric square root of the covariance

es_adjoint / es_apply are E_s^* and E_s written in orthonormal wavelet
coordinates of H^s (so that they are Euclidean adjoints of each other); their
product is exactly the paper's pixel-space operator.  Inputs are promoted to
float64 before any arithmetic.
"""

import numpy as np

from .dwt import dwt, idwt, weight_map
from .filters import daubechies_lowpass


def _prep(x):
    return np.asarray(x, dtype=np.float64)


def es_adjoint(x, order, levels, s):
    x = _prep(x)
    h = daubechies_lowpass(order)
    return weight_map(x.shape, levels, s, 1.0) * dwt(x, h, levels)


def es_apply(c, order, levels, s):
    c = _prep(c)
    h = daubechies_lowpass(order)
    return idwt(weight_map(c.shape, levels, s, 1.0) * c, h, levels)


def matern_cov_apply(x, order, levels, s):
    x = _prep(x)
    h = daubechies_lowpass(order)
    return idwt(weight_map(x.shape, levels, s, 2.0) * dwt(x, h, levels), h, levels)


def matern_sample(xi, order, levels, s):
    xi = _prep(xi)
    h = daubechies_lowpass(order)
    return idwt(weight_map(xi.shape, levels, s, 1.0) * dwt(xi, h, levels), h, levels)


def hs_norm_sq(x, order, levels, s):
    """||x||_{H^s}^2 = ||Gamma x||^2 with Gamma = (E_s^*)^{-1/2} (Sec. 3), i.e. ||D_s^{-1} W x||^2."""
    x = _prep(x)
    h = daubechies_lowpass(order)
    c = dwt(x, h, levels) / weight_map(x.shape, levels, s, 1.0)
    return float(np.sum(c * c))
