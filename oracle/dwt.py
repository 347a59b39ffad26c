"""Periodic orthonormal multi-level DWT and the level weights (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4 (the discrete wavelet transform paragraph) defines W as a depth-m
decomposition X -> [cA_m, cH_m, cV_m, cD_m, ..., cD_1] computed by repeated
low/high-pass filtering.  Boundary handling is not stated in the paper; the
periodic extension is used so that W is orthogonal and W^{-1} = W^T.

One-dimensional step on an axis of even length n (correlation, offset 0):

    a[k] = sum_t h[t] x[(2k+t) mod n],   d[k] = sum_t g[t] x[(2k+t) mod n],

for k < n/2, stored as [a | d] along that axis.  The modular index makes the
step valid for any even n, also when n is shorter than the filter.

A d-dimensional level applies the 1-D step along every axis of the current
all-low block (Mallat's isotropic pyramid: 2^d - 1 detail bands per level,
Sec. 4, the multi-d wavelet indexing and Def. 4.1).  The result is kept in
place in an array of the input's shape ("packed pyramid"): after m levels the
approximation occupies [0, n_k/2^m) on every axis and the band of level i
with high-pass pattern eps in {0,1}^d \\ {0} occupies
[eps_k n_k/2^i, (eps_k + 1) n_k/2^i) on axis k.
"""

import numpy as np

from .filters import quadrature_highpass


def analysis_axis(x, h, axis):
    """One periodic analysis step along `axis`: returns [a | d] on that axis."""
    x = np.asarray(x, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    g = quadrature_highpass(h)
    n = x.shape[axis]
    if n % 2:
        raise ValueError("axis length must be even")
    xm = np.moveaxis(x, axis, 0)
    k = np.arange(n // 2)
    a = np.zeros((n // 2,) + xm.shape[1:])
    d = np.zeros_like(a)
    for t in range(h.size):
        gathered = xm[(2 * k + t) % n]
        a += h[t] * gathered
        d += g[t] * gathered
    return np.moveaxis(np.concatenate([a, d], axis=0), 0, axis)


def synthesis_axis(c, h, axis):
    """Transpose of `analysis_axis`: scatter-add h[t] a[k] + g[t] d[k] into (2k+t) mod n."""
    c = np.asarray(c, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    g = quadrature_highpass(h)
    n = c.shape[axis]
    if n % 2:
        raise ValueError("axis length must be even")
    cm = np.moveaxis(c, axis, 0)
    half = n // 2
    a, d = cm[:half], cm[half:]
    k = np.arange(half)
    x = np.zeros_like(cm)
    for t in range(h.size):
        # (2k + t) mod n is injective in k for fixed t, so a plain fancy-index
        # accumulation is exact (no repeated targets inside one statement).
        x[(2 * k + t) % n] += h[t] * a + g[t] * d
    return np.moveaxis(x, 0, axis)


def _check_levels(shape, levels):
    if levels < 0:
        raise ValueError("levels must be >= 0")
    for n in shape:
        if n % (1 << levels):
            raise ValueError(f"every side must be divisible by 2^levels (side {n}, levels {levels})")


def dwt(x, h, levels):
    """Depth-`levels` periodic DWT of a 1-, 2- or 3-D array, packed pyramid layout."""
    c = np.array(x, dtype=np.float64, copy=True)
    _check_levels(c.shape, levels)
    block = list(c.shape)
    for _ in range(levels):
        sl = tuple(slice(0, b) for b in block)
        blk = c[sl]
        for ax in range(c.ndim):
            blk = analysis_axis(blk, h, ax)
        c[sl] = blk
        block = [b // 2 for b in block]
    return c


def idwt(c, h, levels):
    """Inverse of `dwt` (= its transpose, the transform being orthogonal)."""
    x = np.array(c, dtype=np.float64, copy=True)
    _check_levels(x.shape, levels)
    for lev in range(levels, 0, -1):
        sl = tuple(slice(0, n >> (lev - 1)) for n in x.shape)
        blk = x[sl]
        for ax in range(x.ndim - 1, -1, -1):
            blk = synthesis_axis(blk, h, ax)
        x[sl] = blk
    return x


def level_weights(levels, s, tau):
    """Weights of the detail bands, index i-1 for level i = 1 (finest) .. m (coarsest).

    Sec. 4 (the level-weight rule): level i is scaled by 2^{-2s(m-i)} for the
    covariance (tau = 2); tau = 1 gives the square root used for E_s^* in
    isometric coordinates and for prior samples.  The approximation band is
    weighted 1, the same as the coarsest detail level (Prop. 4.2: V_0 and W_0
    both carry weight 1).
    """
    m = int(levels)
    return np.array([2.0 ** (-(tau * s) * (m - i)) for i in range(1, m + 1)], dtype=np.float64)


def weight_map(shape, levels, s, tau):
    """Per-coefficient weight array in the packed-pyramid layout."""
    _check_levels(shape, levels)
    w = level_weights(levels, s, tau)
    out = np.ones(shape, dtype=np.float64)
    if levels == 0:
        return out
    out[...] = w[0]
    for lev in range(2, levels + 1):
        sl = tuple(slice(0, n >> (lev - 1)) for n in shape)
        out[sl] = w[lev - 1]
    sl = tuple(slice(0, n >> levels) for n in shape)
    out[sl] = 1.0
    return out
