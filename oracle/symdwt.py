"""Non-periodic (half-point symmetric) multi-level DWT and the operator W^{-1} D W (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4 (the discrete wavelet transform paragraph) evaluates W and W^{-1} with
MATLAB's fast wavelet transform, whose band lengths l(i) depend on the depth and
are kept in a book-keeping matrix.  That transform's default boundary handling
is half-point symmetric extension: the signal is mirrored about its end points,
the first and last samples repeated,

    xs[j] = x[j] (0 <= j < n),  xs[-1-j] = x[j],  xs[n+j] = x[n-1-j],

which is periodic with period 2n.  One analysis step of a length-n signal with
a filter of L taps keeps

    l = floor((n + L - 1) / 2)

coefficients per band,

    a[k] = sum_t h[t] xs[2k + t - (L - 2)],   d[k] = sum_t g[t] xs[2k + t - (L - 2)],

(the odd-indexed samples of the full filtered extension).  The step is
redundant (2 l >= n) and not orthogonal; its left inverse, the synthesis of
length n, adds the upsampled bands filtered by h and g and keeps the central n
samples:

    x[i] = sum_k h[i + L - 2 - 2k] a[k] + g[i + L - 2 - 2k] d[k],   0 <= k < l.

Every position 0 <= i < n reads only coefficients 0 <= k < l, and these equal
the coefficients of the infinite symmetric extension, so the synthesis
reconstructs x exactly (W^{-1} W = I) although W^{-1} is not W^T.

A d-dimensional level applies the step along every axis of the current
approximation block (2^d - 1 detail bands per level, as in the periodic
transform).  Bands are returned as arrays, not packed: level i's bands have
side l_i on every axis where the level's approximation has side l_i.

The operator of Sec. 4, E_s^* X = W^{-1}(D (W X)), multiplies detail level i by
2^{-tau s (m-i)} (tau = 2 for the covariance) and the approximation by 1, the
same level-weight reading as for the periodic transform.
"""

import numpy as np

from .dwt import level_weights
from .filters import daubechies_lowpass, quadrature_highpass


def sym_length(n, taps):
    """Band length of one analysis step of a length-n axis with a `taps`-tap filter."""
    return (int(n) + int(taps) - 1) // 2


def sym_lengths(n, taps, levels):
    """Approximation lengths l_1 .. l_levels of one axis (the book-keeping entries)."""
    out, cur = [], int(n)
    for _ in range(levels):
        cur = sym_length(cur, taps)
        out.append(cur)
    return out


def sym_index(j, n):
    """Index into x of position j of the half-point symmetric extension (period 2n)."""
    j = np.mod(j, 2 * n)
    return np.where(j >= n, 2 * n - 1 - j, j)


def sym_analysis_axis(x, h, axis):
    """One analysis step along `axis`: returns (a, d), each of length sym_length(n, L) there."""
    x = np.asarray(x, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    g = quadrature_highpass(h)
    L = h.size
    xm = np.moveaxis(x, axis, 0)
    n = xm.shape[0]
    k = np.arange(sym_length(n, L))
    a = np.zeros((k.size,) + xm.shape[1:])
    d = np.zeros_like(a)
    for t in range(L):
        gathered = xm[sym_index(2 * k + t - (L - 2), n)]
        a += h[t] * gathered
        d += g[t] * gathered
    return np.moveaxis(a, 0, axis), np.moveaxis(d, 0, axis)


def sym_synthesis_axis(a, d, h, axis, n):
    """Left inverse of `sym_analysis_axis` along `axis`, output length n there."""
    a = np.asarray(a, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    g = quadrature_highpass(h)
    L = h.size
    am = np.moveaxis(a, axis, 0)
    dm = np.moveaxis(d, axis, 0)
    l = am.shape[0]
    x = np.zeros((n,) + am.shape[1:])
    i = np.arange(n)
    for k in range(l):
        t = i + L - 2 - 2 * k
        ok = (t >= 0) & (t < L)
        tt = np.where(ok, t, 0)
        hk = np.where(ok, h[tt], 0.0)
        gk = np.where(ok, g[tt], 0.0)
        shape = (n,) + (1,) * (am.ndim - 1)
        x += hk.reshape(shape) * am[k] + gk.reshape(shape) * dm[k]
    return np.moveaxis(x, 0, axis)


def _bands(x, h):
    """One d-dimensional level: the 2^d bands keyed by their high-pass pattern (tuple of 0/1)."""
    bands = {(): np.asarray(x, dtype=np.float64)}
    for ax in range(np.ndim(x)):
        nxt = {}
        for key, arr in bands.items():
            a, d = sym_analysis_axis(arr, h, ax)
            nxt[key + (0,)] = a
            nxt[key + (1,)] = d
        bands = nxt
    return bands


def _unbands(bands, h, shape):
    """Inverse of `_bands` onto a block of `shape`: axes in reverse order."""
    ndim = len(shape)
    cur = dict(bands)
    for ax in range(ndim - 1, -1, -1):
        nxt = {}
        for key in {k[:ax] for k in cur}:
            nxt[key] = sym_synthesis_axis(cur[key + (0,)], cur[key + (1,)], h, ax, shape[ax])
        cur = nxt
    return cur[()]


def sym_dwt(x, h, levels):
    """Depth-`levels` symmetric-extension DWT: (approximation, [details of level 1 .. levels]).

    details[i-1] maps every high-pass pattern eps != 0 of level i to its band.
    """
    cur = np.asarray(x, dtype=np.float64)
    details = []
    for _ in range(levels):
        b = _bands(cur, h)
        low = (0,) * cur.ndim
        details.append({k: v for k, v in b.items() if k != low})
        cur = b[low]
    return cur, details


def sym_idwt(approx, details, h, shape):
    """Left inverse of `sym_dwt` onto an array of `shape` (the transform's W^{-1})."""
    levels = len(details)
    ndim = len(shape)
    shapes = [tuple(int(s) for s in shape)]
    for _ in range(levels):
        shapes.append(tuple(sym_length(s, np.size(h)) for s in shapes[-1]))
    cur = np.asarray(approx, dtype=np.float64)
    low = (0,) * ndim
    for lev in range(levels, 0, -1):
        bands = dict(details[lev - 1])
        bands[low] = cur
        cur = _unbands(bands, h, shapes[lev - 1])
    return cur


def sym_cov_apply(x, order, levels, s, tau=2.0):
    """E_s^* X = W^{-1}(D (W X)) with the symmetric-extension transform (Sec. 4).

    Detail level i is weighted 2^{-tau s (levels - i)}, the approximation 1.
    """
    x = np.asarray(x, dtype=np.float64)
    h = daubechies_lowpass(order)
    approx, details = sym_dwt(x, h, levels)
    w = level_weights(levels, s, tau)
    scaled = [{k: w[i] * v for k, v in lev.items()} for i, lev in enumerate(details)]
    return sym_idwt(approx, scaled, h, x.shape)


# ---- transpose of the operator (the backward of a loss through sym_cov_apply) -------------------
#
# (W^{-1} D W)^T = W^T D W^{-T}.  The adjoint of each 1-D step is written out from its definition:
# the analysis gathers x_ext[2k + t - (L - 2)], so its adjoint scatter-adds h[t] a[k] + g[t] d[k]
# into x[sym_index(2k + t - (L - 2))]; the synthesis reads a[k] with tap h[i + L - 2 - 2k], so its
# adjoint is a[k] = sum_i h[i + L - 2 - 2k] x[i] over 0 <= i < n, i.e. the analysis sum with the
# signal extended by zeros instead of by reflection.

def sym_analysis_axis_adjoint(a, d, h, axis, n):
    """Adjoint of `sym_analysis_axis` along `axis` (output length n there)."""
    a = np.asarray(a, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    g = quadrature_highpass(h)
    L = h.size
    am = np.moveaxis(a, axis, 0)
    dm = np.moveaxis(d, axis, 0)
    k = np.arange(am.shape[0])
    x = np.zeros((n,) + am.shape[1:])
    for t in range(L):
        np.add.at(x, sym_index(2 * k + t - (L - 2), n), h[t] * am + g[t] * dm)
    return np.moveaxis(x, 0, axis)


def sym_synthesis_axis_adjoint(x, h, axis, l):
    """Adjoint of `sym_synthesis_axis` along `axis`: the two bands, each of length l there."""
    x = np.asarray(x, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    g = quadrature_highpass(h)
    L = h.size
    xm = np.moveaxis(x, axis, 0)
    n = xm.shape[0]
    a = np.zeros((l,) + xm.shape[1:])
    d = np.zeros_like(a)
    for k in range(l):
        for t in range(L):
            i = 2 * k + t - (L - 2)
            if 0 <= i < n:
                a[k] += h[t] * xm[i]
                d[k] += g[t] * xm[i]
    return np.moveaxis(a, 0, axis), np.moveaxis(d, 0, axis)


def _unbands_adjoint(y, h, shapes_band):
    """Adjoint of `_unbands`: y (a block) -> the 2^d bands, keyed by high-pass pattern."""
    ndim = np.ndim(y)
    cur = {(): np.asarray(y, dtype=np.float64)}
    for ax in range(ndim):  # _unbands runs the axes in reverse order: its adjoint forward
        nxt = {}
        for key, arr in cur.items():
            a, d = sym_synthesis_axis_adjoint(arr, h, ax, shapes_band[ax])
            nxt[key + (0,)] = a
            nxt[key + (1,)] = d
        cur = nxt
    return cur


def _bands_adjoint(bands, h, shape):
    """Adjoint of `_bands`: the 2^d bands -> a block of `shape`."""
    ndim = len(shape)
    cur = dict(bands)
    for ax in range(ndim - 1, -1, -1):
        nxt = {}
        for key in {k[:ax] for k in cur}:
            nxt[key] = sym_analysis_axis_adjoint(cur[key + (0,)], cur[key + (1,)], h, ax, shape[ax])
        cur = nxt
    return cur[()]


def sym_cov_apply_transpose(y, order, levels, s, tau=2.0):
    """(W^{-1} D W)^T y = W^T D W^{-T} y for the symmetric-extension transform of Sec. 4."""
    y = np.asarray(y, dtype=np.float64)
    h = daubechies_lowpass(order)
    L = h.size
    shapes = [tuple(int(v) for v in y.shape)]
    for _ in range(levels):
        shapes.append(tuple(sym_length(v, L) for v in shapes[-1]))
    w = level_weights(levels, s, tau)
    low = (0,) * y.ndim
    # W^{-T}: the synthesis ran levels m..1 on the way up; its adjoint runs levels 1..m down
    cur = y
    details = []
    for lev in range(1, levels + 1):
        bands = _unbands_adjoint(cur, h, shapes[lev])
        details.append({k: w[lev - 1] * v for k, v in bands.items() if k != low})
        cur = bands[low]
    # W^T: the analysis ran levels 1..m; its adjoint runs m..1 back up
    for lev in range(levels, 0, -1):
        bands = dict(details[lev - 1])
        bands[low] = cur
        cur = _bands_adjoint(bands, h, shapes[lev - 1])
    return cur
