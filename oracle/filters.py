"""Daubechies extremal-phase filters, derived in high precision (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper (Sec. 4, the MRA paragraph and Def. 4.1) asks for a compactly
supported orthonormal scaling function of regularity r; it does not fix a
family.  The wavelet used throughout is Daubechies' extremal-phase family dbN
(N vanishing moments, L = 2N taps), obtained by spectral factorisation:

  |m0(w)|^2 = cos^{2N}(w/2) * P(sin^2(w/2)),
  P(y) = sum_{k<N} binom(N-1+k, k) y^k.

Each root y_k of P gives a reciprocal pair of zeros z, 1/z of the squared
magnitude response through y = (2 - z - 1/z)/4; the minimum-phase factor keeps
the zero with |z| < 1.  Then

  H(z) = c (1 + z^{-1})^N  prod_k (1 - z_k z^{-1}),   h[t] = coeff of z^{-t},

normalised so that sum_t h[t] = sqrt(2).  The high-pass (quadrature mirror)
filter is g[t] = (-1)^t h[L-1-t].

Everything is done in mpmath at 60 significant digits and rounded once to
float64 at the end.
"""

import threading
from functools import lru_cache

import mpmath as mp
import numpy as np

MAX_ORDER = 8  # db1 .. db8, L = 2 .. 16 taps


def _convolve(p, q):
    out = [mp.mpc(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


# mpmath's working precision is process-wide state: a derivation running in one thread while
# another enters or leaves its own precision block would run at the wrong precision.  Callers
# that map the oracle over a pool of threads therefore derive each filter under this lock.
_MP_LOCK = threading.Lock()


def _lowpass_mp(order):
    with _MP_LOCK:
        return _lowpass_mp_cached(order)


@lru_cache(maxsize=None)
def _lowpass_mp_cached(order):
    if not (1 <= order <= MAX_ORDER):
        raise ValueError(f"order must be in 1..{MAX_ORDER}, got {order}")
    with mp.workdps(60):
        n = order
        # P(y) coefficients, highest degree first for polyroots.
        p_coeffs = [mp.binomial(n - 1 + k, k) for k in range(n)][::-1]
        ys = [] if n == 1 else mp.polyroots(p_coeffs, maxsteps=500, extraprec=400)
        zs = []
        for y in ys:
            b = 2 - 4 * mp.mpc(y)
            disc = mp.sqrt(b * b - 4)
            z1, z2 = (b + disc) / 2, (b - disc) / 2
            zs.append(z1 if abs(z1) < 1 else z2)
        poly = [mp.mpc(1)]
        for _ in range(n):
            poly = _convolve(poly, [mp.mpc(1), mp.mpc(1)])
        for z in zs:
            poly = _convolve(poly, [mp.mpc(1), -z])
        h = [mp.re(c) for c in poly]
        scale = mp.sqrt(2) / mp.fsum(h)
        return tuple(c * scale for c in h)


def daubechies_lowpass(order):
    """Scaling (low-pass) filter of dbN as float64, length 2*order."""
    return np.array([float(c) for c in _lowpass_mp(order)], dtype=np.float64)


def daubechies_lowpass_mp(order):
    """Same filter as mpmath numbers (60 digits), for the invariant tests."""
    return list(_lowpass_mp(order))


def quadrature_highpass(h):
    """g[t] = (-1)^t h[L-1-t] (orthonormal quadrature-mirror wavelet filter)."""
    h = np.asarray(h, dtype=np.float64)
    L = h.size
    return np.array([(-1.0) ** t * h[L - 1 - t] for t in range(L)], dtype=np.float64)
