"""Pins of the oracle's Daubechies filters against facts independent of the oracle.

Orthonormality of even shifts, sum sqrt(2), N vanishing moments of the
wavelet filter and minimum phase together determine dbN uniquely; the Haar and
db2 closed forms (Daubechies 1988) are checked exactly.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import daubechies_lowpass, quadrature_highpass
from oracle.filters import daubechies_lowpass_mp

ORDERS = list(range(1, 9))


def test_haar():
    assert np.allclose(daubechies_lowpass(1), [2 ** -0.5, 2 ** -0.5], rtol=0, atol=1e-16)


def test_db2_closed_form():
    r3 = np.sqrt(3.0)
    expect = np.array([1 + r3, 3 + r3, 3 - r3, 1 - r3]) / (4 * np.sqrt(2.0))
    assert np.max(np.abs(daubechies_lowpass(2) - expect)) < 1e-15


@pytest.mark.parametrize("order", ORDERS)
def test_invariants_high_precision(order):
    """Checked in 60-digit arithmetic on the unrounded filter."""
    with mp.workdps(60):
        h = daubechies_lowpass_mp(order)
        L = len(h)
        assert L == 2 * order
        assert abs(mp.fsum(h) - mp.sqrt(2)) < mp.mpf(10) ** -45
        for l in range(order):
            dot = mp.fsum(h[t] * h[t + 2 * l] for t in range(L - 2 * l))
            assert abs(dot - (1 if l == 0 else 0)) < mp.mpf(10) ** -45
        for p in range(order):
            mom = mp.fsum(((-1) ** t) * mp.mpf(t) ** p * h[t] for t in range(L))
            assert abs(mom) < mp.mpf(10) ** -40


def _nontrivial_zero_moduli(h):
    """Moduli of the zeros of H(z) = sum h[t] z^{-t} after dividing out (1 + z^{-1})^N.

    The division is exact synthetic division in 60-digit arithmetic; its
    remainder must vanish, which also checks the N-fold zero at z = -1.
    """
    order = len(h) // 2
    with mp.workdps(60):
        q = [mp.mpf(c) for c in h]  # coefficients of z^{-t}, i.e. of w^{L-1-t} with w = z
        for _ in range(order):
            out = [q[0]]
            for c in q[1:-1]:
                out.append(c - out[-1])
            assert abs(q[-1] - out[-1]) < mp.mpf(10) ** -40  # remainder of division by (w + 1)
            q = out
        if len(q) == 1:
            return np.zeros(0)
        roots = mp.polyroots(q, maxsteps=500, extraprec=400)
        return np.array([float(abs(r)) for r in roots])


@pytest.mark.parametrize("order", ORDERS[1:])
def test_minimum_phase(order):
    h = daubechies_lowpass_mp(order)
    mods = _nontrivial_zero_moduli(h)
    assert mods.size == order - 1
    assert np.all(mods < 1.0)
    # the time-reversed (maximum-phase) filter satisfies every other invariant
    # and must fail this one
    assert np.all(_nontrivial_zero_moduli(h[::-1]) > 1.0)


@pytest.mark.parametrize("order", ORDERS)
def test_float64_invariants(order):
    h = daubechies_lowpass(order)
    g = quadrature_highpass(h)
    L = h.size
    assert abs(h.sum() - np.sqrt(2)) < 4e-16
    assert abs(g.sum()) < 1e-15
    for l in range(-order + 1, order):
        hh = sum(h[t] * h[t + 2 * l] for t in range(L) if 0 <= t + 2 * l < L)
        gg = sum(g[t] * g[t + 2 * l] for t in range(L) if 0 <= t + 2 * l < L)
        hg = sum(h[t] * g[t + 2 * l] for t in range(L) if 0 <= t + 2 * l < L)
        assert abs(hh - (l == 0)) < 2e-15
        assert abs(gg - (l == 0)) < 2e-15
        assert abs(hg) < 2e-15


def test_known_db3_values():
    # Daubechies (1992), Ten Lectures on Wavelets, Table 6.1, N = 3 (rounded to 12 digits there).
    ref = [0.332670552950, 0.806891509311, 0.459877502118, -0.135011020010, -0.085441273882, 0.035226291882]
    assert np.max(np.abs(daubechies_lowpass(3) - np.array(ref))) < 1e-11


def test_order_range():
    with pytest.raises(ValueError):
        daubechies_lowpass(0)
    with pytest.raises(ValueError):
        daubechies_lowpass(9)
