"""Pins of the FP64 Fourier-multiplier oracle (the FFT form of E_s^*, Sec. 4, Implementation) against closed forms,
brute-force DFT sums and the operator's invariants, and a comparison of its spectrum with the
wavelet form's (norm equivalence, Sec. 4)."""
import itertools

import numpy as np
import pytest

from oracle import matern_cov_apply
from oracle.fourier import fft_cov_apply


def _alias(k, n):
    """|signed frequency| of integer wave number k on an n-point periodic axis."""
    r = k % n
    return min(r, n - r)


def _potential(kvec, shape, s, period):
    q = sum((_alias(k, n) / period) ** 2 for k, n in zip(kvec, shape))
    return (1.0 + 4.0 * np.pi ** 2 * q) ** (-s)


@pytest.mark.parametrize("shape,kvec", [((16,), (3,)), ((16,), (8,)), ((16,), (13,)), ((15,), (7,)),
                                        ((12, 10), (5, 9)), ((8, 6, 10), (4, 3, 7)), ((9, 7), (0, 6))])
@pytest.mark.parametrize("s,period", [(1.5, 1.0), (-0.75, 1.0), (0.6, 3.5)])
def test_plane_waves_are_eigenfunctions(shape, kvec, s, period):
    """A sampled plane wave cos(2 pi k.x + phi) is mapped to B(k) times itself, with B the Bessel
    potential at the wave's aliased frequency (wave numbers past n/2 are negative frequencies)."""
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    phase = sum(2 * np.pi * k * g / n for k, g, n in zip(kvec, grids, shape)) + 0.3
    x = np.cos(phase)
    y = fft_cov_apply(x, len(shape), s, period)
    assert np.max(np.abs(y - _potential(kvec, shape, s, period) * x)) < 1e-12


@pytest.mark.parametrize("shape", [(5,), (6,), (4, 6), (3, 4, 2)])
def test_bruteforce_dft_sum(shape):
    """y_j = (1/N) sum_k B(k) sum_j' x_j' exp(2 pi i k.(j - j')/n), summed point by point."""
    s, period = 1.25, 2.0
    x = np.random.default_rng(3).standard_normal(shape)
    N = x.size
    pts = list(itertools.product(*[range(n) for n in shape]))
    y = np.zeros(shape)
    for j in pts:
        acc = 0.0
        for k in pts:
            b = _potential(k, shape, s, period)
            for jp in pts:
                acc += b * x[jp] * np.cos(2 * np.pi * sum(kk * (a - c) / n for kk, a, c, n in zip(k, j, jp, shape)))
        y[j] = acc / N
    assert np.max(np.abs(fft_cov_apply(x, len(shape), s, period) - y)) < 1e-12


def test_invariants():
    """s = 0 is the identity; exponents add under composition; the operator is symmetric, positive
    for s > 0, commutes with circular shifts (which the wavelet form does not), keeps constants and
    acts on the last ndim axes only (batch axes are independent)."""
    rng = np.random.default_rng(7)
    x, z = rng.standard_normal((2, 24, 20)), rng.standard_normal((2, 24, 20))
    assert np.max(np.abs(fft_cov_apply(x, 2, 0.0) - x)) < 1e-13
    a = fft_cov_apply(fft_cov_apply(x, 2, 0.7), 2, 0.4)
    assert np.max(np.abs(a - fft_cov_apply(x, 2, 1.1))) < 1e-13
    assert abs(np.sum(fft_cov_apply(x, 2, 0.9) * z) - np.sum(x * fft_cov_apply(z, 2, 0.9))) < 1e-12
    assert np.sum(x * fft_cov_apply(x, 2, 0.9)) > 0
    shifted = np.roll(x, (3, -5), axis=(1, 2))
    assert np.max(np.abs(fft_cov_apply(shifted, 2, 1.3) - np.roll(fft_cov_apply(x, 2, 1.3), (3, -5), axis=(1, 2)))) < 1e-13
    c = np.full((24, 20), 2.5)
    assert np.max(np.abs(fft_cov_apply(c, 2, 1.3) - c)) < 1e-13
    assert np.max(np.abs(fft_cov_apply(x, 2, 1.3)[1] - fft_cov_apply(x[1], 2, 1.3))) < 1e-14
    assert not np.allclose(matern_cov_apply(np.roll(x[0], 1, axis=0), 4, 2, 1.0),
                           np.roll(matern_cov_apply(x[0], 4, 2, 1.0), 1, axis=0))


@pytest.mark.parametrize("s", [0.5, 1.0, 1.5])
def test_wavelet_and_fourier_spectra_agree_up_to_a_constant(s):
    """On the detail scales the Rayleigh quotient of the wavelet covariance W^T D_2s W on a Fourier
    mode follows the Bessel potential up to one constant (the norm equivalence of the wavelet weights
    with the Sobolev norm, Sec. 4): from the coarsest detail octave to n/4 the ratio varies by less
    than the factor 2^s that B itself falls over half an octave, and it is the same at the two ends of
    that range (a weight shifted by one level would tilt it by 2^(2s) per octave).  Below the coarsest
    scale the wavelet form is flat (approximation weight 1)."""
    n, m, order = 512, 7, 8
    j = np.arange(n)
    ks = [n >> m, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128]
    ratio = []
    for k in ks:
        c, sn = np.cos(2 * np.pi * k * j / n), np.sin(2 * np.pi * k * j / n)
        rw = (c @ matern_cov_apply(c, order, m, s) + sn @ matern_cov_apply(sn, order, m, s)) / (c @ c + sn @ sn)
        ratio.append(rw / _potential((k,), (n,), s, 1.0))
    ratio = np.array(ratio)
    assert np.max(ratio) / np.min(ratio) < 2.0 ** s
    assert abs(np.log(ratio[0] / ratio[-1])) < 0.05
    flat = [(np.cos(2 * np.pi * k * j / n) @ matern_cov_apply(np.cos(2 * np.pi * k * j / n), order, m, s)) / (n / 2)
            for k in (1, 2)]
    assert min(flat) > 0.99
