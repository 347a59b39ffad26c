"""FP64 oracle of the Fourier realisation of E_s^* (Sec. 4, Implementation: the FFT formula).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper characterises E_s^* in the Fourier domain as multiplication by the Bessel potential
(1 + 4 pi^2 |xi|^2)^(-s) (proof of Prop. 3.2, and Sec. 4 (Implementation) where the discrete operator is written as
an inverse FFT of B times the FFT of X).  Reading taken here: the grid samples a periodic box of
side `period` (the same on every axis) at n_k points per axis, the discrete Fourier basis of axis
k has the integer frequencies k_k = -n_k/2 .. n_k/2 - 1 (numpy's fftfreq order), so the sampled
potential is B[k] = (1 + 4 pi^2 sum_k (k_k / period)^2)^(-s).  |k_k| is the same for the two
aliases of the Nyquist frequency, so B is real and even and the operator is real, symmetric and
diagonal in the Fourier basis.  Unlike the wavelet form this operator commutes with every
circular shift of the grid.

Everything is float64 numpy; batch dims lead, the grid is the last `ndim` axes.
"""
import numpy as np


def fourier_multiplier(shape, s, period=1.0):
    """B on the unshifted FFT grid of `shape` (float64, the shape of the grid)."""
    q = np.zeros(tuple(shape), dtype=np.float64)
    for ax, n in enumerate(shape):
        k = np.fft.fftfreq(n, d=1.0 / n) / period          # integer frequencies / side length
        view = [1] * len(shape)
        view[ax] = n
        q = q + (k ** 2).reshape(view)
    return (1.0 + 4.0 * np.pi ** 2 * q) ** (-float(s))


def fft_cov_apply(x, ndim, s, period=1.0):
    """y = ifft(B * fft(x)) over the last `ndim` axes, in float64 (real part; the imaginary part is
    rounding only, because B is real and even)."""
    x = np.asarray(x, dtype=np.float64)
    axes = tuple(range(x.ndim - ndim, x.ndim))
    b = fourier_multiplier(x.shape[x.ndim - ndim:], s, period)
    return np.real(np.fft.ifftn(b * np.fft.fftn(x, axes=axes), axes=axes))
