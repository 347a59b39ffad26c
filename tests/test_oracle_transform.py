"""Pins of the oracle's periodic DWT: orthogonality, dense brute force, vanishing moments."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import daubechies_lowpass, dwt, idwt
from oracle.dense import dwt_matrix


def _rand(shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


CASES = [((64,), 4), ((32, 16), 3), ((8, 8, 16), 2), ((8, 8), 3), ((4, 8, 8), 2), ((2,), 1), ((16, 2), 1)]


@pytest.mark.parametrize("shape,levels", CASES)
@pytest.mark.parametrize("order", [1, 2, 4, 8])
def test_perfect_reconstruction_and_parseval(shape, levels, order):
    """W^T W = I and ||W x|| = ||x||, also when sides are shorter than the filter (folding)."""
    h = daubechies_lowpass(order)
    x = _rand(shape)
    c = dwt(x, h, levels)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) < 1e-13 * np.linalg.norm(x)
    assert np.max(np.abs(idwt(c, h, levels) - x)) < 1e-13 * np.max(np.abs(x))


@pytest.mark.parametrize("order", [1, 2, 4, 6, 8])
@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_dense_kronecker_bruteforce_2d(order, levels):
    """Gather-based transform vs the explicit Kronecker-matrix product on 16x16."""
    shape = (16, 16)
    h = daubechies_lowpass(order)
    W = dwt_matrix(shape, h, levels)
    assert np.max(np.abs(W @ W.T - np.eye(W.shape[0]))) < 1e-13
    for seed in range(3):
        x = _rand(shape, seed)
        assert np.max(np.abs(dwt(x, h, levels).ravel() - W @ x.ravel())) < 1e-13
        assert np.max(np.abs(idwt(x, h, levels).ravel() - W.T @ x.ravel())) < 1e-13


@pytest.mark.parametrize("order", [1, 2, 4, 6, 8])
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_dense_kronecker_bruteforce_3d(order, levels):
    shape = (8, 8, 8)
    h = daubechies_lowpass(order)
    W = dwt_matrix(shape, h, levels)
    x = _rand(shape, 7)
    assert np.max(np.abs(dwt(x, h, levels).ravel() - W @ x.ravel())) < 1e-13
    assert np.max(np.abs(idwt(x, h, levels).ravel() - W.T @ x.ravel())) < 1e-13


def test_dense_bruteforce_1d_nonsquare():
    for shape, levels in [((32,), 4), ((16, 32), 3), ((8, 16, 4), 2)]:
        h = daubechies_lowpass(3)
        W = dwt_matrix(shape, h, levels)
        x = _rand(shape, 3)
        assert np.max(np.abs(dwt(x, h, levels).ravel() - W @ x.ravel())) < 1e-13


def test_one_level_haar_by_hand():
    """a[k] = (x[2k] + x[2k+1]) / sqrt2, d[k] = (x[2k] - x[2k+1]) / sqrt2 (offset-0 correlation)."""
    x = np.array([1.0, 2.0, 3.0, 4.0, -1.0, 5.0])
    c = dwt(x, daubechies_lowpass(1), 1)
    r = 2 ** -0.5
    expect = [3 * r, 7 * r, 4 * r, -1 * r, -1 * r, -6 * r]
    assert np.max(np.abs(c - expect)) < 1e-15


def test_one_level_db2_offset_by_hand():
    """db2, n = 4: a[1] = h0 x2 + h1 x3 + h2 x0 + h3 x1 (periodic wrap, offset 0)."""
    h = daubechies_lowpass(2)
    g = oracle.quadrature_highpass(h)
    x = np.array([0.3, -1.2, 2.5, 0.7])
    c = dwt(x, h, 1)
    assert abs(c[0] - (h[0] * x[0] + h[1] * x[1] + h[2] * x[2] + h[3] * x[3])) < 1e-15
    assert abs(c[1] - (h[0] * x[2] + h[1] * x[3] + h[2] * x[0] + h[3] * x[1])) < 1e-15
    assert abs(c[3] - (g[0] * x[2] + g[1] * x[3] + g[2] * x[0] + g[3] * x[1])) < 1e-15


def _cone_ok(k, level, L, n):
    """Detail coefficient k of `level` depends on samples [2^i k, 2^i k + (2^i - 1)(L - 1)]; True if no wrap."""
    return (k << level) + ((1 << level) - 1) * (L - 1) < n


@pytest.mark.parametrize("order", [2, 3, 4, 6, 8])
def test_vanishing_moments_1d(order):
    n, levels = 256, 3
    h = daubechies_lowpass(order)
    L = h.size
    t = np.arange(n, dtype=np.float64) / n
    coef = np.random.default_rng(order).standard_normal(order)
    x = sum(coef[p] * t ** p for p in range(order))  # degree order-1 < N
    c = dwt(x, h, levels)
    checked = 0
    for lev in range(1, levels + 1):
        half = n >> lev
        for k in range(half):
            if _cone_ok(k, lev, L, n):
                assert abs(c[half + k]) < 1e-10 * np.linalg.norm(x)
                checked += 1
    assert checked > n // 4


@pytest.mark.parametrize("order", [2, 4, 6])
def test_vanishing_moments_2d(order):
    """Polynomials of total degree < N: every detail coefficient whose cone does not wrap on its high-pass axes is 0."""
    n0, n1, levels = 64, 128, 3
    h = daubechies_lowpass(order)
    L = h.size
    i = np.arange(n0)[:, None] / n0
    j = np.arange(n1)[None, :] / n1
    gen = np.random.default_rng(11)
    x = sum(gen.standard_normal() * i ** p * j ** q for p in range(order) for q in range(order) if p + q < order)
    c = dwt(x, h, levels)
    tol = 1e-10 * np.linalg.norm(x)
    checked = 0
    for lev in range(1, levels + 1):
        h0, h1 = n0 >> lev, n1 >> lev
        for e0, e1 in [(0, 1), (1, 0), (1, 1)]:
            band = c[e0 * h0:(e0 + 1) * h0, e1 * h1:(e1 + 1) * h1]
            for k0, k1 in itertools.product(range(h0), range(h1)):
                if (not e0 or _cone_ok(k0, lev, L, n0)) and (not e1 or _cone_ok(k1, lev, L, n1)):
                    assert abs(band[k0, k1]) < tol
                    checked += 1
    assert checked > 1000


def test_rejects_bad_shapes():
    h = daubechies_lowpass(2)
    with pytest.raises(ValueError):
        dwt(np.zeros((12, 16)), h, 3)
    with pytest.raises(ValueError):
        dwt(np.zeros(8), h, -1)
