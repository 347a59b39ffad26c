"""Pins of the symmetric-extension (non-periodic) transform and operator of the oracle.

The transform is pinned through routes that do not share its code: the periodic
oracle (itself pinned by dense brute force and closed forms) applied to the
mirrored signal and to zero-padded coefficients, the Haar closed form, perfect
reconstruction, and the periodic operator for Haar on dyadic sides.
"""
import numpy as np
import pytest

import oracle
from oracle import symdwt

ORDERS = list(range(1, 9))


def _rng(*key):
    return np.random.default_rng(abs(hash(key)) & 0xFFFFFFFF)


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 32, 47])
def test_analysis_matches_periodic_transform_of_mirrored_signal(order, n):
    """xs has period 2n and equals [x, reversed x] on one period, so one symmetric step is the
    periodic step of that length-2n signal, shifted by L/2 - 1 coefficients."""
    h = oracle.daubechies_lowpass(order)
    L = h.size
    x = _rng("mirror", order, n).standard_normal(n)
    a, d = symdwt.sym_analysis_axis(x, h, 0)
    z = np.concatenate([x, x[::-1]])
    per = oracle.analysis_axis(z, h, 0)
    ap, dp = per[:n], per[n:]
    k = np.arange(symdwt.sym_length(n, L))
    idx = np.mod(k - (L // 2 - 1), n)
    np.testing.assert_allclose(a, ap[idx], rtol=0, atol=1e-13)
    np.testing.assert_allclose(d, dp[idx], rtol=0, atol=1e-13)


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("n", [1, 4, 7, 20, 33])
def test_synthesis_matches_periodic_synthesis_of_padded_coefficients(order, n):
    """W^{-1} off its range: the periodic synthesis (the transpose of the periodic analysis) of
    the coefficients placed at the start of a long zero-padded period, read from position L - 2."""
    h = oracle.daubechies_lowpass(order)
    L = h.size
    l = symdwt.sym_length(n, L)
    r = _rng("pad", order, n)
    a, d = r.standard_normal(l), r.standard_normal(l)
    got = symdwt.sym_synthesis_axis(a, d, h, 0, n)
    P = l + L
    c = np.zeros(2 * P)
    c[:l] = a
    c[P:P + l] = d
    full = oracle.synthesis_axis(c, h, 0)
    np.testing.assert_allclose(got, full[L - 2:L - 2 + n], rtol=0, atol=1e-13)


def test_haar_hand_example():
    """Haar on [1, 2, 3]: pairs (1, 2) and (3, 3) (the last sample repeated by the mirror)."""
    h = oracle.daubechies_lowpass(1)
    a, d = symdwt.sym_analysis_axis(np.array([1.0, 2.0, 3.0]), h, 0)
    r = 1 / np.sqrt(2)
    np.testing.assert_allclose(a, [3 * r, 6 * r], atol=1e-15)
    np.testing.assert_allclose(d, [-r, 0.0], atol=1e-15)
    x = symdwt.sym_synthesis_axis(a, d, h, 0, 3)
    np.testing.assert_allclose(x, [1.0, 2.0, 3.0], atol=1e-15)


def test_band_lengths():
    """floor((n + L - 1) / 2) per step: 512 samples, db8 (16 taps), five levels."""
    assert symdwt.sym_lengths(512, 16, 5) == [263, 139, 77, 46, 30]
    assert symdwt.sym_lengths(7, 2, 3) == [4, 2, 1]
    assert symdwt.sym_lengths(1, 16, 2) == [8, 11]


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("shape,levels", [((1,), 2), ((5,), 3), ((100,), 7), ((13, 20), 4), ((6, 9), 3),
                                          ((5, 7, 9), 2), ((8, 8, 8), 3)])
def test_perfect_reconstruction(order, shape, levels):
    h = oracle.daubechies_lowpass(order)
    x = _rng("pr", order, shape, levels).standard_normal(shape)
    approx, details = symdwt.sym_dwt(x, h, levels)
    y = symdwt.sym_idwt(approx, details, h, shape)
    np.testing.assert_allclose(y, x, rtol=0, atol=1e-11 * (1 + np.abs(x).max()))


@pytest.mark.parametrize("order", [2, 4, 8])
def test_dense_left_inverse_not_transpose(order):
    """Dense matrices on a tiny grid: W^{-1} W = I, while W^T W != I (the step is redundant and
    not orthogonal), and the covariance W^{-1} D W is not symmetric."""
    h = oracle.daubechies_lowpass(order)
    n, levels = 11, 2

    def fwd(v):
        approx, det = symdwt.sym_dwt(v, h, levels)
        return np.concatenate([approx.ravel()] + [b.ravel() for lev in det for b in lev.values()])

    W = np.stack([fwd(e) for e in np.eye(n)], axis=1)
    approx0, det0 = symdwt.sym_dwt(np.zeros(n), h, levels)
    sizes = [approx0.size] + [b.size for lev in det0 for b in lev.values()]

    def inv(c):
        parts = np.split(c, np.cumsum(sizes)[:-1])
        approx = parts[0]
        det, j = [], 1
        for lev in det0:
            det.append({k: parts[j + q] for q, k in enumerate(lev)})
            j += len(lev)
        return symdwt.sym_idwt(approx, det, h, (n,))

    R = np.stack([inv(e) for e in np.eye(W.shape[0])], axis=1)
    np.testing.assert_allclose(R @ W, np.eye(n), atol=1e-12)
    assert np.abs(W.T @ W - np.eye(n)).max() > 1e-3
    C = np.stack([symdwt.sym_cov_apply(e, order, levels, 1.0) for e in np.eye(n)], axis=1)
    assert np.abs(C - C.T).max() > 1e-3


@pytest.mark.parametrize("shape,levels", [((64,), 4), ((32, 16), 3), ((8, 16, 8), 2)])
def test_haar_equals_periodic_operator_on_dyadic_sides(shape, levels):
    """With two taps no step reaches past an even-length axis, so the symmetric and the periodic
    transforms coincide, and so do their operators."""
    x = _rng("haar", shape).standard_normal(shape)
    got = symdwt.sym_cov_apply(x, 1, levels, 1.5)
    ref = oracle.matern_cov_apply(x, 1, levels, 1.5)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("shape,levels", [((37,), 4), ((12, 19), 3), ((5, 6, 7), 2)])
def test_operator_identities(order, shape, levels):
    """s = 0 and depth 0 give the identity (W^{-1} W = I); a constant stays constant (the
    mirror of a constant is constant, and every detail filter sums to zero)."""
    x = _rng("ident", order, shape).standard_normal(shape)
    np.testing.assert_allclose(symdwt.sym_cov_apply(x, order, levels, 0.0), x, atol=1e-11)
    np.testing.assert_allclose(symdwt.sym_cov_apply(x, order, 0, 2.0), x, atol=0)
    c = np.full(shape, 0.7)
    np.testing.assert_allclose(symdwt.sym_cov_apply(c, order, levels, 1.3), c, atol=1e-11)


def test_projection_form_equals_definition():
    """The low-pass recurrence y = w_1 x + R_A z_1, z_i = c_i a_i + R_A z_{i+1},
    z_{m-1} = c_{m-1} a_{m-1} (R_A: synthesis from the low band alone) equals W^{-1} D W."""
    order, levels, s = 6, 4, 1.25
    h = oracle.daubechies_lowpass(order)
    x = _rng("proj").standard_normal((23, 30))
    w = oracle.level_weights(levels, s, 2.0)
    c = [w[i + 1] - w[i] for i in range(levels - 1)]
    a = [x]
    for _ in range(levels - 1):
        b = symdwt._bands(a[-1], h)
        a.append(b[(0, 0)])

    def lowsyn(z, shape):
        bands = {k: np.zeros_like(z) for k in [(0, 1), (1, 0), (1, 1)]}
        bands[(0, 0)] = z
        return symdwt._unbands(bands, h, shape)

    z = c[levels - 2] * a[levels - 1]
    for i in range(levels - 2, 0, -1):
        z = c[i - 1] * a[i] + lowsyn(z, a[i].shape)
    y = w[0] * x + lowsyn(z, x.shape)
    np.testing.assert_allclose(y, symdwt.sym_cov_apply(x, order, levels, s), atol=1e-12)


@pytest.mark.parametrize("order", [1, 2, 4, 8])
@pytest.mark.parametrize("n", [1, 3, 8, 13])
def test_step_adjoints(order, n):
    """<A x, (a, d)> = <x, A^T (a, d)> and <S (a, d), x> = <(a, d), S^T x> for one step."""
    h = oracle.daubechies_lowpass(order)
    l = symdwt.sym_length(n, h.size)
    r = _rng("adj", order, n)
    x, a, d = r.standard_normal((n, 3)), r.standard_normal((l, 3)), r.standard_normal((l, 3))
    fa, fd = symdwt.sym_analysis_axis(x, h, 0)
    lhs = np.sum(fa * a) + np.sum(fd * d)
    rhs = np.sum(x * symdwt.sym_analysis_axis_adjoint(a, d, h, 0, n))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    s = symdwt.sym_synthesis_axis(a, d, h, 0, n)
    ta, td = symdwt.sym_synthesis_axis_adjoint(x, h, 0, l)
    assert abs(np.sum(s * x) - (np.sum(a * ta) + np.sum(d * td))) <= 1e-12 * max(1.0, abs(np.sum(s * x)))


@pytest.mark.parametrize("shape", [(5,), (9,), (4, 6), (3, 2, 5)])
@pytest.mark.parametrize("order", [1, 2, 4])
@pytest.mark.parametrize("levels", [0, 1, 2, 3])
def test_transpose_is_the_dense_transpose(shape, order, levels):
    """sym_cov_apply_transpose against the transpose of the operator's dense matrix, built column by
    column from sym_cov_apply (brute force; the operator is not symmetric)."""
    N = int(np.prod(shape))
    cols = []
    tcols = []
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        cols.append(symdwt.sym_cov_apply(e.reshape(shape), order, levels, 1.5).ravel())
        tcols.append(symdwt.sym_cov_apply_transpose(e.reshape(shape), order, levels, 1.5).ravel())
    T, TT = np.array(cols).T, np.array(tcols).T
    np.testing.assert_allclose(TT, T.T, rtol=0, atol=1e-12)
    if levels >= 2 and order > 1 and max(shape) > 2:
        assert np.abs(T - T.T).max() > 1e-6  # not symmetric: the transpose is a different operator
