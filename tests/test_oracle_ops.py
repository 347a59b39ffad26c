"""Pins of the oracle's four operators against closed forms, identities and brute force."""
import os

import numpy as np
import pytest

import oracle
from oracle import (daubechies_lowpass, dwt, es_adjoint, es_apply, idwt, level_weights, matern_cov_apply,
                    matern_sample, weight_map)
from oracle.dense import operator_matrices

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


def test_level_weights_golden():
    """Weights follow the paper's per-level rule (Sec. 4), not the literal listing of D (see DESIGN)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "level_weights.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) >= 8
    for r in rows:
        s, tau, m = float(r[0]), float(r[1]), int(r[2])
        approx_e, det_e = float(r[3]), [float(v) for v in r[4:]]
        assert len(det_e) == m and approx_e == 0
        assert np.array_equal(level_weights(m, s, tau), 2.0 ** np.array(det_e))


def _block_mean(x, b):
    """Mean over aligned blocks of side b on every axis, broadcast back to x's shape."""
    if b == 1:
        return x.copy()
    shp = []
    for n in x.shape:
        shp += [n // b, b]
    y = x.reshape(shp).mean(axis=tuple(range(1, 2 * x.ndim, 2)), keepdims=True)
    return np.broadcast_to(y, shp).reshape(x.shape)


@pytest.mark.parametrize("shape,levels", [((64,), 4), ((32, 64), 5), ((16, 16, 32), 3), ((8, 8), 1)])
@pytest.mark.parametrize("s", [0.5, 1.0, 1.5])
def test_haar_block_mean_closed_form(shape, levels, s):
    """With Haar, P_i is the aligned 2^i-block mean M_i, so
    W^T D_tau W x = M_{m-1} x + sum_{i<m} 2^{-tau s (m-i)} (M_{i-1} - M_i) x."""
    x = _rand(shape, 5)
    for tau, op in [(2.0, matern_cov_apply), (1.0, matern_sample)]:
        m = levels
        y = _block_mean(x, 1 << (m - 1))
        for i in range(1, m):
            y = y + 2.0 ** (-tau * s * (m - i)) * (_block_mean(x, 1 << (i - 1)) - _block_mean(x, 1 << i))
        assert np.max(np.abs(op(x, 1, levels, s) - y)) < 1e-13 * np.max(np.abs(x))


@pytest.mark.parametrize("shape", [(16, 16), (64,), (8, 8, 8)])
@pytest.mark.parametrize("order", [1, 2, 4])
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_spectrum_closed_form(shape, order, levels):
    """Eigenvalues of W^T D_2s W are the weights with their band multiplicities (any filter, any alignment)."""
    s = 0.75
    d = len(shape)
    N = int(np.prod(shape))
    _, _, C, S = operator_matrices(shape, order, levels, s)
    m = levels
    expect = [1.0] * (N >> (d * (m - 1)))
    for i in range(1, m):
        expect += [2.0 ** (-2 * s * (m - i))] * ((2 ** d - 1) * (N >> (d * i)))
    assert len(expect) == N
    assert np.max(np.abs(np.sort(np.linalg.eigvalsh(C)) - np.sort(expect))) < 1e-12
    assert abs(np.trace(C) - sum(expect)) < 1e-11
    assert np.max(np.abs(S @ S - C)) < 1e-13


@pytest.mark.parametrize("order", [1, 2, 4, 6, 8])
@pytest.mark.parametrize("levels", [1, 2, 4])
def test_ops_vs_dense(order, levels):
    shape = (16, 16)
    s = 1.3
    A, B, C, S = operator_matrices(shape, order, levels, s)
    x = _rand(shape, 1)
    assert np.max(np.abs(es_adjoint(x, order, levels, s).ravel() - A @ x.ravel())) < 1e-13
    assert np.max(np.abs(es_apply(x, order, levels, s).ravel() - B @ x.ravel())) < 1e-13
    assert np.max(np.abs(matern_cov_apply(x, order, levels, s).ravel() - C @ x.ravel())) < 1e-13
    assert np.max(np.abs(matern_sample(x, order, levels, s).ravel() - S @ x.ravel())) < 1e-13


def _op_matrix(fn, shape, *args):
    N = int(np.prod(shape))
    M = np.empty((N, N))
    for p in range(N):
        e = np.zeros(N)
        e[p] = 1.0
        M[:, p] = fn(e.reshape(shape), *args).ravel()
    return M


@pytest.mark.parametrize("shape,order,levels", [((16, 16), 4, 3), ((32,), 8, 2), ((8, 8, 8), 2, 2), ((8, 16), 6, 3)])
def test_adjointness_bruteforce(shape, order, levels):
    """<es_adjoint x, c> = <x, es_apply c>: the matrix of es_apply is the transpose of es_adjoint's;
    the covariance and the sampler are symmetric."""
    s = 1.7
    E = _op_matrix(es_adjoint, shape, order, levels, s)
    F = _op_matrix(es_apply, shape, order, levels, s)
    C = _op_matrix(matern_cov_apply, shape, order, levels, s)
    S = _op_matrix(matern_sample, shape, order, levels, s)
    assert np.max(np.abs(F - E.T)) < 1e-13
    assert np.max(np.abs(C - C.T)) < 1e-13
    assert np.max(np.abs(S - S.T)) < 1e-13


@pytest.mark.parametrize("shape,levels", [((128,), 5), ((64, 32), 4), ((16, 16, 16), 3)])
@pytest.mark.parametrize("order", [2, 5, 8])
def test_identities(shape, levels, order):
    x = _rand(shape, 2)
    tol = 1e-13 * np.max(np.abs(x))
    # s = 0 gives the identity; so does m = 0
    for op in (matern_cov_apply, matern_sample):
        assert np.max(np.abs(op(x, order, levels, 0.0) - x)) < tol
        assert np.max(np.abs(op(x, order, 0, 2.0) - x)) < tol
    assert np.array_equal(es_adjoint(x, order, 0, 1.0), x)
    # constants are reproduced exactly (they live in the approximation space, weight 1)
    cst = np.full(shape, 0.37)
    for op in (matern_cov_apply, matern_sample):
        assert np.max(np.abs(op(cst, order, levels, 1.5) - 0.37)) < 1e-14
    # compositions
    s1, s2 = 0.6, 1.1
    c12 = matern_cov_apply(matern_cov_apply(x, order, levels, s1), order, levels, s2)
    assert np.max(np.abs(c12 - matern_cov_apply(x, order, levels, s1 + s2))) < tol
    ss = matern_sample(matern_sample(x, order, levels, s2), order, levels, s2)
    assert np.max(np.abs(ss - matern_cov_apply(x, order, levels, s2))) < tol
    ea = es_apply(es_adjoint(x, order, levels, s2), order, levels, s2)
    assert np.max(np.abs(ea - matern_cov_apply(x, order, levels, s2))) < tol


def test_hs_inner_product_defines_adjoint():
    """<E_s^* x, y>_{H^s} = <x, y>_{L2} with <u, v>_{H^s} = <D_2s^{-1} W u, W v> (Sec. 3: E_s = I, Gamma = (E_s^*)^{-1/2})."""
    shape, order, levels, s = (32, 32), 4, 4, 1.5
    h = daubechies_lowpass(order)
    x, y = _rand(shape, 8), _rand(shape, 9)
    wmap = weight_map(shape, levels, s, 2.0)
    lhs = np.sum(dwt(matern_cov_apply(x, order, levels, s), h, levels) / wmap * dwt(y, h, levels))
    assert abs(lhs - np.sum(x * y)) < 1e-12 * np.linalg.norm(x) * np.linalg.norm(y)
    # ||x||_{H^s}^2 = <x, Gamma^2 x>, and Gamma^2 inverts the covariance
    xc = matern_cov_apply(x, order, levels, s)
    assert abs(oracle.hs_norm_sq(xc, order, levels, s) - np.sum(xc * x)) < 1e-11 * np.sum(x * x)


def test_hs_norm_parseval_and_levels():
    """s = 0: the orthonormal W keeps the Euclidean norm (Parseval); a detail-only input of one
    level scales as 2^{2 s j}; a constant lives in the approximation (weight 1)."""
    shape, order, levels = (32, 16), 4, 3
    x = _rand(shape, 11)
    assert abs(oracle.hs_norm_sq(x, order, levels, 0.0) - np.sum(x * x)) < 1e-12 * np.sum(x * x)
    h = daubechies_lowpass(order)
    c = np.zeros(shape)
    c[8:16, 0:4] = _rand((8, 4), 12)  # band (1, 0) of level 2: rows [n0/4, n0/2), cols [0, n1/4); j = m - 2 = 1
    xi = idwt(c, h, levels)
    for s in (0.5, 1.5, -1.0):
        assert abs(oracle.hs_norm_sq(xi, order, levels, s) - 2.0 ** (2 * s * 1) * np.sum(c * c)) < 1e-11 * np.sum(c * c)
    k = np.full(shape, 0.3)
    assert abs(oracle.hs_norm_sq(k, order, levels, 2.0) - np.sum(k * k)) < 1e-12 * np.sum(k * k)


def test_weight_map_layout():
    """Band geometry of the packed pyramid in 2-D, m = 2, s = 1, tau = 2."""
    w = weight_map((8, 8), 2, 1.0, 2.0)
    assert np.all(w[:2, :2] == 1.0)          # approximation
    assert np.all(w[:4, 2:4] == 1.0) and np.all(w[2:4, :4] == 1.0)  # level 2 (coarsest) details
    assert np.all(w[4:, :] == 0.25) and np.all(w[:, 4:] == 0.25)    # level 1 details: 2^{-2}


@pytest.mark.parametrize("shape,order,levels,s,alpha", [((16, 16), 4, 3, 1.5, 0.05), ((8, 8, 8), 2, 2, 1.0, 0.3),
                                                        ((32,), 8, 3, 2.0, 0.01)])
def test_tikhonov_solve_matches_dense_direct_solve(shape, order, levels, s, alpha):
    """The oracle's CG solution of (M + alpha Gamma^2) x = M p equals a dense direct solve, with
    Gamma^2 built from the dense Kronecker matrices (W^T D_{-2s} W), and is a stationary point
    of J(x) = 1/2||Mx - p||^2 + alpha/2 ||x||^2_{H^s}."""
    gen = np.random.default_rng(21)
    p = gen.standard_normal(shape)
    mask = (gen.random(shape) < 0.4).astype(np.float64)
    x = oracle.tikhonov_solve(p, mask, order, levels, s, alpha)
    G2 = operator_matrices(shape, order, levels, -s)[2]
    A = np.diag(mask.ravel()) + alpha * G2
    xd = np.linalg.solve(A, (mask * p).ravel()).reshape(shape)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    # gradient of J: M(Mx - p) + alpha Gamma^2 x (the H^s norm's gradient is 2 Gamma^2 x)
    grad = mask * (mask * x - p) + alpha * matern_cov_apply(x, order, levels, -s)
    assert np.linalg.norm(grad) <= 1e-10 * np.linalg.norm(mask * p)
    # and J(x) is below J at random perturbations
    def J(v):
        return 0.5 * np.sum((mask * v - p) ** 2) + 0.5 * alpha * oracle.hs_norm_sq(v, order, levels, s)
    for k in range(3):
        assert J(x) < J(x + 1e-3 * gen.standard_normal(shape))


def _gmres_system(shape, order, levels, s, alpha, seed, binary):
    gen = np.random.default_rng(seed)
    p = gen.standard_normal(shape)
    mask = (gen.random(shape) < 0.4).astype(np.float64) if binary else gen.random(shape)
    E = operator_matrices(shape, order, levels, s)[2]  # W^T D_{2s} W, dense
    A = E @ np.diag((mask * mask).ravel()) + alpha * np.eye(E.shape[0])
    b = E @ (mask * p).ravel()
    return p, mask, A, b


@pytest.mark.parametrize("shape,order,levels,s,alpha", [((16, 16), 4, 3, 1.5, 0.05), ((8, 8, 4), 2, 2, 1.0, 0.2)])
def test_tikhonov_gmres_iterates_are_least_residual_in_the_krylov_space(shape, order, levels, s, alpha):
    """Each GMRES iterate x_k is the point of least residual in the Krylov space
    K_k(E_s^* K^* K + alpha I, E_s^* K^* p) (Sec. 5 and its convergence figure), found here by brute
    force: an orthonormal basis of the explicitly built space [b, Ab, ..., A^{k-1} b] and a dense
    least-squares solve.  A non-binary mask makes K^* K = diag(mask^2) differ from diag(mask)."""
    p, mask, A, b = _gmres_system(shape, order, levels, s, alpha, 3, False)
    prev = np.inf
    for k in range(1, 7):
        x = oracle.tikhonov_gmres(p, mask, order, levels, s, alpha, iters=k).ravel()
        cols = [b]
        for _ in range(k - 1):
            cols.append(A @ cols[-1])
        Q = np.linalg.qr(np.stack(cols, axis=1))[0]
        c = np.linalg.lstsq(A @ Q, b, rcond=None)[0]
        xb = Q @ c
        assert np.linalg.norm(x - xb) <= 1e-7 * np.linalg.norm(xb), k
        res = np.linalg.norm(b - A @ x)
        assert res <= prev * (1 + 1e-12)  # minimal residuals never grow with the space
        prev = res


def test_tikhonov_gmres_full_space_is_the_direct_solve():
    """After as many steps as unknowns the Krylov space is the whole space: GMRES returns the dense
    direct solution of (E_s^* K^* K + alpha I) x = E_s^* K^* p; restarted GMRES converges to it too."""
    shape, order, levels, s, alpha = (8, 8), 2, 2, 1.0, 0.1
    p, mask, A, b = _gmres_system(shape, order, levels, s, alpha, 4, False)
    xd = np.linalg.solve(A, b)
    x = oracle.tikhonov_gmres(p, mask, order, levels, s, alpha, iters=64).ravel()
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    xr = oracle.tikhonov_gmres(p, mask, order, levels, s, alpha, iters=400, restart=8).ravel()
    assert np.linalg.norm(xr - xd) <= 1e-8 * np.linalg.norm(xd)


def test_tikhonov_gmres_solution_is_the_cg_solution_for_binary_masks():
    """With a 0/1 mask (K^* K = diag(mask)) the paper's equation and the normal equations solved by
    the CG oracle have the same solution (multiply by Gamma^2 = (E_s^*)^{-1})."""
    shape, order, levels, s, alpha = (16, 16), 4, 3, 1.5, 0.05
    p, mask, A, b = _gmres_system(shape, order, levels, s, alpha, 5, True)
    xg = oracle.tikhonov_gmres(p, mask, order, levels, s, alpha, iters=600, restart=30)
    xc = oracle.tikhonov_solve(p, mask, order, levels, s, alpha)
    assert np.linalg.norm(xg - xc) <= 1e-8 * np.linalg.norm(xc)
