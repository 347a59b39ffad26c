"""Dense-matrix form of the transform and operators, for brute-force tests on tiny grids.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The 1-D analysis matrix of length n has row k (k < n/2) holding h[t] at column
(2k+t) mod n and row n/2+k holding g[t] there (taps that fold onto the same
column add up, which happens when n < L).  One d-dimensional level is the
Kronecker product of the 1-D matrices of the current block sides, acting on the
row-major vectorisation of that block and as the identity elsewhere.  W is the
product of its levels, finest first.  This builds the matrices explicitly, a
formulation independent of the gather-based transform in `dwt`.
"""

import numpy as np

from .filters import daubechies_lowpass, quadrature_highpass


def analysis_matrix_1d(n, h):
    h = np.asarray(h, dtype=np.float64)
    g = quadrature_highpass(h)
    A = np.zeros((n, n))
    for k in range(n // 2):
        for t in range(h.size):
            A[k, (2 * k + t) % n] += h[t]
            A[n // 2 + k, (2 * k + t) % n] += g[t]
    return A


def level_matrix(shape, block, h):
    """N x N matrix of one level acting on the leading sub-block `block` of an array of `shape`."""
    N = int(np.prod(shape))
    K = np.ones((1, 1))
    for b in block:
        K = np.kron(K, analysis_matrix_1d(b, h))
    idx = np.arange(N).reshape(shape)[tuple(slice(0, b) for b in block)].ravel()
    M = np.eye(N)
    M[np.ix_(idx, idx)] = K
    return M


def dwt_matrix(shape, h, levels):
    N = int(np.prod(shape))
    W = np.eye(N)
    block = list(shape)
    for _ in range(levels):
        W = level_matrix(shape, block, h) @ W
        block = [b // 2 for b in block]
    return W


def weight_diagonal(shape, levels, s, tau):
    """Diagonal of D_tau in the packed layout, built level by level from the band geometry."""
    m = levels
    N = int(np.prod(shape))
    dvec = np.empty(N)
    coords = np.indices(shape).reshape(len(shape), -1)
    for p in range(N):
        c = coords[:, p]
        # coarsest level whose leading block [0, n/2^{lev-1}) still contains the point
        lev = 1
        while lev < m and all(c[k] < (shape[k] >> lev) for k in range(len(shape))):
            lev += 1
        if m > 0 and all(c[k] < (shape[k] >> m) for k in range(len(shape))):
            dvec[p] = 1.0  # approximation band
        elif m == 0:
            dvec[p] = 1.0
        else:
            dvec[p] = 2.0 ** (-tau * s * (m - lev))
    return dvec


def operator_matrices(shape, order, levels, s):
    """Dense (es_adjoint, es_apply, matern_cov, matern_sample) matrices."""
    h = daubechies_lowpass(order)
    W = dwt_matrix(shape, h, levels)
    D1 = np.diag(weight_diagonal(shape, levels, s, 1.0))
    D2 = np.diag(weight_diagonal(shape, levels, s, 2.0))
    return D1 @ W, W.T @ D1, W.T @ D2 @ W, W.T @ D1 @ W
