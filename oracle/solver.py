"""FP64 reference solution of the Tikhonov normal equations (TEST INFRASTRUCTURE ONLY).

J(x) = 1/2 ||M x - p||^2 + alpha/2 ||x||^2_{H^s} with M = diag(mask) and ||x||^2_{H^s} = ||Gamma x||^2,
Gamma^2 = W^T D_{-2s} W (Sec. 3 and Sec. 4): the minimiser solves (M + alpha Gamma^2) x = M p.
Solved here by plain conjugate gradients in FP64 (no preconditioner) to a residual of 1e-13,
with the oracle's own operator; pinned against a dense direct solve on tiny grids.
"""
import numpy as np

from .ops import matern_cov_apply


def tikhonov_solve(p, mask, order, levels, s, alpha, tol=1e-13, max_iter=100000):
    p = np.asarray(p, dtype=np.float64)
    mask = np.asarray(mask, dtype=np.float64)

    def A(v):
        return mask * v + alpha * matern_cov_apply(v, order, levels, -s)

    b = mask * p
    x = np.zeros_like(b)
    r = b.copy()
    d = r.copy()
    rr = float(np.sum(r * r))
    bn = np.sqrt(float(np.sum(b * b))) or 1.0
    for _ in range(max_iter):
        if np.sqrt(rr) <= tol * bn:
            break
        ad = A(d)
        a = rr / float(np.sum(d * ad))
        x += a * d
        r -= a * ad
        rr_new = float(np.sum(r * r))
        d = r + (rr_new / rr) * d
        rr = rr_new
    return x
