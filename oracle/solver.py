"""FP64 reference solution of the Tikhonov normal equations (TEST INFRASTRUCTURE ONLY).

J(x) = 1/2 ||M x - p||^2 + alpha/2 ||x||^2_{H^s} with M = diag(mask) and ||x||^2_{H^s} = ||Gamma x||^2,
Gamma^2 = W^T D_{-2s} W (Sec. 3 and Sec. 4): the minimiser solves (M + alpha Gamma^2) x = M p.
Solved here by plain conjugate gradients in FP64 (no preconditioner) to a residual of 1e-13,
with the oracle's own operator; pinned against a dense direct solve on tiny grids.

tikhonov_gmres: the paper's own form of the equation and its solver, GMRES on
(E_s^* K^* K + alpha I) x = E_s^* K^* p, in FP64; pinned by brute force (each iterate is the least
residual point of the explicitly built Krylov space), by a dense direct solve after as many steps
as unknowns, and by the CG solution above for 0/1 masks.
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


def tikhonov_gmres(p, mask, order, levels, s, alpha, iters, restart=None):
    """GMRES in FP64 on the regularised equation in the paper's form (Sec. 3; solved by GMRES in
    Sec. 5):  (E_s^* K^* K + alpha I) x = E_s^* K^* p,  K = diag(mask),  E_s^* = W^T D_{2s} W.

    From x = 0, `iters` Arnoldi steps in cycles of `restart` (default: no restart).  Each cycle
    builds an orthonormal basis V of the Krylov space of A and the cycle's residual r (Arnoldi with
    modified Gram-Schmidt, A V_k = V_{k+1} H_k), takes y minimising ||beta e_1 - H_k y|| (a library
    least-squares solve) and sets x += V_k y: the iterate of least residual in x + K_k(A, r).
    """
    p = np.asarray(p, dtype=np.float64)
    mask = np.asarray(mask, dtype=np.float64)

    def A(v):
        return matern_cov_apply(mask * mask * v, order, levels, s) + alpha * v

    b = matern_cov_apply(mask * p, order, levels, s)
    x = np.zeros_like(b)
    m = iters if restart is None else restart
    done = 0
    while done < iters:
        r = b - A(x)
        beta = np.sqrt(float(np.sum(r * r)))
        if beta == 0.0:
            break
        k = min(m, iters - done)
        V = [r / beta]
        H = np.zeros((k + 1, k))
        steps = 0
        for j in range(k):
            w = A(V[j])
            for i in range(j + 1):
                H[i, j] = float(np.sum(w * V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.sqrt(float(np.sum(w * w)))
            steps = j + 1
            if H[j + 1, j] == 0.0:
                break
            V.append(w / H[j + 1, j])
        e1 = np.zeros(steps + 1)
        e1[0] = beta
        y = np.linalg.lstsq(H[:steps + 1, :steps], e1, rcond=None)[0]
        for i in range(steps):
            x = x + y[i] * V[i]
        done += k
    return x
