"""Matrix-free Tikhonov / MAP reconstruction around the wavelet prior operators.

With a measurement operator K and data p, the Tikhonov functional with the Sobolev penalty
(Sec. 3: ||x||_{H^s} = ||Gamma x||, Gamma^2 = (E_s^*)^{-1}; Sec. 4: the wavelet form of E_s^*)

    J(x) = 1/2 ||K x - p||^2 + alpha/2 ||x||^2_{H^s}

has the normal equations (K^T K + alpha Gamma^2) x = K^T p, with Gamma^2 = W^T D_{-2s} W, the
covariance operator of smoothness -s.  The system is symmetric positive definite; it is solved by
conjugate gradients preconditioned with the inverse of the penalty term, (alpha Gamma^2)^{-1} =
E_s E_s^* / alpha (the covariance of smoothness +s), so every iteration applies the wavelet
operator twice on the GPU; vector updates and inner products are torch operations.  The
synthetic measurement here is a pixel mask (K = K^T = diag(mask)), standing in for the paper's
acoustic forward model, which is not part of this library.

Instances along the leading dimensions are solved independently (per-instance step sizes).
"""
import torch

from . import ops


def _dot(a, b, ndim):
    """Per-instance inner product over the trailing ndim dims (FP32 reduction, returned as FP64)."""
    return torch.linalg.vecdot(a.flatten(a.dim() - ndim), b.flatten(b.dim() - ndim)).double()


def _bcast(v, ndim, like):
    return v.to(like.dtype).reshape(v.shape + (1,) * ndim)


def tikhonov_pcg(p, mask, ndim, order, levels, s, alpha, iters=100, rtol=1e-6, x0=None):
    """Solve (diag(mask) + alpha W^T D_{-2s} W) x = mask * p per instance.

    p, mask: float32 GPU tensors of shape (*batch, *grid).  Returns (x, info) with
    info = {"iterations": int, "rel_residual": float64 tensor of the batch shape}.
    Preconditioner: W^T D_{2s} W (the iterates do not depend on its scale, so the 1/alpha of the
    exact inverse of the penalty term is left out).  Stops when every instance's residual
    ||r|| / ||b|| is below rtol, or after `iters` iterations.
    """
    if alpha <= 0:
        raise ValueError("alpha must be positive")

    def A(v):
        return torch.addcmul(alpha * ops.matern_cov_apply(v, ndim, order, levels, -s), mask, v)

    def P(v):
        return ops.matern_cov_apply(v, ndim, order, levels, s)

    b = mask * p
    x = torch.zeros_like(p) if x0 is None else x0.clone()
    r = b - A(x) if x0 is not None else b.clone()
    bn = _dot(b, b, ndim).sqrt().clamp_min(1e-300)
    z = P(r)
    d = z.clone()
    rz = _dot(r, z, ndim)
    it = 0
    rel = _dot(r, r, ndim).sqrt() / bn
    while it < iters and bool((rel > rtol).any()):
        ad = A(d)
        active = rel > rtol
        a = torch.where(active, rz / _dot(d, ad, ndim).clamp_min(1e-300), torch.zeros_like(rz))
        x.addcmul_(d, _bcast(a, ndim, x))
        r.addcmul_(ad, _bcast(-a, ndim, r))
        z = P(r)
        rz_new = _dot(r, z, ndim)
        beta = torch.where(active, rz_new / rz.clamp_min(1e-300), torch.zeros_like(rz))
        d.mul_(_bcast(beta, ndim, d)).add_(z)
        rz = rz_new
        rel = _dot(r, r, ndim).sqrt() / bn
        it += 1
    return x, {"iterations": it, "rel_residual": rel}
