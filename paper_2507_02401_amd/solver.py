"""Matrix-free Tikhonov / MAP reconstruction around the wavelet prior operators.

With a measurement operator K and data p, the Tikhonov functional with the Sobolev penalty
(Sec. 3: ||x||_{H^s} = ||Gamma x||, Gamma^2 = (E_s^*)^{-1}; Sec. 4: the wavelet form of E_s^* and
its iterative solution by conjugate gradients)

    J(x) = 1/2 ||K x - p||^2 + alpha/2 ||x||^2_{H^s}

has the normal equations (K^T K + alpha Gamma^2) x = K^T p, with Gamma^2 = W^T D_{-2s} W, the
covariance operator of smoothness -s.  The system is symmetric positive definite; the library
solves it by conjugate gradients preconditioned with the inverse of the penalty term up to its
scale, E_s E_s^* (the covariance of smoothness +s), entirely on the GPU (es_tikhonov_pcg).  The
synthetic measurement here is a pixel mask (K = K^T = diag(mask)), standing in for the paper's
acoustic forward model, which is not part of this library.

The paper itself solves the regularised equation in the form (E_s^* K^* K + alpha I) x = E_s^* K^* p
(Sec. 3) by GMRES (Sec. 5); tikhonov_gmres runs restarted GMRES on exactly that system, again on the
GPU (es_tikhonov_gmres).  For a 0/1 mask both solvers have the same solution.

Instances along the leading dimensions are solved independently (per-instance step sizes).
"""
import ctypes
import math

import torch

from ._lib import check, load, shape_arg


def tikhonov_pcg(p, mask, ndim, order, levels, s, alpha, iters=100, rtol=1e-6, check_every=4):
    """Solve (diag(mask) + alpha W^T D_{-2s} W) x = mask * p per instance, from x = 0.

    p, mask: float32 GPU tensors of shape (*batch, *grid).  Returns (x, info) with
    info = {"iterations": int, "rel_residual": float64 CPU tensor of the batch shape}.  Stops when
    every instance's residual ||r|| / ||b|| is at most rtol (checked every `check_every`
    iterations), or after `iters` iterations.
    """
    if alpha <= 0:
        raise ValueError("alpha must be positive")
    if p.shape != mask.shape:
        raise ValueError("p and mask must have the same shape")
    for t in (p, mask):
        if t.dtype != torch.float32 or t.device.type != "cuda":
            raise TypeError("p and mask must be float32 GPU tensors")
    p = p.contiguous()
    mask = mask.contiguous()
    grid = tuple(p.shape[p.dim() - ndim:])
    bshape = tuple(p.shape[:p.dim() - ndim])
    batch = math.prod(bshape)
    lib = load()
    shp = shape_arg(grid)
    need = int(lib.es_tikhonov_pcg_workspace_bytes(ndim, shp, batch, int(order), int(levels)))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=p.device)
    x = torch.empty_like(p)
    its = ctypes.c_int32(0)
    rel = (ctypes.c_float * max(1, batch))()
    with torch.cuda.device(p.device):
        stream = torch.cuda.current_stream(p.device).cuda_stream
        check(lib.es_tikhonov_pcg(ndim, shp, batch, int(order), int(levels), float(s), float(alpha), p.data_ptr(),
                                  mask.data_ptr(), x.data_ptr(), int(iters), float(rtol), int(check_every),
                                  ctypes.byref(its), rel, ws.data_ptr(), need, stream))
    rel_t = torch.tensor(list(rel[:batch]), dtype=torch.float64).reshape(bshape)
    return x, {"iterations": int(its.value), "rel_residual": rel_t}


def tikhonov_gmres(p, mask, ndim, order, levels, s, alpha, iters=15, restart=15, rtol=1e-6):
    """Solve (E_s^* diag(mask)^2 + alpha I) x = E_s^*(mask * p) per instance by restarted GMRES from x = 0.

    p, mask: float32 GPU tensors of shape (*batch, *grid).  At most `iters` Arnoldi steps with a
    basis of `restart` vectors (1..64).  Returns (x, info) with info = {"iterations": int,
    "rel_residual": float64 CPU tensor of the batch shape} (the true relative residual of x).
    """
    if alpha <= 0:
        raise ValueError("alpha must be positive")
    if p.shape != mask.shape:
        raise ValueError("p and mask must have the same shape")
    for t in (p, mask):
        if t.dtype != torch.float32 or t.device.type != "cuda":
            raise TypeError("p and mask must be float32 GPU tensors")
    p = p.contiguous()
    mask = mask.contiguous()
    grid = tuple(p.shape[p.dim() - ndim:])
    bshape = tuple(p.shape[:p.dim() - ndim])
    batch = math.prod(bshape)
    lib = load()
    shp = shape_arg(grid)
    need = int(lib.es_tikhonov_gmres_workspace_bytes(ndim, shp, batch, int(order), int(levels), int(restart)))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=p.device)
    x = torch.empty_like(p)
    its = ctypes.c_int32(0)
    rel = (ctypes.c_float * max(1, batch))()
    with torch.cuda.device(p.device):
        stream = torch.cuda.current_stream(p.device).cuda_stream
        check(lib.es_tikhonov_gmres(ndim, shp, batch, int(order), int(levels), float(s), float(alpha), p.data_ptr(),
                                    mask.data_ptr(), x.data_ptr(), int(restart), int(iters), float(rtol),
                                    ctypes.byref(its), rel, ws.data_ptr(), need, stream))
    rel_t = torch.tensor(list(rel[:batch]), dtype=torch.float64).reshape(bshape)
    return x, {"iterations": int(its.value), "rel_residual": rel_t}
