"""torch.autograd.Function forms of the four operators, the squared H^s norm, the Fourier form and the
non-periodic operator.

Every operator is linear, so the backward pass is the adjoint applied to the incoming
gradient: es_adjoint^T = es_apply (synthesis instead of analysis, same level weights),
es_apply^T = es_adjoint, and the covariance and the sampler are symmetric; the non-periodic
operator W^{-1} D W is not, and its backward is its transpose.  Only the scalar
arguments are saved.
"""
import torch

from . import ops


class EsAdjointFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, ndim, order, levels, s):
        ctx.args = (ndim, order, levels, s)
        return ops.es_adjoint(x, ndim, order, levels, s)

    @staticmethod
    def backward(ctx, g):
        return ops.es_apply(g.contiguous(), *ctx.args), None, None, None, None


class EsApplyFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, ndim, order, levels, s):
        ctx.args = (ndim, order, levels, s)
        return ops.es_apply(c, ndim, order, levels, s)

    @staticmethod
    def backward(ctx, g):
        return ops.es_adjoint(g.contiguous(), *ctx.args), None, None, None, None


class MaternCovFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, ndim, order, levels, s):
        ctx.args = (ndim, order, levels, s)
        return ops.matern_cov_apply(x, ndim, order, levels, s)

    @staticmethod
    def backward(ctx, g):
        return ops.matern_cov_apply(g.contiguous(), *ctx.args), None, None, None, None


class MaternSampleFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xi, ndim, order, levels, s):
        ctx.args = (ndim, order, levels, s)
        return ops.matern_sample(xi, ndim, order, levels, s)

    @staticmethod
    def backward(ctx, g):
        return ops.matern_sample(g.contiguous(), *ctx.args), None, None, None, None


class HsNormSqFn(torch.autograd.Function):
    """||x||^2_{H^s} per instance; its gradient is 2 W^T D_{-2s} W x, the covariance operator with
    smoothness -s (the precision operator), scaled by the incoming gradient of each instance."""

    @staticmethod
    def forward(ctx, x, ndim, order, levels, s):
        ctx.args = (ndim, order, levels, s)
        ctx.save_for_backward(x)
        return ops.hs_norm_sq(x, ndim, order, levels, s)

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        ndim, order, levels, s = ctx.args
        p = ops.matern_cov_apply(x.contiguous(), ndim, order, levels, -s)
        scale = (2.0 * g).to(p.dtype).reshape(g.shape + (1,) * ndim)
        return scale * p, None, None, None, None


class FftCovFn(torch.autograd.Function):
    """Fourier form of E_s^*: real, symmetric (B is real and even), so its backward is itself."""

    @staticmethod
    def forward(ctx, x, ndim, s, period):
        ctx.args = (ndim, s, period)
        return ops.fft_cov_apply(x, ndim, s, period)

    @staticmethod
    def backward(ctx, g):
        return ops.fft_cov_apply(g.contiguous(), *ctx.args), None, None, None


def fft_cov(x, ndim, s, period=1.0):
    return FftCovFn.apply(x, ndim, s, period)


def hs_norm_sq(x, ndim, order, levels, s):
    return HsNormSqFn.apply(x, ndim, order, levels, s)


def es_adjoint(x, ndim, order, levels, s):
    return EsAdjointFn.apply(x, ndim, order, levels, s)


def es_apply(c, ndim, order, levels, s):
    return EsApplyFn.apply(c, ndim, order, levels, s)


def matern_cov(x, ndim, order, levels, s):
    return MaternCovFn.apply(x, ndim, order, levels, s)


def matern_sample(xi, ndim, order, levels, s):
    return MaternSampleFn.apply(xi, ndim, order, levels, s)


class SymCovFn(torch.autograd.Function):
    """W^{-1} D_2s W with the non-periodic transform; backward: its transpose W^T D_2s W^{-T}."""

    @staticmethod
    def forward(ctx, x, ndim, order, levels, s):
        ctx.args = (ndim, order, levels, s)
        return ops.sym_cov_apply(x, ndim, order, levels, s)

    @staticmethod
    def backward(ctx, g):
        return ops.sym_cov_apply_transpose(g.contiguous(), *ctx.args), None, None, None, None


class SymCovTFn(torch.autograd.Function):
    """The transpose of SymCovFn; backward: the operator itself."""

    @staticmethod
    def forward(ctx, y, ndim, order, levels, s):
        ctx.args = (ndim, order, levels, s)
        return ops.sym_cov_apply_transpose(y, ndim, order, levels, s)

    @staticmethod
    def backward(ctx, g):
        return ops.sym_cov_apply(g.contiguous(), *ctx.args), None, None, None, None


def sym_cov_apply(x, ndim, order, levels, s):
    return SymCovFn.apply(x, ndim, order, levels, s)


def sym_cov_apply_transpose(y, ndim, order, levels, s):
    return SymCovTFn.apply(y, ndim, order, levels, s)
