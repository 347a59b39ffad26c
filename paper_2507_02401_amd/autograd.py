"""torch.autograd.Function forms of the four operators.

Every operator is linear, so the backward pass is the adjoint applied to the incoming
gradient: es_adjoint^T = es_apply (synthesis instead of analysis, same level weights),
es_apply^T = es_adjoint, and the covariance and the sampler are symmetric.  Only the scalar
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


def es_adjoint(x, ndim, order, levels, s):
    return EsAdjointFn.apply(x, ndim, order, levels, s)


def es_apply(c, ndim, order, levels, s):
    return EsApplyFn.apply(c, ndim, order, levels, s)


def matern_cov(x, ndim, order, levels, s):
    return MaternCovFn.apply(x, ndim, order, levels, s)


def matern_sample(xi, ndim, order, levels, s):
    return MaternSampleFn.apply(xi, ndim, order, levels, s)
