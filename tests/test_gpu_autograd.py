"""Autograd: the hand-written backward of every operator is the exact adjoint.

Checked against the oracle's transpose (relative L2 <= 1e-5) and against central finite
differences with the loss accumulated in FP64 (the losses are quadratic, so the difference
quotient is exact up to rounding).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2507_02401_amd as es
from paper_2507_02401_amd import autograd as ag
from tests.gpu_util import TOL, rel_l2, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


@pytest.mark.parametrize("shape,ndim,order,levels,s", [((24, 40, 56), 3, 4, 3, 2.0), ((2, 96, 64), 2, 8, 4, 1.5),
                                                       ((4096,), 1, 3, 6, 1.0)])
def test_es_adjoint_backward_is_oracle_transpose(shape, ndim, order, levels, s):
    gen = np.random.default_rng(1)
    x = gen.standard_normal(shape).astype(np.float32)
    y = gen.standard_normal(shape).astype(np.float32)
    say("autograd es_adjoint", shape)
    xt = _t(x).requires_grad_(True)
    c = ag.es_adjoint(xt, ndim, order, levels, s)
    loss = 0.5 * ((c.double() - _t(y).double()) ** 2).sum()
    loss.backward()
    g = xt.grad.cpu().numpy()
    inst = shape[-ndim:]
    xb, yb, gb = x.reshape((-1,) + inst), y.reshape((-1,) + inst), g.reshape((-1,) + inst)
    for b in range(xb.shape[0]):
        r = oracle.es_adjoint(xb[b].astype(np.float64), order, levels, s) - yb[b]
        ref = oracle.es_apply(r, order, levels, s)
        assert rel_l2(gb[b], ref) <= TOL


@pytest.mark.parametrize("fn,ref_fwd,ref_bwd", [
    (ag.es_apply, oracle.es_apply, oracle.es_adjoint),
    (ag.matern_cov, oracle.matern_cov_apply, oracle.matern_cov_apply),
    (ag.matern_sample, oracle.matern_sample, oracle.matern_sample),
])
def test_backward_is_oracle_transpose(fn, ref_fwd, ref_bwd):
    shape, ndim, order, levels, s = (3, 64, 80), 2, 6, 4, 1.5
    gen = np.random.default_rng(2)
    x = gen.standard_normal(shape).astype(np.float32)
    m = (gen.random(shape) < 0.3).astype(np.float32)
    y = gen.standard_normal(shape).astype(np.float32)
    say("autograd", fn.__name__)
    xt = _t(x).requires_grad_(True)
    out = fn(xt, ndim, order, levels, s)
    loss = 0.5 * ((_t(m).double() * out.double() - _t(y).double()) ** 2).sum()
    loss.backward()
    g = xt.grad.cpu().numpy()
    for b in range(shape[0]):
        fwd = ref_fwd(x[b].astype(np.float64), order, levels, s)
        ref = ref_bwd(m[b] * (m[b] * fwd - y[b]), order, levels, s)
        assert rel_l2(g[b], ref) <= TOL


def _fd_check(fn, x, y, ndim, order, levels, s, h=1e-3, seed=3):
    """Central difference of L(x) = 0.5 ||fn(x) - y||^2 (FP64 accumulation) along a dense random v."""
    xt = _t(x).requires_grad_(True)
    out = fn(xt, ndim, order, levels, s)
    loss = 0.5 * ((out.double() - _t(y).double()) ** 2).sum()
    loss.backward()
    v = np.random.default_rng(seed).standard_normal(x.shape).astype(np.float32)
    vt = _t(v)
    with torch.no_grad():
        def L(z):
            o = fn(z, ndim, order, levels, s)
            return 0.5 * ((o.double() - _t(y).double()) ** 2).sum().item()
        fd = (L(_t(x) + h * vt) - L(_t(x) - h * vt)) / (2 * h)
    an = float((xt.grad.double() * vt.double()).sum().item())
    return abs(fd - an) / max(abs(an), 1e-30)


@pytest.mark.parametrize("fn", [ag.es_adjoint, ag.es_apply, ag.matern_cov, ag.matern_sample])
def test_finite_differences_small(fn):
    gen = np.random.default_rng(4)
    x = gen.standard_normal((48, 64, 32)).astype(np.float32)
    y = gen.standard_normal((48, 64, 32)).astype(np.float32)
    say("fd", fn.__name__)
    assert _fd_check(fn, x, y, 3, 4, 3, 2.0) < 1e-3
