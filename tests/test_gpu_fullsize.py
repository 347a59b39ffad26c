"""Parity at the full workload sizes, in the launch configuration the benchmark times.

The oracle recomputes sampled instances one by one; relative L2 <= 1e-5 per result.
"""
import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_2507_02401_amd as es
from paper_2507_02401_amd import autograd as ag
from tests.gpu_util import TOL, rel_l2, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_small_image_128():
    d = inputs.small_image()
    x64 = d["x"].astype(np.float64)
    xt = torch.from_numpy(d["x"]).to(DEV)
    say("128^2 small image")
    for op, ref in [(es.OP_COV, oracle.matern_cov_apply), (es.OP_SAMPLE, oracle.matern_sample),
                    (es.OP_ADJOINT, oracle.es_adjoint), (es.OP_APPLY, oracle.es_apply)]:
        y = es.apply_op(op, xt, 2, d["order"], d["levels"], d["s"]).cpu().numpy()
        assert rel_l2(y, ref(x64, d["order"], d["levels"], d["s"])) <= TOL


def test_image_batch_64x1024():
    d = inputs.image_batch(count=64, side=1024)
    say("64 x 1024^2 db8 m7 cov")
    x = torch.from_numpy(d["x"]).to(DEV)
    y = es.matern_cov_apply(x, 2, d["order"], d["levels"], d["s"])
    for b in (0, 37, 63):
        ref = oracle.matern_cov_apply(d["x"][b].astype(np.float64), d["order"], d["levels"], d["s"])
        assert rel_l2(y[b].cpu().numpy(), ref) <= TOL
    # results do not depend on the neighbours in the batch
    y1 = es.matern_cov_apply(x[37:38].contiguous(), 2, d["order"], d["levels"], d["s"])
    assert torch.equal(y1[0], y[37])
    # constant images stay constant (a constant lives in the approximation band, weight 1)
    c = torch.full((2, 1024, 1024), 0.75, dtype=torch.float32, device=DEV)
    c[1] = -2.5
    yc = es.matern_cov_apply(c, 2, d["order"], d["levels"], d["s"])
    assert float((yc - c).abs().max()) <= 1e-5 * 2.5


def test_volume_256_autograd():
    d = inputs.volume_autograd(side=256)
    say("256^3 db4 m5 es_adjoint fwd + bwd")
    x = torch.from_numpy(d["x"]).to(DEV).requires_grad_(True)
    yt = torch.from_numpy(d["y"]).to(DEV)
    c = ag.es_adjoint(x, 3, d["order"], d["levels"], d["s"])
    loss = 0.5 * ((c.double() - yt.double()) ** 2).sum()
    loss.backward()
    x64 = d["x"].astype(np.float64)
    cref = oracle.es_adjoint(x64, d["order"], d["levels"], d["s"])
    assert rel_l2(c.detach().cpu().numpy(), cref) <= TOL
    gref = oracle.es_apply(cref - d["y"], d["order"], d["levels"], d["s"])
    assert rel_l2(x.grad.cpu().numpy(), gref) <= TOL
    # central finite differences with FP64 loss accumulation.  The loss is quadratic, so the
    # central difference is exact for every h; what remains is the FP32 rounding of the
    # forward outputs o(x +- h v), whose contribution to the difference quotient is about
    # sqrt(sum_i (o_i - y_i)^2 o_i^2) * 2^-23 / h.  At h = 1e-3 and 256^3 voxels that is ~1e-2
    # of the directional derivative, so the h = 1e-3 check uses that bound and a second check
    # at h = 0.5 holds the derivative to 1e-4.
    v = torch.from_numpy(np.random.default_rng(5).standard_normal(d["x"].shape).astype(np.float32)).to(DEV)
    with torch.no_grad():
        def L(z):
            o = es.es_adjoint(z, 3, d["order"], d["levels"], d["s"])
            return 0.5 * ((o.double() - yt.double()) ** 2).sum().item()
        an = (x.grad.double() * v.double()).sum().item()
        o = es.es_adjoint(x.detach(), 3, d["order"], d["levels"], d["s"]).double()
        noise = float(torch.sqrt((((o - yt.double()) * o) ** 2).sum()).item()) * 2.0 ** -23
        for h in (1e-3, 0.5):
            fd = (L(x.detach() + h * v) - L(x.detach() - h * v)) / (2 * h)
            tol = max(1e-4 * abs(an), 4.0 * noise / h)
            say(f"fd h={h}: fd={fd:.6f} analytic={an:.6f} tol={tol:.3e}")
            assert abs(fd - an) <= tol


def test_map_gradient_batch_256x512():
    d = inputs.map_gradient_batch(count=256, side=512)
    say("256 x 512^2 db6 m6 sampler fwd + bwd")
    xi = torch.from_numpy(d["xi"]).to(DEV).requires_grad_(True)
    m = torch.from_numpy(d["mask"]).to(DEV)
    y = torch.from_numpy(d["y"]).to(DEV)
    x = ag.matern_sample(xi, 2, d["order"], d["levels"], d["s"])
    loss = 0.5 * ((m * x - y).double() ** 2).sum()
    loss.backward()
    for b in (0, 255):
        xr = oracle.matern_sample(d["xi"][b].astype(np.float64), d["order"], d["levels"], d["s"])
        assert rel_l2(x[b].detach().cpu().numpy(), xr) <= TOL
        gr = oracle.matern_sample(d["mask"][b] * (d["mask"][b] * xr - d["y"][b]), d["order"], d["levels"], d["s"])
        assert rel_l2(xi.grad[b].cpu().numpy(), gr) <= TOL
