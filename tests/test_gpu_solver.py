"""GPU: matrix-free Tikhonov reconstruction with the H^s prior (preconditioned CG around the
wavelet operators) vs the FP64 oracle solution of the normal equations."""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_02401_amd.solver import tikhonov_pcg
from tests.gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu

# FP32 operator applications carry ~1e-6 relative error; the preconditioned system's condition
# number is about 1 + 1/alpha (<= 21 here), and CG stops at a residual of 1e-6: 1e-4 covers both.
SOLVE_TOL = 1e-4


@pytest.mark.parametrize("shape,ndim,order,levels,s,alpha", [((2, 64, 96), 2, 4, 4, 1.5, 0.05),
                                                             ((16, 32, 32), 3, 2, 3, 1.0, 0.1),
                                                             ((3, 128, 128), 2, 8, 5, 1.0, 0.2),
                                                             ((2, 256, 320), 2, 4, 5, 1.5, 0.05),
                                                             ((1, 512, 512), 2, 8, 6, 1.0, 0.1)])
def test_tikhonov_pcg_matches_oracle(shape, ndim, order, levels, s, alpha):
    gen = np.random.default_rng(31)
    truth = np.cumsum(np.cumsum(gen.standard_normal(shape), axis=-1), axis=-2) / 8.0
    mask = (gen.random(shape) < 0.3).astype(np.float32)
    p = (truth + 0.05 * gen.standard_normal(shape)).astype(np.float32)
    say("tikhonov_pcg", shape, order, levels, s, alpha)
    x, info = tikhonov_pcg(torch.from_numpy(p).cuda(), torch.from_numpy(mask).cuda(), ndim, order, levels, s, alpha,
                           iters=200, rtol=1e-6)
    x = x.cpu().numpy()
    assert info["iterations"] < 200 and bool((info["rel_residual"] <= 1e-6).all())
    xs = x.reshape((-1,) + shape[len(shape) - ndim:])
    ps = p.reshape(xs.shape)
    ms = mask.reshape(xs.shape)
    for b in range(xs.shape[0]):
        ref = oracle.tikhonov_solve(ps[b].astype(np.float64), ms[b].astype(np.float64), order, levels, s, alpha)
        err = rel_l2(xs[b], ref)
        assert err <= SOLVE_TOL, (b, err)


def test_tikhonov_pcg_deterministic_and_frozen_instances():
    """Two solves give the same bits (fixed-order reductions); an instance with an empty mask
    (M p = 0) stays at x = 0 with residual 0 while the others converge."""
    gen = np.random.default_rng(5)
    shape = (3, 64, 64)
    mask = (gen.random(shape) < 0.3).astype(np.float32)
    mask[1] = 0.0
    p = gen.standard_normal(shape).astype(np.float32)
    pt, mt = torch.from_numpy(p).cuda(), torch.from_numpy(mask).cuda()
    say("tikhonov_pcg determinism")
    x1, i1 = tikhonov_pcg(pt, mt, 2, 4, 4, 1.0, 0.1, iters=100, rtol=1e-6)
    x2, i2 = tikhonov_pcg(pt, mt, 2, 4, 4, 1.0, 0.1, iters=100, rtol=1e-6)
    assert torch.equal(x1, x2) and i1["iterations"] == i2["iterations"]
    assert float(x1[1].abs().max()) == 0.0 and float(i1["rel_residual"][1]) == 0.0
    assert bool((i1["rel_residual"] <= 1e-6).all())


def test_tikhonov_pcg_fused_steps_match_separate_kernels():
    """2-D grids whose operator ends in the vector-path synthesis run the mask term and the inner
    products inside the operator's last kernel; the separate-kernel path (ESWAVE_CG_FUSED=0) solves
    the same system: both agree with each other and with the FP64 oracle."""
    from tests.gpu_util import env
    gen = np.random.default_rng(8)
    shape = (2, 256, 384)
    truth = np.cumsum(np.cumsum(gen.standard_normal(shape), axis=-1), axis=-2) / 8.0
    mask = (gen.random(shape) < 0.3).astype(np.float32)
    p = (truth + 0.05 * gen.standard_normal(shape)).astype(np.float32)
    pt, mt = torch.from_numpy(p).cuda(), torch.from_numpy(mask).cuda()
    say("tikhonov_pcg fused vs separate")
    xf, inf_f = tikhonov_pcg(pt, mt, 2, 6, 5, 1.5, 0.05, iters=200, rtol=1e-6)
    with env(ESWAVE_CG_FUSED="0"):
        xs, inf_s = tikhonov_pcg(pt, mt, 2, 6, 5, 1.5, 0.05, iters=200, rtol=1e-6)
    assert bool((inf_f["rel_residual"] <= 1e-6).all()) and bool((inf_s["rel_residual"] <= 1e-6).all())
    xf, xs = xf.cpu().numpy(), xs.cpu().numpy()
    for b in range(shape[0]):
        ref = oracle.tikhonov_solve(p[b].astype(np.float64), mask[b].astype(np.float64), 6, 5, 1.5, 0.05)
        assert rel_l2(xf[b], ref) <= SOLVE_TOL
        assert rel_l2(xs[b], ref) <= SOLVE_TOL
        assert rel_l2(xf[b], xs[b]) <= SOLVE_TOL


# GMRES iterates: FP32 operator applications (~1e-6 relative) through 15 Arnoldi steps on systems
# with eigenvalues in about [alpha, 1 + alpha] (condition <= 11 here); 1e-4 covers both.
GMRES_TOL = 1e-4


@pytest.mark.parametrize("shape,ndim,order,levels,s,alpha", [((2, 64, 96), 2, 4, 4, 1.5, 0.1),
                                                             ((2, 16, 24, 32), 3, 2, 3, 1.0, 0.2),
                                                             ((1, 128, 128), 2, 8, 5, 1.5, 0.1)])
def test_tikhonov_gmres_iterates_match_oracle(shape, ndim, order, levels, s, alpha):
    """15 GMRES steps (the paper's count, Sec. 5) on (E_s^* K^* K + alpha I) x = E_s^* K^* p with a
    non-binary mask: the GPU's 15th iterate against the FP64 oracle's."""
    from paper_2507_02401_amd.solver import tikhonov_gmres
    gen = np.random.default_rng(17)
    truth = np.cumsum(gen.standard_normal(shape), axis=-1) / 4.0
    mask = gen.random(shape).astype(np.float32)
    p = (truth + 0.05 * gen.standard_normal(shape)).astype(np.float32)
    say("tikhonov_gmres 15 steps", shape, order, levels, s, alpha)
    x, info = tikhonov_gmres(torch.from_numpy(p).cuda(), torch.from_numpy(mask).cuda(), ndim, order, levels, s, alpha,
                             iters=15, restart=15, rtol=0.0)
    assert info["iterations"] == 15
    xs = x.cpu().numpy().reshape((-1,) + shape[len(shape) - ndim:])
    ps, ms = p.reshape(xs.shape), mask.reshape(xs.shape)
    for b in range(xs.shape[0]):
        ref = oracle.tikhonov_gmres(ps[b].astype(np.float64), ms[b].astype(np.float64), order, levels, s, alpha, 15)
        err = rel_l2(xs[b], ref)
        assert err <= GMRES_TOL, (b, err)


@pytest.mark.parametrize("restart", [30, 6])
def test_tikhonov_gmres_converges_to_the_solution(restart):
    """Restarted GMRES to a residual of 1e-6 reaches the FP64 solution (for a 0/1 mask the CG
    oracle's); the reported residual is the true one of the returned iterate; an instance with an
    empty mask stays at x = 0 with residual 0; two runs give the same bits."""
    from paper_2507_02401_amd.solver import tikhonov_gmres
    gen = np.random.default_rng(23)
    shape = (3, 96, 80)
    truth = np.cumsum(np.cumsum(gen.standard_normal(shape), axis=-1), axis=-2) / 8.0
    mask = (gen.random(shape) < 0.3).astype(np.float32)
    mask[1] = 0.0
    p = (truth + 0.05 * gen.standard_normal(shape)).astype(np.float32)
    pt, mt = torch.from_numpy(p).cuda(), torch.from_numpy(mask).cuda()
    say("tikhonov_gmres converge, restart", restart)
    x, info = tikhonov_gmres(pt, mt, 2, 4, 4, 1.5, 0.1, iters=600, restart=restart, rtol=1e-6)
    x2, info2 = tikhonov_gmres(pt, mt, 2, 4, 4, 1.5, 0.1, iters=600, restart=restart, rtol=1e-6)
    assert torch.equal(x, x2) and info["iterations"] == info2["iterations"]
    assert info["iterations"] < 600
    rel = info["rel_residual"]
    assert float(rel[1]) == 0.0 and float(x[1].abs().max()) == 0.0
    assert float(rel[0]) <= 1e-5 and float(rel[2]) <= 1e-5
    xs = x.cpu().numpy()
    for b in (0, 2):
        ref = oracle.tikhonov_solve(p[b].astype(np.float64), mask[b].astype(np.float64), 4, 4, 1.5, 0.1)
        assert rel_l2(xs[b], ref) <= SOLVE_TOL, b
