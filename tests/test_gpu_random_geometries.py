"""GPU: fixed-seed random geometries against the FP64 oracle — the periodic operators, the
non-periodic operator and its transpose, and ragged plans (graph replay equal to eager execution).
Each draw covers 1-D to 3-D, every order 1-8, several depths and batch sizes, and sides that are
not multiples of 4 where the operator allows them."""
import numpy as np
import pytest
import torch

import oracle
import paper_2507_02401_amd as es
from oracle import symdwt
from tests.gpu_util import ORACLE_OPS, TOL, rel_l2, say

pytestmark = pytest.mark.gpu
DEV = "cuda"
OPS = [es.es_adjoint, es.es_apply, es.matern_cov_apply, es.matern_sample]


def _periodic_shape(rng, D, levels, cap1, cap2, cap3):
    u = 2 ** levels
    if D == 1:
        return (u * int(rng.integers(1, cap1)),)
    if D == 2:
        return tuple(u * int(v) for v in rng.integers(1, max(2, cap2 // u), 2))
    return tuple(u * int(v) for v in rng.integers(1, max(2, cap3 // u), 3))


def test_random_periodic_geometries():
    rng = np.random.default_rng(2024)
    say("random periodic geometries")
    for _ in range(300):
        D, levels, order = int(rng.integers(1, 4)), int(rng.integers(1, 6)), int(rng.integers(1, 9))
        shape = _periodic_shape(rng, D, levels, 200, 200, 40)
        batch, s, op = int(rng.integers(1, 4)), float(rng.choice([-0.5, 0.5, 1.0, 1.5, 2.0])), int(rng.integers(0, 4))
        x = rng.standard_normal((batch,) + shape).astype(np.float32)
        y = OPS[op](torch.from_numpy(x).to(DEV), D, order, levels, s).cpu().numpy()
        for b in range(batch):
            err = rel_l2(y[b], ORACLE_OPS[op](x[b].astype(np.float64), order, levels, s))
            assert err <= TOL, (op, shape, batch, order, levels, s, b, err)


def test_random_non_periodic_geometries():
    rng = np.random.default_rng(2025)
    say("random non-periodic geometries")
    for _ in range(150):
        D = int(rng.integers(1, 4))
        shape = (tuple(int(v) for v in rng.integers(1, 40, 3)) if D == 3 else
                 tuple(int(v) for v in rng.integers(1, 160, 2)) if D == 2 else (int(rng.integers(1, 2500)),))
        order, levels, batch = int(rng.integers(1, 9)), int(rng.integers(1, 6)), int(rng.integers(1, 4))
        s = float(rng.choice([-0.5, 0.75, 1.0, 1.5, 2.0]))
        x = rng.standard_normal((batch,) + shape).astype(np.float32)
        xt = torch.from_numpy(x).to(DEV)
        yf = es.sym_cov_apply(xt, D, order, levels, s).cpu().numpy()
        yt = es.sym_cov_apply_transpose(xt, D, order, levels, s).cpu().numpy()
        for b in range(batch):
            x64 = x[b].astype(np.float64)
            assert rel_l2(yf[b], symdwt.sym_cov_apply(x64, order, levels, s)) <= TOL, (shape, batch, order, levels, s)
            assert rel_l2(yt[b], symdwt.sym_cov_apply_transpose(x64, order, levels, s)) <= TOL, (shape, batch, order,
                                                                                                  levels, s)


def test_random_ragged_plans():
    rng = np.random.default_rng(2026)
    say("random ragged plans")
    for _ in range(40):
        descs = []
        for _ in range(int(rng.integers(2, 13))):
            D, levels, order = int(rng.integers(1, 4)), int(rng.integers(0, 5)), int(rng.integers(1, 9))
            descs.append((_periodic_shape(rng, D, levels, 100, 120, 32), order, levels,
                          float(rng.choice([0.5, 1.0, 1.5, 2.0]))))
        op = int(rng.integers(0, 4))
        plan = es.RaggedPlan(descs, op)
        xs = [rng.standard_normal(d[0]).astype(np.float32) for d in descs]
        ins = [torch.from_numpy(x).to(DEV) for x in xs]
        eager = [y.cpu().numpy() for y in plan(ins, graph=False)]
        outs = plan(ins, graph=True)
        torch.cuda.synchronize()
        for k, (shape, order, levels, s) in enumerate(descs):
            assert np.array_equal(outs[k].cpu().numpy(), eager[k]), (op, descs[k])
            assert rel_l2(eager[k], ORACLE_OPS[op](xs[k].astype(np.float64), order, levels, s)) <= TOL, (op, descs[k])
        plan.close()
