"""Persistent plans (ESWAVE_PLAN_PERSISTENT=1): one launch per (dimensionality, taps) runs every
step of every instance from per-XCD work-item queues in device memory (matern_cov_apply /
matern_sample plans)."""
import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_2507_02401_amd as es
from paper_2507_02401_amd import _lib
from tests.gpu_util import ORACLE_OPS, OP_NAMES, TOL, env, rel_l2, say

pytestmark = pytest.mark.gpu
DEV = "cuda"

MIXED = [((128, 256), 2, 4, 0.5), ((64, 64, 64), 4, 3, 1.0), ((512,), 8, 5, 2.0), ((256, 128), 8, 4, 1.5),
         ((96, 160), 3, 3, 1.0), ((32, 32, 16), 6, 2, 0.5), ((1024,), 1, 7, 1.0), ((64, 64), 4, 1, 1.0),
         ((16, 16), 8, 4, 1.0), ((128, 128), 2, 0, 1.0), ((512, 512), 8, 6, 1.5), ((128, 128, 128), 2, 4, 2.0),
         ((1024, 256), 4, 5, 0.5), ((256, 256), 8, 5, 1.0)]


def _inputs(descs, seed):
    gen = np.random.default_rng(seed)
    xs = [gen.standard_normal(d[0]).astype(np.float32) for d in descs]
    return xs, [torch.from_numpy(x).to(DEV) for x in xs]


@pytest.mark.parametrize("op", [_lib.OP_COV, _lib.OP_SAMPLE], ids=["cov", "sample"])
def test_persistent_plan_vs_oracle_and_phase_merged(op):
    xs, ins = _inputs(MIXED, 20 + op)
    say("persistent plan", OP_NAMES[op])
    with env(ESWAVE_PLAN_PERSISTENT="1"):
        plan = es.RaggedPlan(MIXED, op)
    assert plan.persistent
    assert plan.num_launches == len({(len(d[0]), d[1]) for d in MIXED})
    eager = plan(ins, graph=False)
    plan.check_errors()
    for k, (shape, order, levels, s) in enumerate(MIXED):
        ref = ORACLE_OPS[op](xs[k].astype(np.float64), order, levels, s)
        assert rel_l2(eager[k].cpu().numpy(), ref) <= TOL, (k, shape)
    # the phase-merged plan with coarse blocks of the same size gives the same bits
    with env(ESWAVE_PLAN_PERSISTENT="0", ESWAVE_TAIL_MAX="2048"):
        merged = es.RaggedPlan(MIXED, op)
        assert not merged.persistent
        ref_bits = merged(ins, graph=False)
    torch.cuda.synchronize()
    for k in range(len(MIXED)):
        assert torch.equal(eager[k], ref_bits[k]), k
    merged.close()
    # graph replays, with eager work and synchronisation between them, equal the eager result
    outs = [torch.empty_like(x) for x in ins]
    for rep in range(3):
        plan(ins, outs, graph=True)
        torch.cuda.synchronize()
        for k in range(len(MIXED)):
            assert torch.equal(outs[k], eager[k]), (rep, k)
        _ = (ins[0] * 2).sum().item()
    plan.check_errors()
    # new pointers: the step tables are refreshed, the graph is reused
    ins2 = [x.clone() for x in ins]
    outs2 = plan(ins2, graph=True)
    torch.cuda.synchronize()
    for k in range(len(MIXED)):
        assert torch.equal(outs2[k], eager[k])
    plan.close()


def test_persistent_uniform_batch_equals_single_call():
    """Eight 1024^2 db8 images as a plan: the single call's bits (with the same coarse blocks)."""
    d = inputs.image_batch(count=8, side=1024)
    x = torch.from_numpy(d["x"]).to(DEV)
    descs = [((1024, 1024), d["order"], d["levels"], d["s"])] * 8
    say("persistent uniform 8 x 1024^2")
    with env(ESWAVE_PLAN_PERSISTENT="1"):
        plan = es.RaggedPlan(descs, _lib.OP_COV)
    assert plan.persistent and plan.num_launches == 1
    outs = plan([x[b] for b in range(8)])
    plan.check_errors()
    with env(ESWAVE_TAIL_MAX="2048"):
        single = es.matern_cov_apply(x, 2, d["order"], d["levels"], d["s"])
    torch.cuda.synchronize()
    for b in range(8):
        assert torch.equal(outs[b], single[b]), b
    ref = oracle.matern_cov_apply(d["x"][3].astype(np.float64), d["order"], d["levels"], d["s"])
    assert rel_l2(outs[3].cpu().numpy(), ref) <= TOL
    plan.close()


def test_persistent_forced_wait_give_up_reports_error():
    """The host forces every dependency wait to give up at once: the launches still run to their
    end, and the plan reports ES_EDEVICE."""
    xs, ins = _inputs(MIXED[:4], 5)
    say("persistent forced give-up")
    with env(ESWAVE_PERSIST_SPIN="-1", ESWAVE_PLAN_PERSISTENT="1"):
        plan = es.RaggedPlan(MIXED[:4], _lib.OP_COV)
    plan(ins, graph=False)
    with pytest.raises(_lib.EswaveError) as exc:
        plan.check_errors()
    assert exc.value.status == _lib.ES_EDEVICE
    plan.close()
    # a normal plan afterwards is unaffected
    with env(ESWAVE_PLAN_PERSISTENT="1"):
        plan = es.RaggedPlan(MIXED[:4], _lib.OP_COV)
    outs = plan(ins, graph=True)
    plan.check_errors()
    for k, (shape, order, levels, s) in enumerate(MIXED[:4]):
        ref = oracle.matern_cov_apply(xs[k].astype(np.float64), order, levels, s)
        assert rel_l2(outs[k].cpu().numpy(), ref) <= TOL
    plan.close()


def test_persistent_autotune_keeps_results():
    xs, ins = _inputs(MIXED, 31)
    say("persistent autotune")
    with env(ESWAVE_PLAN_PERSISTENT="1"):
        plan = es.RaggedPlan(MIXED, _lib.OP_COV)
    plan.autotune(ins, reps=1)
    coarse, lag, items = plan.config()
    assert coarse in (2048, 512) and lag > 0 and items > 0
    eager = plan(ins, graph=False)
    graph = plan(ins, graph=True)
    plan.check_errors()
    torch.cuda.synchronize()
    for k, (shape, order, levels, s) in enumerate(MIXED):
        assert torch.equal(graph[k], eager[k]), k
        ref = oracle.matern_cov_apply(xs[k].astype(np.float64), order, levels, s)
        assert rel_l2(eager[k].cpu().numpy(), ref) <= TOL, (k, shape)
    plan.close()


@pytest.mark.parametrize("lag,chunk", [("0", "1"), ("0.25", "8"), ("64", "2")])
def test_persistent_item_orders_agree(lag, chunk):
    """Instance after instance (lag 0), interleaved, and level after level, with one or several
    tiles per work item: the same bits."""
    xs, ins = _inputs(MIXED, 41)
    res = []
    for lg, ch in (("1", "4"), (lag, chunk)):
        with env(ESWAVE_PLAN_LAG=lg, ESWAVE_PLAN_CHUNK=ch, ESWAVE_PLAN_PERSISTENT="1"):
            plan = es.RaggedPlan(MIXED, _lib.OP_COV)
        say("persistent lag", lg, "chunk", ch)
        res.append(plan(ins, graph=False))
        plan.check_errors()
        plan.close()
    torch.cuda.synchronize()
    for k in range(len(MIXED)):
        assert torch.equal(res[0][k], res[1][k]), k
