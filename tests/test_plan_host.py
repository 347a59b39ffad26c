"""Ragged-plan tables on the host (no GPU): frozen schedules, pointer rebasing and the footprint
check of every launch against the caller's buffers, through the C ABI's host-only plan entries."""
import ctypes

import numpy as np
import pytest

import inputs
from paper_2507_02401_amd import _lib
from tests.gpu_util import env

MIXED = [((128, 256), 2, 4, 0.5), ((64, 64, 64), 4, 3, 1.0), ((512,), 8, 5, 2.0), ((256, 128), 8, 4, 1.5),
         ((96, 160), 3, 3, 1.0), ((32, 32, 16), 6, 2, 0.5), ((1024,), 1, 7, 1.0), ((64, 64), 4, 1, 1.0),
         ((16, 16), 8, 4, 1.0), ((128, 128), 2, 0, 1.0)]


def _descs(descs):
    arr = (_lib.EsDesc * len(descs))()
    for k, (shape, order, levels, s) in enumerate(descs):
        arr[k].ndim = len(shape)
        arr[k].order = order
        for a in range(3):
            arr[k].shape[a] = shape[a] if a < len(shape) else 1
        arr[k].levels = levels
        arr[k].s = s
    return arr


def _layout(descs, base=1 << 32):
    """Addresses a caller could use: every array 256-byte aligned, inputs and outputs apart."""
    ins, outs, cur = [], [], base
    for shape, *_ in descs:
        nb = 4 * int(np.prod(shape))
        ins.append(cur)
        cur = (cur + nb + 255) // 256 * 256
        outs.append(cur)
        cur = (cur + nb + 255) // 256 * 256
    return ins, outs, (cur + 4095) // 256 * 256


class HostPlan:
    def __init__(self, lib, descs, op):
        self.lib, self.descs = lib, descs
        self.p = ctypes.c_void_p()
        _lib.check(lib.es_plan_create_host(_descs(descs), len(descs), op, ctypes.byref(self.p)))

    def fill(self, ins, outs, ws, ws_bytes=None):
        n = len(self.descs)
        if ws_bytes is None:
            ws_bytes = self.lib.es_plan_workspace_bytes(self.p)
        return self.lib.es_plan_fill_host(self.p, (ctypes.c_uint64 * n)(*ins), (ctypes.c_uint64 * n)(*outs),
                                          ws, ws_bytes)

    def work_groups(self):
        return self.lib.es_plan_work_groups(self.p)

    def close(self):
        self.lib.es_plan_destroy(self.p)


@pytest.mark.parametrize("op", range(4))
def test_mixed_plan_tables_fill(lib, op):
    plan = HostPlan(lib, MIXED, op)
    ins, outs, ws = _layout(MIXED)
    assert plan.fill(ins, outs, ws) == _lib.ES_OK, lib.es_last_error()
    wg = plan.work_groups()
    assert wg > 0
    # a second layout: same launches, same work-groups
    ins2, outs2, ws2 = _layout(MIXED, base=7 << 40)
    assert plan.fill(outs2, ins2, ws2) == _lib.ES_OK, lib.es_last_error()
    assert plan.work_groups() == wg
    plan.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_ragged_200_plan_tables(lib, seed):
    """The 200-instance ragged recipe (both draws): every table entry of every launch group stays
    inside the caller's buffers."""
    descs = list(inputs.ragged_descriptors(200, seed))
    plan = HostPlan(lib, descs, _lib.OP_COV)
    ins, outs, ws = _layout(descs)
    assert plan.fill(ins, outs, ws) == _lib.ES_OK, lib.es_last_error()
    assert plan.work_groups() > 0
    plan.close()


@pytest.mark.parametrize("knobs", [{"ESWAVE_TAIL_MAX": "0"}, {"ESWAVE_TAIL_MAX": "64"}, {"ESWAVE_STREAMED": "2"},
                                   {"ESWAVE_STREAMED": "0"}, {"ESWAVE_FORCE_VARIANT": "1"},
                                   {"ESWAVE_FORCE_VARIANT": "0"}, {"ESWAVE_FUSE_UP2": "1"},
                                   {"ESWAVE_NO_REVERSE": "1"}])
@pytest.mark.parametrize("op", range(4))
def test_knobs_changed_after_create_do_not_change_tables(lib, knobs, op):
    """A plan's launches are frozen at creation: knobs read by the planner at every call may change
    between creation and execution without changing what the tables hold."""
    plan = HostPlan(lib, MIXED, op)
    ins, outs, ws = _layout(MIXED)
    assert plan.fill(ins, outs, ws) == _lib.ES_OK
    wg = plan.work_groups()
    with env(**knobs):
        ins2, outs2, ws2 = _layout(MIXED, base=5 << 40)
        assert plan.fill(ins2, outs2, ws2) == _lib.ES_OK, lib.es_last_error()
        assert plan.work_groups() == wg
        # a plan created under the knob is valid too
        other = HostPlan(lib, MIXED, op)
        assert other.fill(ins2, outs2, ws2) == _lib.ES_OK, lib.es_last_error()
        other.close()
    plan.close()


def test_fill_refuses_bad_pointers(lib):
    plan = HostPlan(lib, MIXED, _lib.OP_COV)
    ins, outs, ws = _layout(MIXED)
    need = lib.es_plan_workspace_bytes(plan.p)
    bad = list(ins)
    bad[3] += 4  # not 16-byte aligned
    assert plan.fill(bad, outs, ws) == _lib.ES_EINVAL
    assert plan.fill(ins, outs, ws, need - 4) == _lib.ES_EWORKSPACE
    bad = list(ins)
    bad[0] = outs[0] + 256  # overlaps an output
    assert plan.fill(bad, outs, ws) == _lib.ES_EINVAL
    assert plan.fill(ins, outs, ins[1]) == _lib.ES_EINVAL  # workspace overlaps inputs
    assert plan.fill(ins, outs, ws) == _lib.ES_OK
    plan.close()


def test_host_plan_cannot_execute(lib):
    plan = HostPlan(lib, MIXED[:2], _lib.OP_COV)
    ins, outs, ws = _layout(MIXED[:2])
    n = 2
    st = lib.es_plan_execute(plan.p, (ctypes.c_void_p * n)(*ins), (ctypes.c_void_p * n)(*outs), ws,
                             lib.es_plan_workspace_bytes(plan.p), None)
    assert st != _lib.ES_OK
    plan.close()


@pytest.mark.parametrize("op", [_lib.OP_COV, _lib.OP_SAMPLE])
@pytest.mark.parametrize("descs", ["mixed", "ragged0", "ragged1"])
def test_persistent_plan_tables_fill(lib, op, descs):
    """Persistent plans (ESWAVE_PLAN_PERSISTENT=1): every step of every instance passes the
    footprint check against the instance's own buffers and its (twice as large) workspace slice."""
    d = MIXED if descs == "mixed" else list(inputs.ragged_descriptors(200, int(descs[-1])))
    with env(ESWAVE_PLAN_PERSISTENT="1"):
        plan = HostPlan(lib, d, op)
    assert lib.es_plan_is_persistent(plan.p) == 1
    merged = HostPlan(lib, d, op)
    assert lib.es_plan_is_persistent(merged.p) == 0
    # write-once level arrays: twice the phase-merged workspace
    assert lib.es_plan_workspace_bytes(plan.p) == 2 * lib.es_plan_workspace_bytes(merged.p)
    ins, outs, ws = _layout(d)
    assert plan.fill(ins, outs, ws) == _lib.ES_OK, lib.es_last_error()
    ins2, outs2, ws2 = _layout(d, base=9 << 40)
    assert plan.fill(outs2, ins2, ws2) == _lib.ES_OK, lib.es_last_error()
    assert merged.fill(ins, outs, ws) == _lib.ES_OK
    assert plan.work_groups() > 0 and merged.work_groups() > 0
    plan.close()
    merged.close()
