"""The allocation-free covariance entry point (matern_cov_apply_noalloc) through the C ABI:
its results equal matern_cov_apply's (with a caller workspace) bit for bit, on two calls in a
row, the second with a smaller input; a geometry whose level arrays exceed the scratch is
refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2507_02401_amd import _lib
from tests.gpu_util import TOL, rel_l2, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _cov_with_workspace(lib, x, shape, order, levels, s, stream):
    batch = x.shape[0]
    shp = _lib.shape_arg(shape)
    need = lib.es_workspace_bytes(len(shape), shp, batch, order, levels, _lib.OP_COV)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=DEV)
    y = torch.empty_like(x)
    _lib.check(lib.matern_cov_apply(len(shape), shp, batch, order, levels, s, x.data_ptr(), y.data_ptr(),
                                    ws.data_ptr() if need else None, need, stream))
    return y


def _cov_noalloc(lib, x, shape, order, levels, s, stream):
    y = torch.empty_like(x)
    _lib.check(lib.matern_cov_apply_noalloc(len(shape), _lib.shape_arg(shape), x.shape[0], order, levels, s,
                                            x.data_ptr(), y.data_ptr(), stream))
    return y


def test_noalloc_matches_workspace_entry_point():
    lib = _lib.load()
    stream = torch.cuda.current_stream().cuda_stream
    cases = [((512, 512), 8, 6, 1.5, 6), ((256, 128), 4, 4, 1.0, 3)]  # second call: smaller input
    gen = np.random.default_rng(77)
    for shape, order, levels, s, batch in cases:
        say("noalloc", shape, order, levels, s, batch)
        xh = gen.standard_normal((batch,) + shape).astype(np.float32)
        x = torch.from_numpy(xh).to(DEV)
        need = lib.es_workspace_bytes(len(shape), _lib.shape_arg(shape), batch, order, levels, _lib.OP_COV)
        assert 0 < need <= lib.es_noalloc_scratch_bytes()
        y0 = _cov_noalloc(lib, x, shape, order, levels, s, stream)
        y1 = _cov_with_workspace(lib, x, shape, order, levels, s, stream)
        torch.cuda.synchronize()
        assert torch.equal(y0, y1)
        ref = oracle.matern_cov_apply(xh[0].astype(np.float64), order, levels, s)
        assert rel_l2(y0[0].cpu().numpy(), ref) <= TOL


def test_noalloc_refuses_oversize():
    lib = _lib.load()
    shape = (1024, 1024)
    need = lib.es_workspace_bytes(2, _lib.shape_arg(shape), 64, 8, 7, _lib.OP_COV)
    assert need > lib.es_noalloc_scratch_bytes()
    x = torch.zeros((2, 16), dtype=torch.float32, device=DEV)  # never touched: refused on the host
    st = lib.matern_cov_apply_noalloc(2, _lib.shape_arg(shape), 64, 8, 7, 1.5, x.data_ptr(), x[1].data_ptr(),
                                      None)
    assert st == _lib.ES_EWORKSPACE
    assert b"scratch" in lib.es_last_error()
