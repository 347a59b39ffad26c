"""Host-side checks of the C-ABI library: no device call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2507_02401_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "eswave.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("es_", "matern_"))))


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in _lib.SIGNATURES}
    assert set(names) == bound


@pytest.mark.parametrize("order", range(1, 9))
def test_host_filter_matches_oracle(lib, order):
    """The library derives dbN on its own (long-double Durand-Kerner); it must agree with the
    oracle's 60-digit mpmath derivation."""
    h = (ctypes.c_double * 16)()
    assert lib.es_filter(order, h) == _lib.ES_OK
    got = np.array(h[:2 * order])
    assert np.max(np.abs(got - oracle.daubechies_lowpass(order))) < 2e-16 * 8


def test_filter_rejects_bad_order(lib):
    h = (ctypes.c_double * 16)()
    assert lib.es_filter(0, h) == _lib.ES_EINVAL
    assert lib.es_filter(9, h) == _lib.ES_EINVAL
    assert lib.es_filter(3, None) == _lib.ES_EINVAL


@pytest.mark.parametrize("levels,s,tau", [(5, 1.0, 2.0), (6, 1.5, 1.0), (7, 1.5, 2.0), (3, -0.5, 2.0), (1, 2.0, 1.0)])
def test_level_weights_match_oracle(lib, levels, s, tau):
    w = (ctypes.c_float * (levels + 1))()
    assert lib.es_level_weights(levels, s, tau, w) == _lib.ES_OK
    ref = oracle.level_weights(levels, s, tau).astype(np.float32)
    assert np.array_equal(np.array(w[:levels], dtype=np.float32), ref)
    assert w[levels] == 1.0


def _ws(lib, shape, batch, order, levels, op):
    return lib.es_workspace_bytes(len(shape), _lib.shape_arg(shape), batch, order, levels, op)


def test_workspace_sizes(lib):
    # level arrays a_1..a_m, each rounded up to 64 floats
    def expect(shape, batch, levels):
        tot = 0
        for i in range(1, levels + 1):
            n = int(np.prod([v >> i for v in shape]))
            tot += (n + 63) // 64 * 64
        return tot * 4 * batch
    for shape, batch, levels in [((128, 128), 1, 5), ((1024, 1024), 64, 7), ((256, 256, 256), 1, 5), ((4096,), 3, 4)]:
        for op in range(4):
            identity = levels <= 1 if op >= 2 else levels == 0
            assert _ws(lib, shape, batch, 4, levels, op) == (0 if identity else expect(shape, batch, levels))
    assert _ws(lib, (16, 16), 1, 4, 1, _lib.OP_COV) == 0
    assert _ws(lib, (16, 16), 1, 4, 0, _lib.OP_ADJOINT) == 0
    assert _ws(lib, (12, 16), 1, 4, 3, _lib.OP_COV) == 0  # invalid geometry -> 0


FAKE_IN, FAKE_OUT, FAKE_WS = 0x100000, 0x900000, 0x2000000


def _call(lib, name="matern_cov_apply", ndim=2, shape=(64, 64), batch=1, order=4, levels=3, s=1.0,
          x=FAKE_IN, y=FAKE_OUT, ws=FAKE_WS, ws_bytes=1 << 30):
    return getattr(lib, name)(ndim, _lib.shape_arg(shape), batch, order, levels, s, x, y, ws, ws_bytes, None)


@pytest.mark.parametrize("kw,status", [
    (dict(ndim=0), _lib.ES_EINVAL),
    (dict(ndim=4, shape=(8, 8, 8, 8)), _lib.ES_EINVAL),
    (dict(order=0), _lib.ES_EINVAL),
    (dict(order=9), _lib.ES_EINVAL),
    (dict(levels=-1), _lib.ES_EINVAL),
    (dict(levels=31), _lib.ES_EINVAL),
    (dict(shape=(48, 64), levels=5), _lib.ES_EINVAL),
    (dict(shape=(0, 64)), _lib.ES_EINVAL),
    (dict(s=float("nan")), _lib.ES_EINVAL),
    (dict(s=float("inf")), _lib.ES_EINVAL),
    (dict(batch=-1), _lib.ES_EINVAL),
    (dict(x=0), _lib.ES_EINVAL),
    (dict(y=0), _lib.ES_EINVAL),
    (dict(x=FAKE_IN + 4), _lib.ES_EINVAL),
    (dict(y=FAKE_IN + 64), _lib.ES_EINVAL),
    (dict(ws=0), _lib.ES_EWORKSPACE),
    (dict(ws_bytes=16), _lib.ES_EWORKSPACE),
    (dict(ws=FAKE_WS + 8), _lib.ES_EINVAL),
    (dict(ws=FAKE_IN), _lib.ES_EINVAL),
    (dict(shape=(1 << 16, 1 << 16), levels=1), _lib.ES_EINVAL),
])
@pytest.mark.parametrize("name", ["es_adjoint", "es_apply", "matern_cov_apply", "matern_sample"])
def test_validation_before_any_device_call(lib, kw, status, name):
    assert _call(lib, name=name, **kw) == status
    assert len(lib.es_last_error()) > 0


def test_every_schedule_fits_the_coarse_kernels(lib):
    """Schedules for many geometries build (the host checks each coarse block against the LDS
    the coarse kernels hold, including the 3-D synthesis temporaries)."""
    sides = [8, 16, 32, 64, 128, 256, 512]
    for ndim in (1, 2, 3):
        for n in sides:
            shape = (n * (8 if ndim == 1 else 1),) * ndim if ndim > 1 else (n * n,)
            N = int(np.prod(shape))
            for levels in range(0, 8):
                if min(shape) % (1 << levels):
                    continue
                for order in (1, 4, 8):
                    for op in range(4):
                        r = lib.es_schedule_length(op, ndim, _lib.shape_arg(shape), 2, order, levels)
                        assert r >= 0, (op, shape, order, levels, lib.es_last_error())


def test_norm_workspace_and_validation(lib):
    shp = _lib.shape_arg((64, 96))
    assert lib.es_hs_norm_workspace_bytes(2, shp, 3, 4, 0) == 0  # identity: no workspace
    need = lib.es_hs_norm_workspace_bytes(2, shp, 3, 4, 3)
    # level arrays (a_1 .. a_3 of 3 instances) plus at least one partial sum per launch and instance
    assert need >= 3 * 4 * (32 * 48 + 16 * 24 + 8 * 12) + 3 * 8 * 2
    x, o, w = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 32)
    assert lib.es_hs_norm_sq(2, shp, 3, 4, 7, 1.0, x, o, w, need, None) == 1  # 64 not divisible by 2^7
    assert lib.es_hs_norm_sq(2, shp, 3, 4, 3, 1.0, ctypes.c_void_p((1 << 20) + 4), o, w, need, None) == 1  # misaligned
    assert lib.es_hs_norm_sq(2, shp, 3, 4, 3, 1.0, x, ctypes.c_void_p((1 << 30) + 2), w, need, None) == 1  # misaligned
    assert lib.es_hs_norm_sq(2, shp, 3, 4, 3, 1.0, x, o, w, need - 1, None) == 2  # workspace too small
    assert lib.es_hs_norm_sq(2, shp, 3, 4, 3, 1.0, x, o, None, 0, None) == 2
    assert lib.es_hs_norm_sq(2, shp, 0, 4, 3, 1.0, None, None, None, 0, None) == 0  # empty batch


def test_batch_zero_is_noop(lib):
    assert _call(lib, batch=0, x=0, y=0, ws=0, ws_bytes=0) == _lib.ES_OK


def test_status_strings(lib):
    for st in range(6):
        assert lib.es_status_string(st).startswith(b"ES_")
    assert b"unknown" in lib.es_status_string(77)


def test_plain_and_plan_validation(lib):
    shp = _lib.shape_arg((64, 64))
    assert lib.es_plain_apply_op(9, 2, shp, 1, 4, 3, 1.0, FAKE_IN, FAKE_OUT, FAKE_WS, 1 << 30, None) == _lib.ES_EINVAL
    p = ctypes.c_void_p()
    assert lib.es_plan_create(None, 3, 2, None, ctypes.byref(p)) == _lib.ES_EINVAL
    assert lib.es_plan_create(None, 0, 7, None, ctypes.byref(p)) == _lib.ES_EINVAL
    assert lib.es_plan_workspace_bytes(None) == 0
    lib.es_plan_destroy(None)


def test_noalloc_refuses_oversize_on_host(lib):
    """The allocation-free covariance refuses, before any device call, a geometry whose level
    arrays exceed the library's scratch (64 x 1024^2 db8, 7 levels: 89 MB > 64 MiB)."""
    shp = _lib.shape_arg((1024, 1024))
    need = lib.es_workspace_bytes(2, shp, 64, 8, 7, _lib.OP_COV)
    assert need > lib.es_noalloc_scratch_bytes() == 64 << 20
    assert lib.matern_cov_apply_noalloc(2, shp, 64, 8, 7, 1.5, 1 << 20, 1 << 30, None) == _lib.ES_EWORKSPACE
    assert b"scratch" in lib.es_last_error()


def test_tikhonov_pcg_validates_on_host(lib):
    """The solver entry point refuses bad arguments before any device call."""
    shp = _lib.shape_arg((64, 64))
    need = lib.es_tikhonov_pcg_workspace_bytes(2, shp, 2, 4, 3)
    assert need >= 4 * 2 * 64 * 64 * 4
    rel = (ctypes.c_float * 2)()
    its = ctypes.c_int32()
    P, M, X, WS = 1 << 20, 1 << 24, 1 << 28, 1 << 32
    def call(alpha=0.1, rtol=1e-6, max_iter=10, ws=WS, ws_bytes=need, x=X):
        return lib.es_tikhonov_pcg(2, shp, 2, 4, 3, 1.0, alpha, P, M, x, max_iter, rtol, 4, ctypes.byref(its), rel,
                                   ws, ws_bytes, None)
    assert call(alpha=0.0) == _lib.ES_EINVAL
    assert call(alpha=float("nan")) == _lib.ES_EINVAL
    assert call(rtol=-1.0) == _lib.ES_EINVAL
    assert call(max_iter=-1) == _lib.ES_EINVAL
    assert call(ws_bytes=need - 1) == _lib.ES_EWORKSPACE
    assert call(ws=WS + 16) == _lib.ES_EINVAL          # workspace alignment
    assert call(x=P + 64) == _lib.ES_EINVAL            # x overlaps p


def test_tikhonov_gmres_validates_on_host(lib):
    """The GMRES entry point refuses bad arguments before any device call; its workspace holds the
    basis (restart + 1 vectors) and three more vectors."""
    shp = _lib.shape_arg((64, 64))
    need = lib.es_tikhonov_gmres_workspace_bytes(2, shp, 2, 4, 3, 15)
    assert need >= (15 + 4) * 2 * 64 * 64 * 4
    assert lib.es_tikhonov_gmres_workspace_bytes(2, shp, 2, 4, 3, 30) > need
    assert lib.es_tikhonov_gmres_workspace_bytes(2, shp, 2, 4, 3, 0) == 0
    assert lib.es_tikhonov_gmres_workspace_bytes(2, shp, 2, 4, 3, 65) == 0
    rel = (ctypes.c_float * 2)()
    its = ctypes.c_int32()
    P, M, X, WS = 1 << 20, 1 << 24, 1 << 28, 1 << 32
    def call(alpha=0.1, rtol=1e-6, max_iter=10, restart=15, ws=WS, ws_bytes=need, x=X):
        return lib.es_tikhonov_gmres(2, shp, 2, 4, 3, 1.0, alpha, P, M, x, restart, max_iter, rtol, ctypes.byref(its),
                                     rel, ws, ws_bytes, None)
    assert call(alpha=0.0) == _lib.ES_EINVAL
    assert call(alpha=float("inf")) == _lib.ES_EINVAL
    assert call(rtol=-1.0) == _lib.ES_EINVAL
    assert call(max_iter=-1) == _lib.ES_EINVAL
    assert call(restart=0) == _lib.ES_EINVAL and b"restart" in lib.es_last_error()
    assert call(restart=65) == _lib.ES_EINVAL
    assert call(ws_bytes=need - 1) == _lib.ES_EWORKSPACE
    assert call(ws=WS + 16) == _lib.ES_EINVAL          # workspace alignment
    assert call(x=P + 64) == _lib.ES_EINVAL            # x overlaps p


def test_every_library_knob_is_created_before_device_use():
    """The test session creates every environment knob the library reads before the first device
    call (tests switch them by replacing values only)."""
    import re
    import conftest
    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2507_02401_amd", "csrc")
    names = set()
    for fn in os.listdir(csrc):
        if fn.endswith((".cpp", ".hip", ".h")):
            names |= set(re.findall(r'getenv\("(ESWAVE_[A-Z0-9_]+)"\)', open(os.path.join(csrc, fn)).read()))
    assert names and names <= set(conftest.KNOBS), sorted(names - set(conftest.KNOBS))
    assert all(k in os.environ for k in conftest.KNOBS)
