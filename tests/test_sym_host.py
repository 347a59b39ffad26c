"""Host-side checks of the non-periodic entry points (no device call): book-keeping band lengths
against the oracle, workspace sizes, and argument validation before any launch."""
import numpy as np
import pytest

from oracle import symdwt
from paper_2507_02401_amd import _lib

FAKE_IN, FAKE_OUT, FAKE_WS = 0x100000, 0x900000, 0x2000000


@pytest.mark.parametrize("order", range(1, 9))
@pytest.mark.parametrize("n", [1, 2, 3, 7, 14, 15, 16, 100, 1023, 1024, 5184])
def test_band_lengths_match_oracle(lib, order, n):
    levels = 9
    out = (_lib.ctypes.c_int64 * levels)()
    assert lib.es_sym_band_lengths(n, order, levels, out) == _lib.ES_OK
    assert list(out) == symdwt.sym_lengths(n, 2 * order, levels)


def test_band_lengths_fixed_point_and_errors(lib):
    """Lengths settle at L - 1, where floor((l + L - 1) / 2) = l."""
    out = (_lib.ctypes.c_int64 * 30)()
    assert lib.es_sym_band_lengths(1 << 20, 4, 30, out) == _lib.ES_OK
    assert list(out)[-1] == 7
    assert lib.es_sym_band_lengths(8, 4, 3, None) == _lib.ES_EINVAL
    assert lib.es_sym_band_lengths(0, 4, 3, out) == _lib.ES_EINVAL
    assert lib.es_sym_band_lengths(8, 9, 3, out) == _lib.ES_EINVAL
    assert lib.es_sym_band_lengths(8, 4, 31, out) == _lib.ES_EINVAL


def _ws(lib, shape, batch, order, levels):
    return lib.es_sym_workspace_bytes(len(shape), _lib.shape_arg(shape), batch, order, levels)


@pytest.mark.parametrize("shape,batch,order,levels", [
    ((1024, 1024), 64, 8, 7), ((37, 53), 3, 2, 4), ((9, 10, 11), 2, 4, 3), ((5,), 7, 8, 6), ((64,), 1, 1, 1),
    ((64,), 1, 3, 0)])
def test_workspace_is_the_level_arrays(lib, shape, batch, order, levels):
    """a_1 .. a_{m-1} of every instance, rows padded to a multiple of 4 floats, each level rounded
    up to 64 floats."""
    dims = [list(shape)]
    for _ in range(levels):
        dims.append([symdwt.sym_length(v, 2 * order) for v in dims[-1]])

    def stored(d):
        return int(np.prod(d[:-1])) * ((d[-1] + 3) // 4 * 4)
    tot = sum((batch * stored(dims[i]) + 63) // 64 * 64 for i in range(1, levels))
    assert _ws(lib, shape, batch, order, levels) == 4 * tot


def test_workspace_zero_for_invalid(lib):
    assert _ws(lib, (0, 4), 1, 4, 2) == 0
    assert _ws(lib, (8, 8), 0, 4, 2) == 0
    assert _ws(lib, (8, 8), 1, 9, 2) == 0


def _call(lib, ndim=2, shape=(37, 53), batch=1, order=4, levels=3, s=1.0, x=FAKE_IN, y=FAKE_OUT, ws=FAKE_WS,
          ws_bytes=1 << 30):
    return lib.es_sym_cov_apply(ndim, _lib.shape_arg(shape), batch, order, levels, s, x, y, ws, ws_bytes, None)


@pytest.mark.parametrize("kw,status", [
    (dict(ndim=0), _lib.ES_EINVAL),
    (dict(ndim=4, shape=(8, 8, 8, 8)), _lib.ES_EINVAL),
    (dict(order=0), _lib.ES_EINVAL),
    (dict(order=9), _lib.ES_EINVAL),
    (dict(levels=-1), _lib.ES_EINVAL),
    (dict(levels=31), _lib.ES_EINVAL),
    (dict(shape=(0, 64)), _lib.ES_EINVAL),
    (dict(shape=(1 << 31, 2)), _lib.ES_EINVAL),
    (dict(shape=(1 << 16, 1 << 16), levels=1), _lib.ES_EINVAL),
    (dict(s=float("nan")), _lib.ES_EINVAL),
    (dict(s=float("-inf")), _lib.ES_EINVAL),
    (dict(batch=-1), _lib.ES_EINVAL),
    (dict(x=0), _lib.ES_EINVAL),
    (dict(y=0), _lib.ES_EINVAL),
    (dict(x=FAKE_IN + 4), _lib.ES_EINVAL),
    (dict(y=FAKE_IN + 64), _lib.ES_EINVAL),
    (dict(ws=0), _lib.ES_EWORKSPACE),
    (dict(ws_bytes=16), _lib.ES_EWORKSPACE),
    (dict(ws=FAKE_WS + 16), _lib.ES_EINVAL),
    (dict(ws=FAKE_IN), _lib.ES_EINVAL),
])
def test_validation_before_any_device_call(lib, kw, status):
    assert _call(lib, **kw) == status
    assert len(lib.es_last_error()) > 0


def test_batch_zero_is_a_noop(lib):
    assert _call(lib, batch=0, x=0, y=0, ws=0) == _lib.ES_OK


def _shell_scratch_floats(shape, batch, order, levels):
    """Largest boundary-shell scratch over the up-levels of a 1-D or 2-D transposed operator: the
    rows of u that the axis-1 images read (all columns), then the shell columns of every row."""
    L, H = 2 * order, order
    dims = [tuple(shape)]
    for _ in range(levels):
        dims.append(tuple(symdwt.sym_length(v, L) for v in dims[-1]))
    dims = [((1,) + d) if len(shape) == 1 else d for d in dims]
    best = 0
    for j in range(1, levels):
        (n1, n2), (l1, l2) = dims[j - 1], dims[j]
        if n2 >= L - 1:
            e0, e1 = L - 2, max(L - 2, min(n2, 2 * n2 - 2 * l2))
        else:
            e0 = e1 = 0
        m2 = n2 - (e1 - e0)
        if len(shape) == 2:
            rt = min(l1, H - 1) if n1 >= L - 1 else l1
            rb = max(rt, min(l1, n1 // 2)) if n1 >= L - 1 else l1
            ny = rt + (l1 - rb)
        else:
            ny = 0
        a64 = lambda v: (v + 63) // 64 * 64
        best = max(best, a64(batch * ny * n2) + a64(batch * l1 * m2))
    return best


@pytest.mark.parametrize("shape,batch,order,levels", [((1024, 1024), 2, 8, 7), ((37, 53), 3, 2, 4), ((9, 10, 11), 2, 4, 3),
                                                      ((5,), 7, 8, 6), ((64,), 1, 1, 1)])
def test_transpose_workspace(lib, shape, batch, order, levels):
    """The level arrays; on 3-D grids then the extended synthesis of the finest level (every axis
    over -(L-2) .. 2 l_1 - 1, rows padded to a multiple of 4 floats), on 1-D and 2-D grids the
    boundary-shell scratch of the largest level."""
    fwd = lib.es_sym_workspace_bytes(len(shape), _lib.shape_arg(shape), batch, order, levels)
    tr = lib.es_sym_transpose_workspace_bytes(len(shape), _lib.shape_arg(shape), batch, order, levels)
    if levels < 2:
        assert tr == fwd == 0
        return
    if len(shape) < 3:
        assert tr == fwd + 4 * _shell_scratch_floats(shape, batch, order, levels)
        return
    ext = [2 * symdwt.sym_length(v, 2 * order) + 2 * order - 2 for v in shape]
    stored = int(np.prod(ext[:-1])) * ((ext[-1] + 3) // 4 * 4)
    assert tr == fwd + 4 * ((batch * stored + 63) // 64 * 64)


@pytest.mark.parametrize("kw,status", [(dict(order=0), _lib.ES_EINVAL), (dict(levels=31), _lib.ES_EINVAL),
                                       (dict(x=FAKE_IN + 4), _lib.ES_EINVAL), (dict(ws=0), _lib.ES_EWORKSPACE),
                                       (dict(y=FAKE_IN + 64), _lib.ES_EINVAL), (dict(s=float("nan")), _lib.ES_EINVAL)])
def test_transpose_validation_before_any_device_call(lib, kw, status):
    args = dict(ndim=2, shape=(37, 53), batch=1, order=4, levels=3, s=1.0, x=FAKE_IN, y=FAKE_OUT, ws=FAKE_WS,
                ws_bytes=1 << 30)
    args.update(kw)
    st = lib.es_sym_cov_apply_transpose(args["ndim"], _lib.shape_arg(args["shape"]), args["batch"], args["order"],
                                        args["levels"], args["s"], args["x"], args["y"], args["ws"],
                                        args["ws_bytes"], None)
    assert st == status


def _fold_div(d):
    """Host mirror of the fold kernel's divider: s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1."""
    s = 0
    while (1 << s) < d:
        s += 1
    return ((1 << 32) * ((1 << s) - d)) // d + 1, s


def test_fold_divider_exact_on_31_bit_numerators():
    # the kernel takes floor(x / d) as (mulhi(x, m) + x) >> s for 0 <= x < 2^31 and 1 <= d <= 2^31;
    # checked against integer division, with the multiples of d and their neighbours included
    rng = np.random.default_rng(7)
    divisors = list(range(1, 1200)) + [int(v) for v in rng.integers(1, 2 ** 31, 300)] + [2 ** 30, 2 ** 30 + 1,
                                                                                        2 ** 31 - 1, 2 ** 31]
    for d in divisors:
        m, s = _fold_div(d)
        assert 0 < m < 2 ** 32
        xs = [int(v) for v in rng.integers(0, 2 ** 31, 200)] + list(range(0, 2100)) + [2 ** 31 - 1]
        xs += [k * d + o for k in range(1, 40) for o in (-1, 0) if 0 <= k * d + o < 2 ** 31]
        for x in xs:
            assert (((x * m) >> 32) + x) >> s == x // d, (d, x)


def _fold_edge_split(no, nl, ext):
    """Host mirror of the 3-D fold's row split: interior [alo, ahi) of axes 0 and 1, edge rows."""
    alo, ahi = [0, 0], [0, 0]
    for a in range(2):
        n = no[a]
        lo, simple = min(ext, n), n >= ext + 1
        alo[a] = lo if simple else n
        ahi[a] = max(min(2 * n - 2 * nl[a], n), lo) if simple else n
    if no[2] < ext + 1:
        alo[0] = ahi[0] = no[0]
    ce1 = alo[1] + no[1] - ahi[1]
    erows = (alo[0] + no[0] - ahi[0]) * no[1] + (ahi[0] - alo[0]) * ce1
    return alo, ahi, ce1, erows


def _fold_edge_row(s, no, alo, ahi, ce1):
    """The fold's decode of edge-row index s into (j0, j1)."""
    c0rows = (alo[0] + no[0] - ahi[0]) * no[1]
    if s < c0rows:
        k, j1 = divmod(s, no[1])
        return (k if k < alo[0] else ahi[0] + (k - alo[0])), j1
    k0, k1 = divmod(s - c0rows, ce1)
    return alo[0] + k0, (k1 if k1 < alo[1] else ahi[1] + (k1 - alo[1]))


def _images(j, n, lo, hi):
    """Every extension position in [lo, hi] that reflects to j (p = j or -1 - j mod 2n), by brute force."""
    return sorted(p for p in range(lo, hi + 1) if p % (2 * n) in (j, (-1 - j) % (2 * n)))


@pytest.mark.parametrize("order", [1, 2, 4, 8, 10])
def test_fold_row_split_covers_every_row_once(lib, order):
    # edge rows decode onto exactly the rows with another image along axis 0 or 1 (or every row
    # when axis 2 is shorter than L - 1); interior rows have one image along axes 0 and 1 and at
    # most the two axis-2 images the interior part loads
    L = 2 * order
    ext = L - 2
    for no in [(1, 1, 1), (3, 2, 6), (5, 9, 3), (13, 17, 19), (20, 30, 40), (33, 4, 7), (8, 2, 1)]:
        nl = [int(symdwt.sym_length(n, L)) for n in no]
        alo, ahi, ce1, erows = _fold_edge_split(no, nl, ext)
        edge = [_fold_edge_row(s, no, alo, ahi, ce1) for s in range(erows)]
        assert all(0 <= a < no[0] and 0 <= b < no[1] for a, b in edge)
        assert len(set(edge)) == erows
        for j0 in range(no[0]):
            for j1 in range(no[1]):
                interior = alo[0] <= j0 < ahi[0] and alo[1] <= j1 < ahi[1]
                assert interior != ((j0, j1) in set(edge))
                if not interior:
                    continue
                assert _images(j0, no[0], -ext, 2 * nl[0] - 1) == [j0]
                assert _images(j1, no[1], -ext, 2 * nl[1] - 1) == [j1]
                for j2 in range(no[2]):
                    pa, pb = -1 - j2, 2 * no[2] - 1 - j2
                    want = sorted([j2] + [pa] * (pa >= -ext) + [pb] * (pb <= 2 * nl[2] - 1))
                    assert _images(j2, no[2], -ext, 2 * nl[2] - 1) == want
