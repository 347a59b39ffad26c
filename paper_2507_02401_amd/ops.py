"""Torch-facing wrappers of the C ABI (argument marshalling only; every step runs in HIP).

Arrays are float32 CUDA (HIP) tensors of shape (*batch, *grid) where `grid` is the last
`ndim` dims.  Work is enqueued on torch's current stream of the tensor's device.
"""
import ctypes
import math

import torch

from ._lib import (OP_ADJOINT, OP_APPLY, OP_COV, OP_SAMPLE, EsDesc, check, load, shape_arg)

_NAMES = {OP_ADJOINT: "es_adjoint", OP_APPLY: "es_apply", OP_COV: "matern_cov_apply", OP_SAMPLE: "matern_sample"}


def _split(x, ndim):
    if not isinstance(x, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if x.dtype != torch.float32:
        raise TypeError(f"expected float32, got {x.dtype}")
    if x.device.type != "cuda":
        raise TypeError("expected a GPU tensor (the library has no CPU path)")
    if x.dim() < ndim:
        raise ValueError(f"tensor has {x.dim()} dims, need at least ndim={ndim}")
    grid = tuple(x.shape[x.dim() - ndim:])
    batch = math.prod(x.shape[:x.dim() - ndim])
    return grid, batch


def workspace_bytes(op, grid, batch, order, levels):
    lib = load()
    return int(lib.es_workspace_bytes(len(grid), shape_arg(grid), int(batch), int(order), int(levels), int(op)))


def _ws(need, device, workspace):
    if need == 0:
        return None
    if workspace is not None:
        if workspace.device != device or workspace.numel() * workspace.element_size() < need:
            raise ValueError(f"workspace must hold {need} bytes on {device}")
        return workspace
    return torch.empty(need, dtype=torch.uint8, device=device)


def apply_op(op, x, ndim, order, levels, s, out=None, workspace=None):
    grid, batch = _split(x, ndim)
    x = x.contiguous()
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of the input's shape")
    lib = load()
    shp = shape_arg(grid)
    need = int(lib.es_workspace_bytes(ndim, shp, batch, int(order), int(levels), op))
    ws = _ws(need, x.device, workspace)
    with torch.cuda.device(x.device):
        stream = torch.cuda.current_stream(x.device).cuda_stream
        st = getattr(lib, _NAMES[op])(ndim, shp, batch, int(order), int(levels), float(s), x.data_ptr(),
                                      out.data_ptr(), ws.data_ptr() if ws is not None else None, need, stream)
    check(st)
    return out


def es_adjoint(x, ndim, order, levels, s, out=None, workspace=None):
    """coeff = D_s W x (packed-pyramid coefficients, same shape as x)."""
    return apply_op(OP_ADJOINT, x, ndim, order, levels, s, out, workspace)


def es_apply(c, ndim, order, levels, s, out=None, workspace=None):
    """x = W^T D_s c (exact transpose of es_adjoint)."""
    return apply_op(OP_APPLY, c, ndim, order, levels, s, out, workspace)


def matern_cov_apply(x, ndim, order, levels, s, out=None, workspace=None):
    """y = W^T D_2s W x = E_s E_s^* x (the paper's pixel-space E_s^*)."""
    return apply_op(OP_COV, x, ndim, order, levels, s, out, workspace)


def matern_sample(xi, ndim, order, levels, s, out=None, workspace=None):
    """x = W^T D_s W xi (symmetric square root of the covariance)."""
    return apply_op(OP_SAMPLE, xi, ndim, order, levels, s, out, workspace)


def hs_norm_sq(x, ndim, order, levels, s, workspace=None):
    """||x||^2_{H^s} per instance (float32 tensor of the batch shape): sum of 2^{2sj} c^2 over
    the orthonormal wavelet coefficients c = W x, summed on the GPU (compensated FP32) without
    storing c."""
    grid, batch = _split(x, ndim)
    x = x.contiguous()
    lib = load()
    shp = shape_arg(grid)
    out = torch.empty(batch, dtype=torch.float32, device=x.device)
    need = int(lib.es_hs_norm_workspace_bytes(ndim, shp, batch, int(order), int(levels)))
    ws = _ws(need, x.device, workspace)
    with torch.cuda.device(x.device):
        stream = torch.cuda.current_stream(x.device).cuda_stream
        st = lib.es_hs_norm_sq(ndim, shp, batch, int(order), int(levels), float(s), x.data_ptr(), out.data_ptr(),
                               ws.data_ptr() if ws is not None else None, need, stream)
    check(st)
    return out.reshape(x.shape[:x.dim() - ndim])


def fft_workspace_bytes(grid, batch):
    lib = load()
    n = ctypes.c_size_t(0)
    check(lib.es_fft_workspace_bytes(len(grid), shape_arg(grid), int(batch), ctypes.byref(n)))
    return int(n.value)


def fft_cov_apply(x, ndim, s, period=1.0, out=None, workspace=None):
    """y = ifft(B fft(x)) over the last ndim axes, B = (1 + 4 pi^2 |k/period|^2)^(-s): the Fourier form
    of E_s^* (Sec. 4, Implementation).  out may be x itself (in place)."""
    grid, batch = _split(x, ndim)
    x = x.contiguous()
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of the input's shape")
    lib = load()
    shp = shape_arg(grid)
    with torch.cuda.device(x.device):
        need = fft_workspace_bytes(grid, batch)
        ws = _ws(need, x.device, workspace)
        stream = torch.cuda.current_stream(x.device).cuda_stream
        st = lib.es_fft_cov_apply(ndim, shp, batch, float(s), float(period), x.data_ptr(), out.data_ptr(),
                                  ws.data_ptr() if ws is not None else None, need, stream)
    check(st)
    return out


def sym_band_lengths(n, order, levels):
    """Band lengths l_1 .. l_levels of one axis of length n in the non-periodic transform."""
    lib = load()
    out = (ctypes.c_int64 * max(1, int(levels)))()
    check(lib.es_sym_band_lengths(int(n), int(order), int(levels), out))
    return [int(out[i]) for i in range(int(levels))]


def sym_cov_apply(x, ndim, order, levels, s, out=None, workspace=None):
    """y = W^{-1} D_2s W x with the non-periodic (half-point symmetric extension) DWT of Sec. 4;
    any side lengths.  Not symmetric (W^{-1} is not W^T): its transpose is sym_cov_apply_transpose."""
    return _sym(x, ndim, order, levels, s, out, workspace, False)


def sym_cov_apply_transpose(y, ndim, order, levels, s, out=None, workspace=None):
    """x = (W^{-1} D_2s W)^T y, the transpose of sym_cov_apply."""
    return _sym(y, ndim, order, levels, s, out, workspace, True)


def _sym(x, ndim, order, levels, s, out, workspace, transpose):
    grid, batch = _split(x, ndim)
    x = x.contiguous()
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of the input's shape")
    lib = load()
    shp = shape_arg(grid)
    size = lib.es_sym_transpose_workspace_bytes if transpose else lib.es_sym_workspace_bytes
    fn = lib.es_sym_cov_apply_transpose if transpose else lib.es_sym_cov_apply
    need = int(size(ndim, shp, batch, int(order), int(levels)))
    ws = _ws(need, x.device, workspace)
    with torch.cuda.device(x.device):
        stream = torch.cuda.current_stream(x.device).cuda_stream
        st = fn(ndim, shp, batch, int(order), int(levels), float(s), x.data_ptr(), out.data_ptr(),
                ws.data_ptr() if ws is not None else None, need, stream)
    check(st)
    return out


def plain_op(op, x, ndim, order, levels, s, out=None):
    """Reference variant: one launch per 1-D pass per level per instance."""
    grid, batch = _split(x, ndim)
    x = x.contiguous()
    out = torch.empty_like(x) if out is None else out
    lib = load()
    shp = shape_arg(grid)
    need = int(lib.es_workspace_bytes_plain(ndim, shp, batch, int(order), int(levels), op))
    ws = _ws(need, x.device, None)
    with torch.cuda.device(x.device):
        stream = torch.cuda.current_stream(x.device).cuda_stream
        st = lib.es_plain_apply_op(op, ndim, shp, batch, int(order), int(levels), float(s), x.data_ptr(),
                                   out.data_ptr(), ws.data_ptr() if ws is not None else None, need, stream)
    check(st)
    return out


def autotune(op, x, ndim, order, levels, s, out=None, reps=3):
    """Measure every tile variant of every launch for this geometry and batch; later calls with
    the same geometry use the fastest.  Returns the operator's result (computed with them)."""
    grid, batch = _split(x, ndim)
    x = x.contiguous()
    out = torch.empty_like(x) if out is None else out
    lib = load()
    shp = shape_arg(grid)
    need = int(lib.es_workspace_bytes(ndim, shp, batch, int(order), int(levels), int(op)))
    ws = _ws(need, x.device, None)
    with torch.cuda.device(x.device):
        stream = torch.cuda.current_stream(x.device).cuda_stream
        st = lib.es_autotune(int(op), ndim, shp, batch, int(order), int(levels), float(s), x.data_ptr(), out.data_ptr(),
                             ws.data_ptr() if ws is not None else None, need, int(reps), stream)
    check(st)
    return out


def matern_to_s(nu, d):
    """Sobolev index s = nu + d/2 of the Matern covariance Gamma_{nu, sqrt(2 nu)} (Prop. 3.2)."""
    return nu + d / 2.0


def matern_depth(nu, rho, spacing):
    """Depth m of the wavelet form of the Matern covariance Gamma_{nu, rho} on a grid of the given
    spacing (Cor. 4.3).  The unweighted (approximation) scale of the wavelet form sits at the
    correlation scale rho / sqrt(2 nu); detail level i (1 = finest, scale 2^i spacing) is weighted
    2^{-2s(m-i)}, so the coarsest level m is the one whose scale 2^m * spacing equals it.  The
    corollary requires rho / sqrt(2 nu) = 2^m on the level scale: a non-integer m raises
    ValueError.  The overall Matern constant is not applied (Remark 3.3)."""
    if not (nu > 0 and rho > 0 and spacing > 0):
        raise ValueError("nu, rho and spacing must be positive")
    m = math.log2(rho / (math.sqrt(2.0 * nu) * spacing))
    k = round(m)
    if abs(m - k) > 1e-9 or k < 0:
        raise ValueError(f"rho / (sqrt(2 nu) * spacing) = 2^{m:.6g} is not a non-negative power of two")
    return int(k)


def matern_parameters(nu, rho, d, spacing):
    """(s, levels) of matern_cov_apply / matern_sample for Gamma_{nu, rho} in d dimensions on a grid
    of the given spacing: s = nu + d/2 (Prop. 3.2), levels from matern_depth (Cor. 4.3)."""
    return matern_to_s(nu, d), matern_depth(nu, rho, spacing)


class RaggedPlan:
    """Many instances of different geometry in one captured launch sequence (es_plan_*).

    descs: list of (grid_shape, order, levels, s).  Call with lists of input and output
    tensors (one per instance, matching the descriptors).
    """

    def __init__(self, descs, op, device=None):
        self.lib = load()
        self.op = int(op)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        n = len(descs)
        arr = (EsDesc * max(1, n))()
        self.shapes = []
        for i, (shape, order, levels, s) in enumerate(descs):
            arr[i].ndim = len(shape)
            for k, v in enumerate(shape):
                arr[i].shape[k] = int(v)
            arr[i].order = int(order)
            arr[i].levels = int(levels)
            arr[i].s = float(s)
            self.shapes.append(tuple(int(v) for v in shape))
        self._p = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            check(self.lib.es_plan_create(arr, n, self.op, stream, ctypes.byref(self._p)))
        self.ws_bytes = int(self.lib.es_plan_workspace_bytes(self._p))
        self.workspace = torch.empty(max(1, self.ws_bytes), dtype=torch.uint8, device=self.device)
        self.num_launches = int(self.lib.es_plan_num_launches(self._p))
        self.persistent = bool(self.lib.es_plan_is_persistent(self._p))

    def _ptrs(self, inputs, outputs):
        n = len(inputs)
        ip = (ctypes.c_void_p * max(1, n))(*[x.data_ptr() for x in inputs])
        op = (ctypes.c_void_p * max(1, n))(*[y.data_ptr() for y in outputs])
        return ip, op

    def config(self):
        """(coarse limit, pipeline lag, work items per execution): -1 / -1.0 / 0 where they do not
        apply (a phase-merged plan on the default coarse limit)."""
        c, l, n = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
        check(self.lib.es_plan_config(self._p, ctypes.byref(c), ctypes.byref(l), ctypes.byref(n)))
        return int(c.value), float(l.value), int(n.value)

    def check_errors(self):
        """Synchronise and raise if a persistent launch's bounded dependency wait gave up."""
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            check(self.lib.es_plan_errors(self._p, stream))

    def autotune(self, inputs, outputs=None, reps=3):
        """Tune the plan on these buffers and keep the fastest (es_plan_autotune): coarse fusion depth
        and per-launch tile choices (phase-merged), or coarse fusion depth and pipeline lag
        (persistent)."""
        if outputs is None:
            outputs = [torch.empty_like(x) for x in inputs]
        ip, op = self._ptrs(inputs, outputs)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            check(self.lib.es_plan_autotune(self._p, ip, op, self.workspace.data_ptr(), self.ws_bytes, int(reps), stream))
        return outputs

    def __call__(self, inputs, outputs=None, graph=True):
        if len(inputs) != len(self.shapes):
            raise ValueError("one input per descriptor")
        if outputs is None:
            outputs = [torch.empty_like(x) for x in inputs]
        for x, y, shp in zip(inputs, outputs, self.shapes):
            if tuple(x.shape) != shp or tuple(y.shape) != shp:
                raise ValueError(f"tensor shape must be {shp}")
            if x.dtype != torch.float32 or not x.is_contiguous() or not y.is_contiguous():
                raise ValueError("contiguous float32 tensors required")
        ip, op = self._ptrs(inputs, outputs)
        fn = self.lib.es_plan_execute if graph else self.lib.es_plan_execute_eager
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            check(fn(self._p, ip, op, self.workspace.data_ptr(), self.ws_bytes, stream))
        return outputs

    def close(self):
        if getattr(self, "_p", None) is not None and self._p.value:
            self.lib.es_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
