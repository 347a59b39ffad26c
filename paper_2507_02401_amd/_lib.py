"""ctypes binding of libeswave.so: argument marshalling only.

Every computation runs in the HIP library; there is no fallback.  A missing library raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeswave.so")

ES_OK, ES_EINVAL, ES_EWORKSPACE, ES_EUNSUPPORTED, ES_EDEVICE, ES_ENOMEM = range(6)
OP_ADJOINT, OP_APPLY, OP_COV, OP_SAMPLE = range(4)

# (name, restype, argtypes) of every symbol declared in include/eswave.h
_i64p = ctypes.POINTER(ctypes.c_int64)
_fp = ctypes.c_void_p
_OP_ARGS = [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
            _fp, _fp, _fp, ctypes.c_size_t, _fp]


class EsDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("order", ctypes.c_int32), ("shape", ctypes.c_int64 * 3),
                ("levels", ctypes.c_int32), ("reserved", ctypes.c_int32), ("s", ctypes.c_double)]


SIGNATURES = [
    ("es_adjoint", ctypes.c_int, _OP_ARGS),
    ("es_apply", ctypes.c_int, _OP_ARGS),
    ("matern_cov_apply", ctypes.c_int, _OP_ARGS),
    ("matern_sample", ctypes.c_int, _OP_ARGS),
    ("matern_cov_apply_noalloc", ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_double, _fp, _fp, _fp]),
    ("es_noalloc_scratch_bytes", ctypes.c_size_t, []),
    ("es_workspace_bytes", ctypes.c_size_t, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    ("es_plain_apply_op", ctypes.c_int, [ctypes.c_int] + _OP_ARGS),
    ("es_workspace_bytes_plain", ctypes.c_size_t, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    ("es_hs_norm_sq", ctypes.c_int, _OP_ARGS),
    ("es_hs_norm_workspace_bytes", ctypes.c_size_t, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int]),
    ("es_tikhonov_pcg", ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, _fp, _fp, _fp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float), _fp,
                                       ctypes.c_size_t, _fp]),
    ("es_tikhonov_pcg_workspace_bytes", ctypes.c_size_t, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int]),
    ("es_tikhonov_gmres", ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_double, _fp, _fp, _fp, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_double, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float),
                                         _fp, ctypes.c_size_t, _fp]),
    ("es_tikhonov_gmres_workspace_bytes", ctypes.c_size_t, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int,
                                                             ctypes.c_int, ctypes.c_int32]),
    ("es_fft_cov_apply", ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                        _fp, _fp, _fp, ctypes.c_size_t, _fp]),
    ("es_fft_workspace_bytes", ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    ("es_fft_release_plans", ctypes.c_int, []),
    ("es_sym_cov_apply", ctypes.c_int, _OP_ARGS),
    ("es_sym_workspace_bytes", ctypes.c_size_t, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int]),
    ("es_sym_cov_apply_transpose", ctypes.c_int, _OP_ARGS),
    ("es_sym_transpose_workspace_bytes", ctypes.c_size_t, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int]),
    ("es_sym_band_lengths", ctypes.c_int, [ctypes.c_int64, ctypes.c_int, ctypes.c_int, _i64p]),
    ("es_plan_create", ctypes.c_int, [ctypes.POINTER(EsDesc), ctypes.c_int32, ctypes.c_int, _fp, ctypes.POINTER(ctypes.c_void_p)]),
    ("es_plan_execute", ctypes.c_int, [_fp, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), _fp, ctypes.c_size_t, _fp]),
    ("es_plan_execute_eager", ctypes.c_int, [_fp, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), _fp, ctypes.c_size_t, _fp]),
    ("es_plan_workspace_bytes", ctypes.c_size_t, [_fp]),
    ("es_plan_num_launches", ctypes.c_int32, [_fp]),
    ("es_plan_destroy", None, [_fp]),
    ("es_plan_create_host", ctypes.c_int, [ctypes.POINTER(EsDesc), ctypes.c_int32, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    ("es_plan_fill_host", ctypes.c_int, [_fp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.c_uint64, ctypes.c_size_t]),
    ("es_plan_work_groups", ctypes.c_int64, [_fp]),
    ("es_plan_is_persistent", ctypes.c_int32, [_fp]),
    ("es_plan_errors", ctypes.c_int, [_fp, _fp]),
    ("es_plan_autotune", ctypes.c_int, [_fp, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), _fp,
                                        ctypes.c_size_t, ctypes.c_int32, _fp]),
    ("es_plan_config", ctypes.c_int, [_fp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]),
    ("es_autotune", ctypes.c_int, [ctypes.c_int] + _OP_ARGS[:-1] + [ctypes.c_int32, _fp]),
    ("es_schedule_length", ctypes.c_int32, [ctypes.c_int, ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int]),
    ("es_schedule_describe", ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t, _i64p,
                                            ctypes.POINTER(ctypes.c_int32)]),
    ("es_schedule_run_step", ctypes.c_int, [ctypes.c_int] + _OP_ARGS[:-1] + [ctypes.c_int32, _fp]),
    ("es_filter", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    ("es_level_weights", ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_float)]),
    ("es_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("es_last_error", ctypes.c_char_p, []),
    ("es_version", ctypes.c_char_p, []),
]

_lib = None


class EswaveError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2507_02401_amd.build` "
                           "(or __graft_entry__.build()); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != ES_OK:
        lib = load()
        msg = lib.es_last_error().decode(errors="replace")
        raise EswaveError(status, f"{lib.es_status_string(status).decode()}: {msg}")


def shape_arg(shape):
    arr = (ctypes.c_int64 * max(1, len(shape)))(*[int(v) for v in shape])
    return arr
