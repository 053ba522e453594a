"""ctypes loader for libmgemm.so (the C ABI in include/mgemm.h).

Argument marshalling only.  If the library has not been built this module
raises on first use: there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgemm.so")

PREC_FP32 = 0
PREC_BF16X3 = 1
PREC_FP16_SCALED = 2
PRECISIONS = {"fp32": PREC_FP32, "bf16x3": PREC_BF16X3, "fp16s": PREC_FP16_SCALED}

ACT_NONE = 0
ACT_TANH = 1
ACT_TANH_GRAD = 2
ACTIVATIONS = {None: ACT_NONE, "none": ACT_NONE, "tanh": ACT_TANH, "tanh_grad": ACT_TANH_GRAD}

OK = 0
ERR_HIP = 100
ERR_NO_DEVICE = 101
ERR_ARCH = 102
ERR_ALLOC = 103
ERR_ALIAS = 105
ERR_UNSUPPORTED = 106
ERR_BAD_PLAN = 107
ERR_BAD_PROBLEM = 108

NOALLOC_SCRATCH_BYTES = 64 << 20   # MGEMM_NOALLOC_SCRATCH_BYTES

# The exported functions and their C signatures (kept in step with
# include/mgemm.h; the ABI test checks every declared name resolves).
_i64, _i32, _f32, _vp, _ch = (ctypes.c_int64, ctypes.c_int, ctypes.c_float,
                              ctypes.c_void_p, ctypes.c_char)


class Problem(ctypes.Structure):
    """struct mgemm_problem."""
    _fields_ = [("transA", _ch), ("transB", _ch),
                ("M", _i64), ("N", _i64), ("K", _i64),
                ("alpha", _f32), ("beta", _f32),
                ("A", _vp), ("lda", _i64),
                ("B", _vp), ("ldb", _i64),
                ("C", _vp), ("ldc", _i64)]


_SIGS = {
    "mgemm_sgemm": (_i32, [_ch, _ch, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32, _vp,
                           _i64, _vp]),
    "mgemm_sgemm_ex": (_i32, [_ch, _ch, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32,
                              _vp, _i64, _vp, _i32, _i32]),
    "mgemm_sgemm_act": (_i32, [_ch, _ch, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32,
                               _vp, _i64, _vp, _i32, _i32, _i32, _vp]),
    "mgemm_sgemm_ex_noalloc": (_i32, [_ch, _ch, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64,
                                      _f32, _vp, _i64, _vp, _i32, _i32]),
    "mgemm_config_count": (_i32, [_i32]),
    "mgemm_config_info": (_i32, [_i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                 ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "mgemm_default_config": (_i32, [_i32, _ch, _ch, _i64, _i64, _i64]),
    "mgemm_tune_sgemm": (_i32, [_ch, _ch, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32,
                                _vp, _i64, _vp, _i32, _i32, ctypes.POINTER(_i32),
                                ctypes.POINTER(ctypes.c_float)]),
    "mgemm_record_choice": (_i32, [_i32, _ch, _ch, _i64, _i64, _i64, _i32]),
    "mgemm_clear_choices": (_i32, []),
    "mgemm_trim_workspace": (_i32, []),
    "mgemm_save_choices": (_i32, [ctypes.c_char_p]),
    "mgemm_load_choices": (_i32, [ctypes.c_char_p, ctypes.POINTER(_i64)]),
    "mgemm_grouped_plan_create": (_i32, [ctypes.POINTER(Problem), _i64, _i32, ctypes.c_char_p,
                                         _vp, ctypes.POINTER(_vp), ctypes.POINTER(_i64)]),
    "mgemm_grouped_plan_create_ex": (_i32, [ctypes.POINTER(Problem), _i64, _i32,
                                            ctypes.POINTER(_i32), _vp, ctypes.POINTER(_vp),
                                            ctypes.POINTER(_i64), ctypes.POINTER(_i32)]),
    "mgemm_grouped_plan_launch": (_i32, [_vp, _vp]),
    "mgemm_grouped_plan_run": (_i32, [_vp, _vp]),
    "mgemm_grouped_plan_info": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "mgemm_grouped_plan_destroy": (_i32, [_vp]),
    "mgemm_grouped_bucket": (_i32, [_i64, _i64, _i64]),
    "mgemm_grouped_variant_count": (_i32, [_i32]),
    "mgemm_grouped_variant_info": (_i32, [_i32, _i32, ctypes.POINTER(_i32),
                                          ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "mgemm_grouped_tune": (_i32, [ctypes.POINTER(Problem), _i64, _i32, _vp, _i32,
                                  ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_float)]),
    "mgemm_pack_b": (_i32, [_ch, _i64, _i64, _vp, _i64, _i32, _vp, ctypes.POINTER(_vp)]),
    "mgemm_packed_b_info": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                   ctypes.POINTER(_i32), ctypes.POINTER(_i64)]),
    "mgemm_sgemm_packed_b": (_i32, [_ch, _i64, _f32, _vp, _i64, _vp, _f32, _vp, _i64, _vp]),
    "mgemm_packed_b_destroy": (_i32, [_vp]),
    "mgemm_status_string": (ctypes.c_char_p, [_i32]),
    "mgemm_last_error": (ctypes.c_char_p, []),
    "mgemm_version": (_i32, []),
}

_lib = None


class MgemmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("mgemm status %d: %s" % (status, message))
        self.status = status


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libmgemm.so is not built (%s); run __graft_entry__.build() or "
                "python paper_1912_04379_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    """Raise MgemmError for a non-zero status, with the library's text."""
    if status != OK:
        L = lib()
        detail = L.mgemm_last_error().decode() or L.mgemm_status_string(status).decode()
        raise MgemmError(status, detail)
    return status
