"""Pre-packed B: argument and handle errors, raised before any HIP call."""
import ctypes

import pytest

import paper_1912_04379_amd as mg
from paper_1912_04379_amd import _lib

L = None


def lib():
    global L
    if L is None:
        L = mg.lib()
    return L


def pack(transB="N", K=10, N=10, B=0x1000, ldb=10, prec=_lib.PREC_BF16X3, out=True):
    h = ctypes.c_void_p()
    return lib().mgemm_pack_b(transB.encode(), K, N, B, ldb, prec, None,
                              ctypes.byref(h) if out else None), h


@pytest.mark.parametrize("args,status", [
    (dict(transB="X"), -2), (dict(N=-1), -4), (dict(K=-1), -5), (dict(B=None), -9),
    (dict(ldb=9), -10), (dict(transB="T", N=20, ldb=19), -10),
    (dict(prec=7), _lib.ERR_UNSUPPORTED),
    (dict(prec=_lib.PREC_FP32, ldb=9), -10), (dict(prec=_lib.PREC_FP32, transB="X"), -2),
    (dict(prec=_lib.PREC_FP32, K=2 ** 40, N=2 ** 40, ldb=2 ** 40), _lib.ERR_UNSUPPORTED),
    (dict(out=False), _lib.ERR_UNSUPPORTED)])
def test_pack_b_rejects_bad_arguments(args, status):
    st, h = pack(**args)
    assert st == status
    assert not h.value


def test_calls_on_a_null_handle_are_rejected():
    assert lib().mgemm_sgemm_packed_b(b"N", 4, 1.0, 0x1000, 4, None, 0.0, 0x2000, 4,
                                      None) == _lib.ERR_BAD_PLAN
    assert lib().mgemm_packed_b_destroy(None) == _lib.ERR_BAD_PLAN
    assert lib().mgemm_packed_b_info(None, None, None, None, None) == _lib.ERR_BAD_PLAN


def test_unknown_handle_is_rejected():
    fake = ctypes.c_void_p(0x12345678)
    assert lib().mgemm_sgemm_packed_b(b"N", 4, 1.0, 0x1000, 4, fake, 0.0, 0x2000, 4,
                                      None) == _lib.ERR_BAD_PLAN
    assert lib().mgemm_packed_b_destroy(fake) == _lib.ERR_BAD_PLAN
