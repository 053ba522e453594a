"""Pre-packed op(B): packed once by the library, reused by many products.

Argument marshalling only: the packing and the products run in libmgemm
(``mgemm_pack_b``, ``mgemm_sgemm_packed_b``; BF16x3, scaled FP16, and FP32 with
op(B) transposed once into the k-contiguous layout).
"""
import ctypes

from ._lib import check, lib, MgemmError, ERR_BAD_PLAN
from .api import _prec, _ptr, check_operands, stream_handle


class PackedB:
    """op(B) (K x N) of a column-major device buffer B at ldb, packed on the
    current (or given) stream.  ``close()`` frees the device copy."""

    def __init__(self, transB, K, N, B, ldb, *, precision="bf16x3", stream=None):
        # The extent check of B uses the SGEMM operand rules (M = 1 stands
        # in for the unused A and C).
        check_operands("N", transB, 1, N, K, 1.0, None, 1, B, ldb, None, 1)
        h = ctypes.c_void_p()
        check(lib().mgemm_pack_b(transB.encode(), K, N, _ptr(B), ldb, _prec(precision),
                                 stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.K, self.N, self.precision = K, N, precision

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise MgemmError(ERR_BAD_PLAN, "packed B is closed")
        return self._h

    def info(self):
        K, N, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        p = ctypes.c_int()
        check(lib().mgemm_packed_b_info(self.handle, ctypes.byref(K), ctypes.byref(N),
                                        ctypes.byref(p), ctypes.byref(b)))
        return dict(K=K.value, N=N.value, precision=p.value, bytes=b.value)

    def sgemm(self, transA, M, alpha, A, lda, beta, C, ldc, *, stream=None):
        """C <- alpha op(A) op(B) + beta C with this op(B)."""
        check_operands(transA, "N", M, self.N, self.K, alpha, A, lda, None, max(1, self.K), C,
                       ldc)
        check(lib().mgemm_sgemm_packed_b(transA.encode(), M, alpha, _ptr(A), lda, self.handle,
                                         beta, _ptr(C), ldc, stream_handle(stream)))

    def close(self):
        if self._h is not None and self._h.value:
            check(lib().mgemm_packed_b_destroy(self._h))
        self._h = None

    def __del__(self):
        # A handle left open frees its device copy when collected (the
        # library may already be unloaded at interpreter exit).
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
