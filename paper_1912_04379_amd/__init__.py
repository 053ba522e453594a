"""mgemm: SGEMM (C <- alpha op(A) op(B) + beta C) for AMD MI355X (gfx950).

Python binding of libmgemm.so.  Every computation runs in the library's
HIP kernels; this package only passes device pointers, sizes and the
current HIP stream.  PyTorch supplies device memory and streams.

* ``sgemm``: the BLAS-style call on column-major device buffers.
* ``matmul``: row-major torch convenience (Y = X @ W) on the same call.
* ``linear``: Y = X @ W with a hand-written backward (autograd).
* ``GroupedPlan``: many independent products in one persistent launch,
  replayed from a HIP graph.
"""
from ._lib import (MgemmError, PREC_BF16X3, PREC_FP16_SCALED, PREC_FP32, PRECISIONS,
                   check, lib)
from .api import (config_count, config_info, default_config, matmul, sgemm, stream_handle,
                  version)

__all__ = ["MgemmError", "PREC_FP32", "PREC_BF16X3", "PREC_FP16_SCALED", "PRECISIONS",
           "sgemm", "matmul", "config_count", "config_info", "default_config",
           "version", "lib", "check", "stream_handle"]
