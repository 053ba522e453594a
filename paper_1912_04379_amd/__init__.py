"""mgemm: SGEMM (C <- alpha op(A) op(B) + beta C) for AMD MI355X (gfx950).

Python binding of libmgemm.so.  Every computation runs in the library's
HIP kernels; this package only passes device pointers, sizes and the
current HIP stream.  PyTorch supplies device memory and streams.

* ``sgemm``: the BLAS-style call on column-major device buffers.
* ``matmul``: row-major torch convenience (Y = X @ W) on the same call.
* ``linear``: Y = X @ W with a hand-written backward (autograd).
* ``GroupedPlan``: many independent products in one persistent launch,
  replayed from a HIP graph.
* ``MLP``: multilayer-perceptron training steps whose products (and the
  weight update, fused into them) run in the library.
* ``PackedB``: op(B) packed once (BF16x3 form) and reused by many products.
"""
from ._lib import (MgemmError, PREC_BF16X3, PREC_FP16_SCALED, PREC_FP32, PRECISIONS,
                   check, lib)
from .api import (clear_choices, config_count, config_info, default_config, matmul,
                  matmul_args, record_choice, sgemm, stream_handle, trim_workspace, tune_sgemm,
                  version)


def linear(X, W, precision="fp32"):
    """Y = X @ W with the hand-written backward (see autograd.py)."""
    from .autograd import linear as _linear
    return _linear(X, W, precision)


from .grouped import GroupedPlan, tune as tune_grouped  # noqa: E402
from .mlp import MLP, step_flops as mlp_step_flops  # noqa: E402
from .packed import PackedB  # noqa: E402

__all__ = ["GroupedPlan", "tune_grouped", "MLP", "mlp_step_flops", "PackedB", "MgemmError", "PREC_FP32", "PREC_BF16X3", "PREC_FP16_SCALED", "PRECISIONS",
           "sgemm", "matmul", "matmul_args", "linear", "config_count", "config_info",
           "default_config", "version", "lib", "check", "stream_handle", "tune_sgemm",
           "record_choice", "clear_choices", "trim_workspace"]
