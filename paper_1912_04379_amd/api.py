"""BLAS-style and torch-style entry points (argument marshalling only)."""
import ctypes

from ._lib import ACTIVATIONS, PRECISIONS, check, lib


def stream_handle(stream=None):
    """hipStream_t of a torch stream (None: torch's current stream, read
    through torch's raw-stream query where it has one: constructing a Stream
    object costs more than the rest of a small call's host work)."""
    if isinstance(stream, int):
        return stream
    import torch
    if stream is None:
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:
            return raw(torch.cuda.current_device())
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _prec(precision):
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _check_tensor(t, name):
    if t is None or isinstance(t, int):
        return
    import torch
    if t.dtype != torch.float32:
        raise TypeError("%s must be float32, got %s" % (name, t.dtype))
    if not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)


def _check_extent(t, name, rows, cols, ld):
    """The referenced part of a rows x cols column-major array at leading
    dimension ld, starting at a tensor argument's data_ptr(), must lie in
    the tensor's storage, so that no kernel reads or writes past it (views
    such as W.t() are fine; raw addresses are the caller's own)."""
    if t is None or isinstance(t, int) or rows <= 0 or cols <= 0 or ld < rows:
        return          # nothing referenced, or the library rejects ld
    need = 4 * ((cols - 1) * ld + rows)
    if need <= 4 * t.numel() and t.is_contiguous():
        return          # within the tensor's own elements (the common case, no storage query)
    storage = t.untyped_storage()
    lo, hi = storage.data_ptr(), storage.data_ptr() + storage.nbytes()
    if t.data_ptr() < lo or t.data_ptr() + need > hi:
        raise ValueError("%s: a %d x %d array at ld %d needs %d bytes from data_ptr(); the "
                         "tensor's storage has %d" % (name, rows, cols, ld, need,
                                                     hi - t.data_ptr()))


def check_operands(transA, transB, M, N, K, alpha, A, lda, B, ldb, C, ldc):
    """Dtype, device and extent checks of tensor arguments."""
    for t, n in ((A, "A"), (B, "B"), (C, "C")):
        _check_tensor(t, n)
    ta, tb = transA in "TtCc", transB in "TtCc"
    if alpha != 0 and K > 0:
        _check_extent(A, "A", K if ta else M, M if ta else K, lda)
        _check_extent(B, "B", N if tb else K, K if tb else N, ldb)
    _check_extent(C, "C", M, N, ldc)


def sgemm(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, *,
          precision="fp32", config=-1, stream=None, activation=None, aux=None):
    """C <- act(alpha op(A) op(B) + beta C) on column-major device buffers.

    A, B, C are float32 device tensors (read as flat column-major arrays
    from data_ptr(); the part the call references must lie in the tensor's
    storage, else ValueError) or raw device addresses.  activation: None,
    "tanh" or "tanh_grad" (C <- v * (1 - aux^2), aux M x N at ldc).  Raises
    MgemmError on any non-zero status.
    """
    check_operands(transA, transB, M, N, K, alpha, A, lda, B, ldb, C, ldc)
    p = _prec(precision)
    s = stream_handle(stream)
    L = lib()
    act = ACTIVATIONS[activation] if not isinstance(activation, int) else activation
    if act != 0:
        if aux is not None:
            _check_tensor(aux, "aux")
            _check_extent(aux, "aux", M, N, ldc)
        st = L.mgemm_sgemm_act(transA.encode(), transB.encode(), M, N, K, alpha, _ptr(A), lda,
                               _ptr(B), ldb, beta, _ptr(C), ldc, s, p, config, act, _ptr(aux))
    elif p == 0 and config == -1:
        st = L.mgemm_sgemm(transA.encode(), transB.encode(), M, N, K, alpha, _ptr(A), lda,
                           _ptr(B), ldb, beta, _ptr(C), ldc, s)
    else:
        st = L.mgemm_sgemm_ex(transA.encode(), transB.encode(), M, N, K, alpha, _ptr(A), lda,
                              _ptr(B), ldb, beta, _ptr(C), ldc, s, p, config)
    return check(st)


def matmul_args(x_shape, x_strides, w_shape, w_strides):
    """Column-major SGEMM arguments for Y = X @ W with a row-major (b x o) Y.

    Row-major Y is the column-major array Y^T (o x b, ld o), and
    Y^T = W^T X^T: op(A) = W^T comes from W's storage, op(B) = X^T from X's.
    Returns (transA, transB, M, N, K, lda, ldb, ldc).  Pure host logic.
    """
    b, i = x_shape
    i2, o = w_shape
    if i != i2:
        raise ValueError("inner dimensions differ: %d vs %d" % (i, i2))
    tw, ldw = _view(w_shape, w_strides)
    tx, ldx = _view(x_shape, x_strides)
    return tw, tx, o, b, i, ldw, ldx, max(1, o)


def _view(shape, strides):
    """(trans, ld) such that op(stored array) = T^T for a 2-D tensor T.

    A row-major T (stride (ld, 1)) is stored column-major as T^T: op 'N'.
    A column-major T (stride (1, ld)), e.g. a transposed view, is stored as
    T itself: op 'T'.
    """
    r, c = shape
    s0, s1 = strides
    if s1 == 1 and (s0 >= max(1, c) or r <= 1):
        return "N", max(1, s0, c)
    if s0 == 1 and (s1 >= max(1, r) or c <= 1):
        return "T", max(1, s1, r)
    raise ValueError("tensor must have unit stride in one dimension")


def colmajor_view(T):
    """(trans, ld) of a 2-D tensor entering a column-major product as T^T."""
    return _view(tuple(T.shape), tuple(T.stride()))


def matmul(X, W, *, alpha=1.0, beta=0.0, precision="fp32", config=-1, out=None, stream=None,
           activation=None, aux=None):
    """Y = act(alpha X @ W + beta Y) for 2-D float32 device tensors; Y is a
    new (or the given contiguous) row-major (b x o) tensor.  beta != 0 needs
    ``out``, whose values it scales.  activation: None, "tanh", or
    "tanh_grad" with ``aux`` a contiguous (b x o) tensor (Y = v * (1 -
    aux^2)).  One library call."""
    import torch
    ta, tb, M, N, K, lda, ldb, ldc = matmul_args(tuple(X.shape), tuple(X.stride()),
                                                 tuple(W.shape), tuple(W.stride()))
    b, o = X.shape[0], W.shape[1]
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        out = torch.empty((b, o), dtype=torch.float32, device=X.device)
    elif tuple(out.shape) != (b, o) or (b > 1 and o > 0 and out.stride() != (o, 1)):
        raise ValueError("out must be a contiguous (b x o) tensor")
    if aux is not None and (tuple(aux.shape) != (b, o) or (b > 1 and o > 0 and
                                                          aux.stride() != (o, 1))):
        raise ValueError("aux must be a contiguous (b x o) tensor")
    sgemm(ta, tb, M, N, K, alpha, W, lda, X, ldb, beta, out, ldc,
          precision=precision, config=config, stream=stream, activation=activation, aux=aux)
    return out


def config_count(precision="fp32"):
    return lib().mgemm_config_count(_prec(precision))


def config_info(precision, config):
    v = [ctypes.c_int() for _ in range(4)]
    check(lib().mgemm_config_info(_prec(precision), config, *[ctypes.byref(x) for x in v]))
    return dict(bm=v[0].value, bn=v[1].value, bk=v[2].value, threads=v[3].value)


def default_config(precision, transA, transB, M, N, K):
    return lib().mgemm_default_config(_prec(precision), transA.encode(), transB.encode(),
                                      M, N, K)


def tune_sgemm(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, *,
               precision="fp32", reps=3, stream=None):
    """Time every tile configuration for this product (C is overwritten) and
    record the fastest as the library's choice for it.  Returns
    (config, milliseconds); config is -1 when the library's own path for an
    FP32 product (the split at its ragged edges, or the thin path for at most
    8 rows or columns of C) stays the choice (nothing recorded)."""
    check_operands(transA, transB, M, N, K, alpha, A, lda, B, ldb, C, ldc)
    cfg = ctypes.c_int(-1)
    ms = ctypes.c_float(0.0)
    check(lib().mgemm_tune_sgemm(transA.encode(), transB.encode(), M, N, K, alpha, _ptr(A), lda,
                                 _ptr(B), ldb, beta, _ptr(C), ldc, stream_handle(stream),
                                 _prec(precision), reps, ctypes.byref(cfg), ctypes.byref(ms)))
    return cfg.value, ms.value


def record_choice(precision, transA, transB, M, N, K, config):
    """Make `config` the choice for this exact product (no timing)."""
    check(lib().mgemm_record_choice(_prec(precision), transA.encode(), transB.encode(), M, N,
                                    K, config))


def clear_choices():
    check(lib().mgemm_clear_choices())


def version():
    return lib().mgemm_version()


def trim_workspace():
    """Return the memory the library's workspace pools keep to the device."""
    check(lib().mgemm_trim_workspace())
