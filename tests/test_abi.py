"""The C ABI without a GPU: every declared symbol is exported, arguments are
checked in BLAS order before any HIP call, quick returns launch nothing."""
import ctypes
import os
import random
import re

import pytest

import paper_1912_04379_amd as mg
from paper_1912_04379_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgemm.h")

# Fake device addresses: validation and quick returns never dereference them.
FA, FB, FC = 0x10000000, 0x20000000, 0x30000000


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgemm_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 14
    L = mg.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib._SIGS), "binding and header disagree"


def test_version_and_status_strings():
    assert mg.version() == 100
    L = mg.lib()
    assert L.mgemm_status_string(0) == b"success"
    assert b"lda" in L.mgemm_status_string(-8)
    assert L.mgemm_status_string(_lib.ERR_ARCH) == b"device is not gfx950"


def call(transA="N", transB="N", M=4, N=4, K=4, alpha=1.0, A=FA, lda=4, B=FB, ldb=4,
         beta=0.0, C=FC, ldc=4, precision=0, config=-1):
    return mg.lib().mgemm_sgemm_ex(transA.encode(), transB.encode(), M, N, K, alpha, A, lda,
                                   B, ldb, beta, C, ldc, None, precision, config)


@pytest.mark.parametrize("kw,code", [
    (dict(transA="X"), -1),
    (dict(transB="q"), -2),
    (dict(M=-1), -3),
    (dict(N=-1), -4),
    (dict(K=-1), -5),
    (dict(A=None), -7),
    (dict(lda=3), -8),
    (dict(B=None), -9),
    (dict(ldb=3), -10),
    (dict(C=None), -12),
    (dict(ldc=3), -13),
    (dict(transA="T", lda=3, K=4), -8),          # stored rows of A^T are K
    (dict(transB="T", ldb=3, N=4), -10),         # stored rows of B^T are N
    (dict(transA="X", M=-1, ldc=0), -1),         # first bad argument wins
    (dict(M=-1, lda=0), -3),
])
def test_argument_codes(kw, code):
    assert call(**kw) == code
    assert mg.lib().mgemm_last_error() != b""


def test_null_operands_allowed_when_not_read():
    # alpha == 0 with beta == 1: nothing to do, A and B never read.
    assert call(A=None, B=None, alpha=0.0, beta=1.0) == 0
    # K == 0 with beta == 1: quick return.
    assert call(A=None, B=None, K=0, lda=4, ldb=1, beta=1.0) == 0
    # M == 0: quick return, even with C NULL.
    assert call(M=0, C=None, lda=1, ldc=1) == 0
    assert call(N=0, C=None) == 0


def test_lowercase_and_conjugate_flags():
    assert call(transA="c", transB="t", M=0) == 0


def test_unsupported_precision_and_config():
    assert call(precision=7) == _lib.ERR_UNSUPPORTED
    assert call(config=99) == _lib.ERR_UNSUPPORTED
    assert mg.config_count("fp32") == 13
    # test_precision enumerates the 16-bit configurations by this count
    assert mg.config_count("bf16x3") == 14 and mg.config_count("fp16s") == 14
    for prec in ("fp32", "bf16x3", "fp16s"):
        for cfg in range(mg.config_count(prec)):
            info = mg.config_info(prec, cfg)
            assert info["bm"] > 0 and info["bn"] > 0 and info["threads"] % 64 == 0


def test_alias_detected_before_any_launch():
    # C overlaps A's referenced extent (returned before any HIP call).
    assert call(C=FA + 8) == _lib.ERR_ALIAS
    assert call(C=FB + 60) == _lib.ERR_ALIAS


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="would reach a launch on a GPU")
def test_adjacent_buffers_are_not_an_alias():
    # A ends exactly where C starts: legal, fails later only for lack of a GPU.
    assert call(A=FA, C=FA + 4 * 16) == _lib.ERR_NO_DEVICE


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU driver is present")
def test_valid_call_without_gpu_reports_no_device():
    assert call() == _lib.ERR_NO_DEVICE
    with pytest.raises(mg.MgemmError) as e:
        mg.sgemm("N", "N", 4, 4, 4, 1.0, FA, 4, FB, 4, 0.0, FC, 4, stream=0)
    assert e.value.status == _lib.ERR_NO_DEVICE


def test_bucket_function_is_total():
    L = mg.lib()
    for m, n in ((16, 16), (64, 64), (200, 100), (512, 512), (1000, 9000)):
        b = L.mgemm_grouped_bucket(m, n, 64)
        assert 0 <= b <= 3


def test_plan_functions_reject_null():
    L = mg.lib()
    assert L.mgemm_grouped_plan_destroy(None) == _lib.ERR_BAD_PLAN
    assert L.mgemm_grouped_plan_launch(None, None) == _lib.ERR_BAD_PLAN
    assert L.mgemm_grouped_plan_run(None, None) == _lib.ERR_BAD_PLAN
    t, w = ctypes.c_int64(), ctypes.c_int64()
    assert L.mgemm_grouped_plan_info(None, ctypes.byref(t), ctypes.byref(w)) == _lib.ERR_BAD_PLAN


def test_recorded_choice_overrides_the_heuristic():
    L = mg.lib()
    base = mg.default_config("fp32", "N", "N", 777, 555, 333)
    tn_base = mg.default_config("fp32", "T", "N", 777, 555, 333)
    other = (base + 1) % mg.config_count("fp32")
    mg.record_choice("fp32", "N", "N", 777, 555, 333, other)
    try:
        assert mg.default_config("fp32", "N", "N", 777, 555, 333) == other
        assert mg.default_config("fp32", "T", "N", 777, 555, 333) == tn_base   # exact key only
    finally:
        mg.clear_choices()
    assert mg.default_config("fp32", "N", "N", 777, 555, 333) == base
    assert L.mgemm_record_choice(0, b"N", b"N", 1, 1, 1, 99) == _lib.ERR_UNSUPPORTED
    assert L.mgemm_record_choice(0, b"Q", b"N", 1, 1, 1, 0) == -1


def test_default_configs_are_valid_and_scale_with_the_problem():
    """The built-in choice is a valid configuration for every shape and
    transpose; a 1 x 1 x 1 product takes a tile of at most 64 x 64 and a
    large square product a 256-row tile."""
    rng = random.Random(11)
    dims = [1, 2, 17, 255, 256, 511, 1000, 3001, 4608, 8192, 40000, 2**20]
    for prec in ("fp32", "bf16x3", "fp16s"):
        n_cfg = mg.config_count(prec)
        for _ in range(200):
            M, N, K = (rng.choice(dims) for _ in range(3))
            for ta in "NT":
                for tb in "NT":
                    assert 0 <= mg.default_config(prec, ta, tb, M, N, K) < n_cfg
        tiny = mg.config_info(prec, mg.default_config(prec, "N", "N", 1, 1, 1))
        assert tiny["bm"] * tiny["bn"] <= 64 * 64
        big = mg.config_info(prec, mg.default_config(prec, "N", "N", 8192, 8192, 8192))
        assert big["bm"] == 256


class _FakeStorage:
    def __init__(self, ptr, nbytes):
        self.ptr, self.n = ptr, nbytes

    def data_ptr(self):
        return self.ptr

    def nbytes(self):
        return self.n


class _FakeTensor:
    """Enough of a device tensor for the binding's argument checks."""
    is_cuda = True

    def __init__(self, ptr, nbytes, offset=0, contiguous=False):
        import torch
        self.dtype = torch.float32
        self._st = _FakeStorage(ptr, nbytes)
        self._off = offset
        self._contiguous = contiguous

    def untyped_storage(self):
        return self._st

    def numel(self):
        return max(0, (self._st.n - self._off) // 4)

    def is_contiguous(self):
        return self._contiguous

    def data_ptr(self):
        return self._st.ptr + self._off


def test_tensor_extent_is_checked_before_any_call():
    """A tensor too small for the referenced M x K (ld) array is rejected
    by the binding, so no kernel can run past it."""
    from paper_1912_04379_amd.api import check_operands
    ok = _FakeTensor(FA, 4 * 64 * 64)
    check_operands("N", "N", 64, 64, 64, 1.0, ok, 64, _FakeTensor(FB, 4 * 64 * 64), 64,
                   _FakeTensor(FC, 4 * 64 * 64), 64)
    with pytest.raises(ValueError):        # A one float short
        check_operands("N", "N", 64, 64, 64, 1.0, _FakeTensor(FA, 4 * 64 * 64 - 4), 64,
                       ok, 64, ok, 64)
    with pytest.raises(ValueError):        # C as a view starting 1 KB in
        check_operands("N", "T", 64, 64, 64, 1.0, ok, 64, ok, 64,
                       _FakeTensor(FC, 4 * 64 * 64, offset=1024), 64)
    # A contiguous tensor whose own elements hold the array needs no storage
    # query; one whose elements fall short is still checked against its storage.
    check_operands("N", "N", 64, 64, 64, 1.0, _FakeTensor(FA, 4 * 64 * 64, contiguous=True), 64,
                   ok, 64, ok, 64)
    with pytest.raises(ValueError):
        check_operands("N", "N", 64, 64, 64, 1.0,
                       _FakeTensor(FA, 4 * 64 * 64 - 4, contiguous=True), 64, ok, 64, ok, 64)
    # alpha == 0: A and B are not referenced, so an empty A is fine
    check_operands("N", "N", 64, 64, 64, 0.0, _FakeTensor(FA, 0), 64, _FakeTensor(FB, 0), 64,
                   _FakeTensor(FC, 4 * 64 * 64), 64)


@pytest.mark.parametrize("shape,cfg", [
    ((1024, 1024, 8192), 11), ((512, 512, 2048), 11), ((256, 256, 65536), 11),
    ((1000, 1000, 4000), 11), ((2048, 2048, 4096), 11),
    ((1024, 1024, 2048), None),      # pieces too short for 128 x 128 tiles
    ((256, 256, 2048), 9),           # the small-product kernel
    ((3072, 3072, 8192), None),      # more than one 128 x 128 tile per CU
    ((8192, 8192, 8192), 8)])
def test_fp32_default_rule_split_k(shape, cfg):
    """The FP32 rule as documented: split-K (configuration 11) for at most one
    128 x 128 tile per CU and a long enough k range; otherwise another
    configuration."""
    got = mg.default_config("fp32", "N", "N", *shape)
    if cfg is None:
        assert got != 11
    else:
        assert got == cfg


@pytest.mark.parametrize("shape,cfg", [
    ((6144, 3072, 3072), 11), ((3072, 6144, 2048), 11),   # 288 tiles of 256 x 256
    ((4096, 4096, 4096), 0), ((12288, 1024, 4096), 0), ((3072, 3072, 8192), 0),
    ((8192, 8192, 8192), 10)])
def test_bf16x3_default_rule_slot_share(shape, cfg):
    """From 144 tiles of 256 x 256 (below the pre-packing size), the
    in-staging 256 x 256 tile (0) or the packed 128 x 128 tile (11) by slot
    share; 8192^3 takes the pipelined packed 256 x 256 tile (10)."""
    assert mg.default_config("bf16x3", "N", "N", *shape) == cfg


@pytest.mark.parametrize("prec,shape,split", [
    ("bf16x3", (512, 512, 16384), True), ("bf16x3", (1024, 1024, 8192), True),
    ("bf16x3", (256, 256, 65536), True), ("bf16x3", (2048, 1024, 3072), True),
    ("bf16x3", (1024, 4096, 8192), True), ("bf16x3", (1024, 1024, 1024), False),
    ("bf16x3", (2048, 2048, 4096), False), ("bf16x3", (8192, 8192, 8192), False),
    ("fp16s", (512, 512, 16384), True), ("fp16s", (1024, 1024, 8192), True),
    ("fp16s", (1000, 1000, 4000), True), ("fp16s", (2048, 1024, 3072), True),
    ("fp16s", (1536, 1536, 4096), True), ("fp16s", (1280, 1280, 2048), False),
    ("fp16s", (1024, 4096, 8192), False), ("fp16s", (2048, 2048, 4096), False)])
def test_lowp_default_rule_split_k(prec, shape, split):
    """The 16-bit split-K rule as documented: BF16x3 for at most half a round
    of 128 x 128 tiles with K >= 2048 or a full round with K >= 8192; FP16
    for at most a quarter round with K >= 2048 or five eighths of a round
    with K >= 3072."""
    got = mg.default_config(prec, "N", "N", *shape)
    assert (got == mg.config_count(prec) - 1) == split


def test_choices_round_trip_through_a_cache_file(tmp_path):
    """Recorded single-call choices are saved to a file stamped with the
    device key ("nodevice" 0 without a GPU) and the library version, and
    loaded back into an empty table; lines for another device or version,
    and lines that are not entries, are ignored."""
    L = mg.lib()
    path = str(tmp_path / "tune.txt").encode()
    L.mgemm_clear_choices()
    assert L.mgemm_record_choice(0, b"N", b"T", 777, 555, 333, 2) == 0
    assert L.mgemm_record_choice(1, b"T", b"N", 640, 320, 4096, 5) == 0
    assert L.mgemm_save_choices(path) == 0
    lines = open(path).read().splitlines()
    assert len(lines) == 2
    assert all(l.startswith("mgemm-tune v1 single ") for l in lines)
    with open(path, "a") as f:
        f.write("mgemm-tune v1 single otherarch 8 %d 0 NN 777 555 333 4\n" % mg.version())
        f.write("mgemm-tune v1 single %s 0 99999 0 NN 1 2 3 1\n" % lines[0].split()[3])
        f.write("# a comment line\nrubbish\n")
    L.mgemm_clear_choices()
    assert L.mgemm_default_config(0, b"N", b"T", 777, 555, 333) != 2
    n = ctypes.c_int64(-1)
    assert L.mgemm_load_choices(path, ctypes.byref(n)) == 0
    assert n.value == 2
    assert L.mgemm_default_config(0, b"N", b"T", 777, 555, 333) == 2
    assert L.mgemm_default_config(1, b"T", b"N", 640, 320, 4096) == 5
    L.mgemm_clear_choices()
    assert L.mgemm_load_choices(str(tmp_path / "missing.txt").encode(), None) == \
        _lib.ERR_UNSUPPORTED
