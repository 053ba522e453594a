"""mgemm_sgemm_ex_noalloc: the entry point whose workspace is the library's
static per-device scratch array.  Its results must equal mgemm_sgemm_ex's
(same kernels, same order of every sum: bitwise) on two calls in a row, the
second with a smaller product, and stay within the oracle's bar."""
import numpy as np
import pytest

import paper_1912_04379_amd as mg
import synth
from gpu_util import full_check, log, sampled_check, to_dev
from paper_1912_04379_amd import _lib

pytestmark = pytest.mark.gpu

PREC = {"fp32": 0, "bf16x3": 1, "fp16s": 2}


def _call(fn, c, A, B, C, prec, cfg):
    import torch
    s = torch.cuda.current_stream().cuda_stream
    return fn(c["transA"].encode(), c["transB"].encode(), c["M"], c["N"], c["K"],
              float(c["alpha"]), A.data_ptr(), c["lda"], B.data_ptr(), c["ldb"],
              float(c["beta"]), C.data_ptr(), c["ldc"], s, PREC[prec], cfg)


def _both(c, prec, cfg=-1, ex_cfg=None):
    """C from the no-allocation call and from mgemm_sgemm_ex (config
    `ex_cfg`, default the same) on the same inputs."""
    import torch
    L = mg.lib()
    A, B = to_dev(c["A"]), to_dev(c["B"])
    C1, C2 = to_dev(c["C"]), to_dev(c["C"])
    st = _call(L.mgemm_sgemm_ex_noalloc, c, A, B, C1, prec, cfg)
    assert st == 0, (st, L.mgemm_last_error())
    st = _call(L.mgemm_sgemm_ex, c, A, B, C2, prec, cfg if ex_cfg is None else ex_cfg)
    assert st == 0, (st, L.mgemm_last_error())
    torch.cuda.synchronize()
    return C1.cpu().numpy(), C2.cpu().numpy()


def _log_lines(path):
    return path.read_text().strip().splitlines() if path.exists() else []


# Each pair: a product whose chosen configuration takes workspace, then a
# smaller one, so the second call reads a scratch array the first has
# filled with other data.
PAIRS = [
    # FP32 split-K: S partial products in the scratch array.
    ("fp32", (512, 512, 16384, "T", "N"), (200, 136, 5000, "N", "T"), "f32_split_k"),
    # FP32 thin products (the library's choice): k-piece partial sums and,
    # on the first call, the gathered small operand.
    ("fp32", (8192, 3, 8193, "T", "T"), (1000, 1, 700, "T", "T"), "f32_thin"),
    # Scaled FP16: panel exponents and partial maxima, plus packed operands
    # (2048^3: 16 MiB) on the first call.
    ("fp16s", (2048, 2048, 2048, "N", "N"), (300, 260, 700, "T", "N"), "packed"),
    # BF16x3 through the packed engine (2048^3: 32 MiB of hi and lo halves).
    ("bf16x3", (2048, 2048, 2048, "N", "T"), (520, 390, 1500, "T", "T"), "packed"),
]


@pytest.mark.parametrize("prec,first,second,path", PAIRS, ids=["%s-%s" % (p[0], p[3]) for p in PAIRS])
def test_noalloc_equals_sgemm_ex_twice(prec, first, second, path, tmp_path, monkeypatch):
    logf = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", str(logf))
    cfg = 11 if path == "f32_split_k" else -1
    for i, (M, N, K, ta, tb) in enumerate((first, second)):
        log("noalloc %s call %d: %s%s %dx%dx%d config %d" % (prec, i + 1, ta, tb, M, N, K, cfg))
        c = synth.sgemm_case(20 + i, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=3)
        got, ref = _both(c, prec, cfg)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), \
            "no-allocation result differs from mgemm_sgemm_ex"
        tol = 1e-3 if prec == "fp16s" else 1e-5
        if M * N * K <= 600 ** 3:
            full_check(c, got, bound_fn=None, normwise=tol)
        else:
            sampled_check(c, got, count=600, bound_fn=None, normwise=tol)
    lines = _log_lines(logf)
    noalloc = [l for l in lines if l.startswith("mgemm: sgemm_noalloc")]
    assert len(noalloc) == 2, lines
    assert ("-> %s " % path) in noalloc[0], noalloc[0]
    ws = int(noalloc[0].split("workspace=")[1].split()[0])
    assert 0 < ws <= _lib.NOALLOC_SCRATCH_BYTES, noalloc[0]


def test_noalloc_named_config_beyond_scratch_is_refused():
    """BF16x3 packed 256 x 256 at 4096^3 needs 128 MiB of packed halves:
    refused with MGEMM_ERR_UNSUPPORTED, nothing launched; the library's
    choice for the same product runs a configuration that fits."""
    import torch
    L = mg.lib()
    c = synth.sgemm_case(30, "N", "N", 4096, 4096, 4096, alpha=1.0, beta=0.5, pad=0)
    A, B, C = to_dev(c["A"]), to_dev(c["B"]), to_dev(c["C"])
    log("noalloc bf16x3 4096^3 config 10 (beyond the scratch array)")
    st = _call(L.mgemm_sgemm_ex_noalloc, c, A, B, C, "bf16x3", 10)
    assert st == _lib.ERR_UNSUPPORTED
    assert b"more than the fixed" in L.mgemm_last_error()
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), c["C"])
    log("noalloc bf16x3 4096^3 library's choice (falls back to configuration 0)")
    got, ref = _both(c, "bf16x3", -1, ex_cfg=0)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    sampled_check(c, got, count=400, bound_fn=None, normwise=1e-5)


def test_noalloc_argument_errors_match_sgemm_ex():
    L = mg.lib()
    args = (b"N", b"N", 4, 4, 4, 1.0, 0x1000, 3, 0x2000, 4, 0.0, 0x3000, 4, None, 0, -1)
    assert L.mgemm_sgemm_ex_noalloc(*args) == L.mgemm_sgemm_ex(*args) == -8


def test_fp16s_split_pieces_staged_and_packed_agree(tmp_path, monkeypatch):
    """1024 x 1024 x 16384 scaled FP16 in split-K (eight pieces of 2048 k,
    128 x 128 tiles): the pool holds packed copies of both operands (64 MiB)
    beside the 32 MiB of partial products and the pieces run on them; the
    64 MiB scratch array cannot, so there the pieces scale while staging.
    Both issue the same MFMAs in the same order: equal bitwise."""
    logf = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", str(logf))
    log("noalloc fp16s split-K staged against packed pieces")
    c = synth.sgemm_case(24, "N", "N", 1024, 1024, 16384, alpha=1.5, beta=-0.5, pad=3)
    got, ref = _both(c, "fp16s", 13)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), \
        "in-staging pieces differ from packed pieces"
    sampled_check(c, got, count=600, bound_fn=None, normwise=1e-3)
    lines = _log_lines(logf)
    noalloc = [l for l in lines if l.startswith("mgemm: sgemm_noalloc")]
    pooled = [l for l in lines if l.startswith("mgemm: sgemm fp16s")]
    assert len(noalloc) == 1 and "-> lowp_split_k cfg=13 splits=8" in noalloc[0], lines
    assert len(pooled) == 1 and "-> lowp_split_k_packed cfg=13 splits=8" in pooled[0], lines
