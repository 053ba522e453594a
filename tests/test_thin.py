"""FP32 products with at most 8 columns (or rows) of C: the library's choice
streams the large operand once in k pieces and adds the pieces' partial
sums in a fixed order.  Against the FP64 oracle element by element."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import full_check, log, logical_c, run

pytestmark = pytest.mark.gpu

TRANS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]
# (M, N, K): few columns, few rows, ragged everywhere, K not a multiple of
# 4 or of the 256-deep pieces.
SHAPES = [(1000, 1, 1000), (4097, 3, 513), (300, 8, 2049), (1, 1000, 1000), (5, 4097, 777),
          (8, 256, 4097), (2, 2, 300),
          # At least 2^25 elements of the large operand: with TT (few
          # columns) or NN (few rows) the small operand is gathered first.
          (8200, 2, 4099), (3, 8200, 4099)]


@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("shape", SHAPES)
def test_thin_products(ta, tb, shape, tmp_path, monkeypatch):
    M, N, K = shape
    logf = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", str(logf))
    c = synth.sgemm_case(60, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=5)
    log("thin %s %s%s" % (shape, ta, tb))
    full_check(c, run(c))
    cols = N <= 8
    kcontig = (ta == "T") if cols else (tb == "N")
    P, r = (M, N) if cols else (N, M)
    thin = (min(M, N) <= 8 and max(M, N) >= 256 and K >= 256
            and not (kcontig and r > 4 and P * K < 2 ** 25))
    assert ("-> f32_thin " in logf.read_text()) == thin


def test_thin_beta_zero_ignores_nan_in_c():
    c = synth.sgemm_case(61, "N", "T", 2000, 4, 1500, alpha=2.0, beta=0.0, pad=3)
    C = c["C"].copy()
    C[:] = np.nan
    c["C"] = C
    got = logical_c(run(c), c)
    assert np.all(np.isfinite(got))
    ref = oracle.sgemm(*(c[k] for k in ("transA", "transB", "M", "N", "K", "alpha", "A", "lda",
                                         "B", "ldb", "beta", "C", "ldc")))
    assert oracle.normwise_rel_err(got, ref) <= 1e-6


def test_thin_integers_bitwise():
    """Small integers: every partial sum is exact, so a k block missing from
    a piece, or taken twice, would show."""
    for (M, N, K, ta, tb) in ((3000, 7, 4099, "N", "N"), (6, 3000, 4099, "T", "T"),
                              (2500, 1, 2000, "T", "N"), (1, 2500, 2000, "N", "T"),
                              (8200, 7, 4099, "T", "T"), (6, 8200, 4099, "N", "N")):
        c = synth.sgemm_case(62, ta, tb, M, N, K, alpha=1.0, beta=1.0, dist="int16",
                             dist_c="int16")
        got = logical_c(run(c), c)
        ref = oracle.sgemm(*(c[k] for k in ("transA", "transB", "M", "N", "K", "alpha", "A",
                                             "lda", "B", "ldb", "beta", "C", "ldc")))
        assert np.array_equal(got, ref), (M, N, K, ta, tb)


def test_thin_is_deterministic():
    c = synth.sgemm_case(63, "T", "N", 4096, 5, 8191, alpha=1.0, beta=0.5, pad=2)
    a = run(c)
    b = run(c)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_thin_tuner_keeps_the_library_path(tmp_path, monkeypatch):
    """8192 x 1 x 8193: the thin path is the library's choice and the one
    the tuner must beat by 2% before it records a configuration; no tile
    configuration does (they compute at least 64 columns), so nothing is
    recorded (an earlier choice is dropped) and calls stay on the thin path."""
    import paper_1912_04379_amd as mg
    import torch
    M, N, K = 8192, 1, 8193
    c = synth.sgemm_case(64, "N", "N", M, N, K, alpha=1.0, beta=0.0, pad=3)
    A, B = (torch.from_numpy(c[k]).cuda() for k in ("A", "B"))
    scratch = torch.from_numpy(c["C"]).cuda()
    logf = tmp_path / "mgemm.log"
    try:
        mg.record_choice("fp32", "N", "N", M, N, K, 3)        # dropped by the tuner
        cfg, ms = mg.tune_sgemm("N", "N", M, N, K, 1.0, A, c["lda"], B, c["ldb"], 0.0,
                                scratch, c["ldc"], reps=2)
        log("tuner at 8192x1x8193: config %d, %.4f ms" % (cfg, ms))
        assert cfg == -1 and ms > 0
        monkeypatch.setenv("MGEMM_LOG", str(logf))
        full_check(c, run(c))
        assert "-> f32_thin " in logf.read_text()
    finally:
        mg.clear_choices()

