"""BF16x3 and scaled-FP16 forms on the GPU against the FP64 oracle.

Three checks per case:
* against the exact product: normwise error within the stated tolerance
  (BF16x3 <= 1e-5, FP16s <= 1e-3);
* against the oracle's FP64 evaluation of the same form (same splits and
  scalings, exact sums): the difference must be pure FP32 accumulation
  error, gamma_n |terms| elementwise (any order, any rounding inside the
  MFMA), and, normwise, within the statistical bar of form_bars.stat_bar
  for round-to-nearest accumulation.  A dropped correction term, a wrong
  scale or a truncating conversion fails the elementwise bar by orders of
  magnitude; a truncating split or a kept lo*lo (K <= 2048) fails the
  statistical one.
"""
import numpy as np
import pytest

import oracle
import synth
from form_bars import stat_bar
from gpu_util import log, logical_c, padding_untouched, run, sampled_check, wide_ldc_case

# Tile configurations of the 16-bit forms: 0..3 split while staging, the
# rest stream pre-packed operands (test_abi checks the count).
N_CONFIGS = 14
PACKED_CONFIGS = list(range(4, N_CONFIGS - 1))
SPLITK_CONFIG = N_CONFIGS - 1

pytestmark = pytest.mark.gpu

TRANS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]
FORMS = {"bf16x3": (oracle.bf16x3, 1e-5), "fp16s": (oracle.f16_scaled, 1e-3)}
ENTRIES = {"bf16x3": oracle.bf16x3_entries, "fp16s": oracle.f16_scaled_entries}


def args_of(c):
    return (c["transA"], c["transB"], c["M"], c["N"], c["K"], c["alpha"], c["A"], c["lda"],
            c["B"], c["ldb"], c["beta"], c["C"], c["ldc"])


def abs_case(c):
    d = dict(c)
    d["A"] = np.abs(np.where(np.isfinite(c["A"]), c["A"], 0)).astype(np.float32)
    d["B"] = np.abs(np.where(np.isfinite(c["B"]), c["B"], 0)).astype(np.float32)
    d["C"] = np.abs(c["C"]).astype(np.float32)
    d["alpha"], d["beta"] = abs(c["alpha"]), abs(c["beta"])
    return d


def check_form(c, prec, got_buf):
    emulate, tol = FORMS[prec]
    got = logical_c(got_buf, c)
    assert padding_untouched(got_buf, c), "C padding was written"
    assert np.all(np.isfinite(got))
    exact = oracle.sgemm(*args_of(c))
    err = oracle.normwise_rel_err(got, exact)
    assert err <= tol, "%s normwise error %.3e > %.0e" % (prec, err, tol)
    emu = emulate(*args_of(c))
    if prec == "fp16s":
        # FP16 rounding and power-of-two scaling commute with |.|, so the
        # form applied to |A|, |B| sums the magnitudes of its own terms.
        mag = emulate(*args_of(abs_case(c)))
    else:
        # |hi| <= |x| (1 + 2^-8) and |lo| <= 2^-8 |x|: the three terms sum
        # to at most (1 + 2^-6) |a||b| in magnitude.
        mag = (1 + 2.0 ** -6) * oracle.abs_product(*args_of(c))
    nterms = 3 * c["K"] + 2 if prec == "bf16x3" else c["K"] + 2
    bound = oracle.gamma(nterms, 2.0 ** -23) * mag
    bad = np.abs(got - emu) > bound
    assert not bad.any(), "%s differs from its FP64 emulation beyond FP32 rounding at %s" % (
        prec, np.argwhere(bad)[:4])
    check_stat(prec, got, emu, c["K"])
    return err


def check_stat(prec, got, emu, K):
    """Normwise distance to the form's emulation within the statistical bar."""
    d = oracle.normwise_rel_err(got, emu)
    log("  %s vs emulation %.3e (%.2f of the bar)" % (prec, d, d / stat_bar(K)))
    assert d <= stat_bar(K), "%s normwise %.3e from its emulation > bar %.3e" % (
        prec, d, stat_bar(K))


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("shape", [(256, 256, 256), (300, 270, 77), (33, 65, 7),
                                   (1, 1, 1), (129, 5, 1000)])
def test_forms_small(prec, ta, tb, shape):
    M, N, K = shape
    c = synth.sgemm_case(31, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=3)
    log("%s %s %s%s" % (prec, shape, ta, tb))
    check_form(c, prec, run(c, precision=prec))


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
@pytest.mark.parametrize("cfg", range(N_CONFIGS))
def test_forms_every_config(prec, cfg):
    c = synth.sgemm_case(32, "T", "N", 520, 390, 200, alpha=1.5, beta=-0.5, dist="loguni")
    log("%s cfg %d" % (prec, cfg))
    check_form(c, prec, run(c, precision=prec, config=cfg))


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
@pytest.mark.parametrize("cfg", range(N_CONFIGS))
def test_forms_every_config_every_trans_pair(prec, cfg):
    """Each configuration instantiates its tile once per operand layout:
    every one of them on a ragged product."""
    for ta, tb in TRANS:
        c = synth.sgemm_case(33, ta, tb, 301, 259, 97, alpha=-1.25, beta=0.5, pad=7)
        log("%s cfg %d %s%s" % (prec, cfg, ta, tb))
        check_form(c, prec, run(c, precision=prec, config=cfg))


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("shape", [(200, 136, 5000), (300, 260, 3001)])
def test_forms_split_k(prec, ta, tb, shape, tmp_path, monkeypatch):
    """Split-K of the 16-bit forms: pieces of the k range as in-staging
    tiles, added in a fixed order.  Against the exact product and the form's
    emulation, bitwise the same on a second run, and taken (not a
    fallback)."""
    M, N, K = shape
    logf = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", str(logf))
    c = synth.sgemm_case(33, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=3, dist="loguni")
    log("%s split-K %s %s%s" % (prec, shape, ta, tb))
    got = run(c, precision=prec, config=SPLITK_CONFIG)
    check_form(c, prec, got)
    again = run(c, precision=prec, config=SPLITK_CONFIG)
    assert np.array_equal(got.view(np.uint32), again.view(np.uint32))
    assert "-> lowp_split_k cfg=%d splits=" % SPLITK_CONFIG in logf.read_text()


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
def test_forms_split_k_integer_inputs_bitwise(prec):
    """|v| <= 16, K = 8192: every partial sum is an integer below 2**24, so
    the split sums are exact and equal the oracle bitwise."""
    c = synth.sgemm_case(34, "N", "T", 130, 70, 8192, alpha=1.0, beta=1.0, dist="int16",
                         dist_c="int16")
    log("%s split-K integers" % prec)
    got = logical_c(run(c, precision=prec, config=SPLITK_CONFIG), c)
    assert np.array_equal(got, oracle.sgemm(*args_of(c)))


# 81 tiles of 128 x 128 (at least a quarter of the CUs), K = 2080: seven
# pieces of 320 k (the last 160), each on packed operands for the FP16 form.
PACKED_SPLIT_SHAPE = (1040, 1030, 2080)


@pytest.mark.parametrize("ta,tb", TRANS)
def test_fp16s_split_k_on_packed_operands(ta, tb, tmp_path, monkeypatch):
    """Split-K of the scaled-FP16 form with 128 x 128 pieces packs each
    operand once and runs the pieces on the packed copies: within the form's
    bars, bitwise the same on a second run, and that path taken."""
    M, N, K = PACKED_SPLIT_SHAPE
    logf = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", str(logf))
    c = synth.sgemm_case(35, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=3, dist="loguni")
    log("fp16s packed split-K %s%s" % (ta, tb))
    got = run(c, precision="fp16s", config=SPLITK_CONFIG)
    check_form(c, "fp16s", got)
    again = run(c, precision="fp16s", config=SPLITK_CONFIG)
    assert np.array_equal(got.view(np.uint32), again.view(np.uint32))
    assert "-> lowp_split_k_packed cfg=%d splits=7" % SPLITK_CONFIG in logf.read_text()


def test_fp16s_split_k_on_packed_operands_integers_bitwise(tmp_path, monkeypatch):
    """Small integers: every partial sum is exact, so a block of k missing
    from a piece, or taken twice, would show in the sum."""
    M, N, K = PACKED_SPLIT_SHAPE
    logf = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", str(logf))
    c = synth.sgemm_case(36, "T", "N", M, N, K, alpha=1.0, beta=1.0, dist="int16",
                         dist_c="int16")
    log("fp16s packed split-K integers")
    got = logical_c(run(c, precision="fp16s", config=SPLITK_CONFIG), c)
    assert np.array_equal(got, oracle.sgemm(*args_of(c)))
    assert "-> lowp_split_k_packed" in logf.read_text()


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
def test_wide_range_inputs_2048(prec):
    """Sign-random magnitudes 2**U[-8, 8], NN at 2048^3, lda = rows + 16,
    alpha 1, beta 0: the error is the product's own."""
    c = synth.sgemm_case(0, "N", "N", 2048, 2048, 2048, dist="loguni")
    log("%s 2048^3 loguni" % prec)
    err = check_form(c, prec, run(c, precision=prec))
    log("normwise %.3e" % err)


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
def test_wide_range_inputs_8192_sampled(prec):
    """The full-size precision-form product, in the launch the benchmark
    times: sampled entries against the exact product (normwise) and against
    the form's emulation (elementwise and statistical bars)."""
    c = synth.sgemm_case(0, "N", "N", 8192, 8192, 8192, dist="loguni")
    log("%s 8192^3 loguni (sampled)" % prec)
    got_buf = run(c, precision=prec)
    err = sampled_check(c, got_buf, count=1500, bound_fn=None, normwise=FORMS[prec][1])
    log("sampled normwise %.3e" % err)
    rows, cols = synth.sample_entries(0, 8192, 8192, 1500)
    got = got_buf.reshape(8192, c["ldc"])[cols, rows].astype(np.float64)
    emu = ENTRIES[prec](*args_of(c), rows, cols)
    if prec == "fp16s":
        mag = ENTRIES[prec](*args_of(abs_case(c)), rows, cols)
        nterms = c["K"] + 2
    else:
        a = abs_case(c)
        mag = (1 + 2.0 ** -6) * oracle.sgemm_entries(*args_of(a), rows, cols)
        nterms = 3 * c["K"] + 2
    assert np.all(np.abs(got - emu) <= oracle.gamma(nterms, 2.0 ** -23) * mag)
    check_stat(prec, got, emu, c["K"])


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
@pytest.mark.parametrize("ta,tb", TRANS)
def test_integer_inputs_bitwise(prec, ta, tb):
    """|v| <= 16 is exact in BF16 and in scaled FP16: both forms equal the
    oracle bitwise."""
    c = synth.sgemm_case(33, ta, tb, 200, 170, 300, alpha=1.0, beta=1.0, dist="int16",
                         dist_c="int16")
    got = logical_c(run(c, precision=prec), c)
    assert np.array_equal(got, oracle.sgemm(*args_of(c)))


def test_bf16x3_identity_within_split_residue():
    """op(A) = I: C = hi(B) + lo(B), within 2**-16 |B| elementwise."""
    n, N = 96, 50
    rng = np.random.default_rng(4)
    A = np.eye(n, dtype=np.float32).ravel(order="F")
    B = synth.matrix(rng, n, N, n, dist="loguni")
    C = np.zeros(n * N, dtype=np.float32)
    c = dict(transA="N", transB="N", M=n, N=N, K=n, alpha=np.float32(1), beta=np.float32(0),
             A=A, lda=n, B=B, ldb=n, C=C, ldc=n)
    got = logical_c(run(c, precision="bf16x3"), c)
    Bl = B.reshape(N, n).T.astype(np.float64)
    assert np.all(np.abs(got - Bl) <= 2.0 ** -16 * np.abs(Bl))


@pytest.mark.parametrize("scale", [1e-6, 1e6])
def test_fp16s_extreme_magnitudes(scale):
    """Values far outside FP16's range (or below its normal range) are
    brought into range by the panel scaling: error stays within 1e-3."""
    c = synth.sgemm_case(34, "N", "T", 300, 200, 150)
    c["A"] = (c["A"] * np.float32(scale)).astype(np.float32)
    c["B"] = (c["B"] * np.float32(scale)).astype(np.float32)
    check_form(c, "fp16s", run(c, precision="fp16s"))


def test_fp16s_panels_with_different_scales():
    """Each 32-row panel of op(A) gets its own scale: rows 0..31 tiny, rows
    32..63 huge, a zero panel, and the ragged last panel."""
    M, N, K = 100, 70, 90
    c = synth.sgemm_case(35, "N", "N", M, N, K)
    A = c["A"].reshape(K, c["lda"]).copy()
    A[:, 0:32] *= np.float32(1e-5)
    A[:, 32:64] *= np.float32(3e4)
    A[:, 64:96] = 0
    c["A"] = A.reshape(-1).astype(np.float32)
    got = run(c, precision="fp16s")
    check_form(c, "fp16s", got)
    assert np.all(logical_c(got, c)[64:96, :] == 0)


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
def test_forms_alpha_beta_rules(prec):
    c = synth.sgemm_case(36, "N", "N", 64, 48, 40, alpha=0.0, beta=-0.5)
    got = run(c, precision=prec)
    assert np.array_equal(logical_c(got, c), -0.5 * logical_c(c["C"], c))
    c = synth.sgemm_case(36, "T", "T", 64, 48, 40)
    c["C"] = np.where(c["C"] == synth.C_SENTINEL, c["C"], np.float32(np.nan)).astype(np.float32)
    assert np.all(np.isfinite(logical_c(run(c, precision=prec), c)))


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
@pytest.mark.parametrize("ta,tb", TRANS)
def test_packed_equals_in_staging_bitwise(prec, ta, tb):
    """Configuration 4 (operands pre-packed, streamed into LDS by direct
    loads) and configuration 0 (split while staging) use the same 256 x 256
    tile, the same splits and the same MFMA operand order: equal bitwise."""
    c = synth.sgemm_case(40, ta, tb, 600, 520, 333, alpha=1.5, beta=-0.5, pad=5)
    log("%s packed vs in-staging %s%s" % (prec, ta, tb))
    a = run(c, precision=prec, config=0)
    b = run(c, precision=prec, config=4)
    assert np.array_equal(a, b)
    check_form(c, prec, b)
    # Other packed tiles, stage depths and loop schedules keep the order of
    # the MFMAs into every accumulator.
    for cfg in (5, 6, 10, 11, 12):
        assert np.array_equal(a, run(c, precision=prec, config=cfg)), cfg


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
@pytest.mark.parametrize("cfg", PACKED_CONFIGS)
def test_packed_ragged_and_tiny(prec, cfg):
    for shape in ((1, 1, 1), (33, 65, 7), (300, 129, 1000), (257, 255, 31)):
        M, N, K = shape
        c = synth.sgemm_case(41, "T", "N", M, N, K, alpha=1.5, beta=-0.5, pad=3)
        log("%s packed cfg %d %s" % (prec, cfg, shape))
        check_form(c, prec, run(c, precision=prec, config=cfg))


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
@pytest.mark.parametrize("cfg", [-1, 4])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "T")])
def test_forms_leading_dimension_beyond_32bit_offsets(prec, cfg, ta, tb):
    """ldc above 2**21 floats takes the 64-bit address path in both forms."""
    c = wide_ldc_case(14, ta, tb, 300, 6, 600, alpha=1.5, beta=-0.5)
    log("%s wide ldc cfg %d %s%s" % (prec, cfg, ta, tb))
    check_form(c, prec, run(c, precision=prec, config=cfg))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16s"])
def test_golden_integer_cases_bitwise(prec):
    """The stored exact integer results (tests/golden): every partial sum is
    exact in all three forms, so each must reproduce them bitwise."""
    from golden_util import golden_cases
    for c, want in golden_cases():
        log("%s golden %s%s %dx%dx%d" % (prec, c["transA"], c["transB"], c["M"], c["N"], c["K"]))
        got_buf = run(c, precision=prec)
        assert padding_untouched(got_buf, c)
        assert np.array_equal(logical_c(got_buf, c), want)


@pytest.mark.parametrize("prec", ["bf16x3", "fp16s"])
def test_workspace_pool_across_streams_and_trim(prec):
    """The 16-bit forms take their workspace from the library's pool: calls
    alternate between a side stream and the default stream, with
    synchronisations and a trim of the pool in between; every result is
    checked against the oracle."""
    import torch
    import paper_1912_04379_amd as mg
    cases = [synth.sgemm_case(50 + i, "N", "T", 700 + 64 * i, 650, 900, alpha=1.5, beta=-0.5)
             for i in range(3)]
    side = torch.cuda.Stream()
    for rep in range(2):
        for i, c in enumerate(cases):
            log("%s pool rep %d case %d" % (prec, rep, i))
            if i % 2:
                with torch.cuda.stream(side):
                    got = run(c, precision=prec, config=4, stream=side)
            else:
                got = run(c, precision=prec, config=4, stream=0)
            check_form(c, prec, got)
        mg.trim_workspace()


def test_fp16s_nan_in_a_row_reaches_that_row_only():
    """A NaN in row i of op(A): its panel's exponent is 0 (reading of the
    scale rule), row i of C is NaN, and every other row, including the rest
    of that panel computed unscaled, matches the form's emulation."""
    c = synth.sgemm_case(37, "N", "N", 150, 90, 120)
    A = c["A"].copy()
    A[40 + 7 * c["lda"]] = np.nan            # op(A)[40, 7], panel 1
    c["A"] = A
    log("fp16s NaN row")
    got = logical_c(run(c, precision="fp16s"), c)
    assert np.all(np.isnan(got[40, :]))
    rest = np.r_[0:40, 41:150]
    assert np.all(np.isfinite(got[rest, :]))
    emu = oracle.f16_scaled(*args_of(c))
    assert np.all(np.isnan(emu[40, :]))
    mag = oracle.f16_scaled(*args_of(abs_case(c)))
    bound = oracle.gamma(c["K"] + 2, 2.0 ** -23) * mag[rest, :]
    assert np.all(np.abs(got[rest, :] - emu[rest, :]) <= bound)


@pytest.mark.parametrize("ta", ["N", "T"])
def test_fp16s_panel_grouping_on_subnormals(ta):
    """op(A) 40 x 1 (K = 1), op(B) = [1 1]: rows 0-15 are 32, rows 16-39 are
    a = 2^-25 (1 + 3*2^-10).  Rows 16-31 share the first 32-row panel with
    the 32s, are scaled by 2^9 into FP16's subnormal range and round to
    257 * 2^-24, so C = 2^-25 + 2^-33; rows 32-39 form the second panel,
    scaled by 2^39, where a is an FP16 value, so C = a.  Each value is
    worked out by hand and must be reproduced bitwise."""
    a = np.float32(2.0 ** -25 * (1 + 3 * 2.0 ** -10))
    Avals = np.array([32.0] * 16 + [a] * 24, dtype=np.float32)
    want_col = np.array([32.0] * 16 + [2.0 ** -25 + 2.0 ** -33] * 16 + [float(a)] * 8)
    c = dict(transA=ta, transB="N", M=40, N=2, K=1, alpha=np.float32(1), beta=np.float32(0),
             A=Avals, lda=40 if ta == "N" else 1, B=np.ones(2, dtype=np.float32), ldb=1,
             C=np.zeros(80, dtype=np.float32), ldc=40)
    for cfg in (-1, 0, 4):
        log("fp16s subnormal panels %s cfg %d" % (ta, cfg))
        got = logical_c(run(c, precision="fp16s", config=cfg), c)
        assert np.array_equal(got, np.stack([want_col, want_col], axis=1)), cfg
