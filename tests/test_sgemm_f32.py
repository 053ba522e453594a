"""FP32 path on the GPU against the FP64 oracle (element by element)."""
import numpy as np
import pytest

import oracle
import paper_1912_04379_amd as mg
import synth
from gpu_util import (full_check, log, logical_c, padding_untouched, run, sampled_check,
                      wide_ldc_case)

pytestmark = pytest.mark.gpu

TRANS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]


def test_small_square_unpadded():
    """256^3, NN, ld 256, alpha 1, beta 0, uniform inputs, seed 0."""
    c = synth.sgemm_case(0, "N", "N", 256, 256, 256, pad=0)
    log("f32 256^3 NN")
    err = full_check(c, run(c))
    log("normwise %.3e" % err)


@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("n", [1000, 1024])
def test_square_all_trans_full(ta, tb, n):
    c = synth.sgemm_case(0, ta, tb, n, n, n, alpha=1.5, beta=-0.5)
    log("f32 %d^3 %s%s" % (n, ta, tb))
    full_check(c, run(c))


@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("n", [2048, 3001, 4096, 4097, 8192])
def test_square_all_trans_sampled(ta, tb, n):
    c = synth.sgemm_case(0, ta, tb, n, n, n, alpha=1.5, beta=-0.5)
    log("f32 %d^3 %s%s (sampled)" % (n, ta, tb))
    sampled_check(c, run(c), count=1500)


# Products a little past whole 256 x 256 tiles, run as the whole-tile block
# and the thin remainders: both remainders, only the rows, only the columns.
EDGE_CASES = [("N", "N", (4097, 4097, 4097)), ("T", "T", (4160, 4100, 4096)),
              ("N", "T", (4096, 4127, 5000)), ("T", "N", (4129, 4096, 4097))]


@pytest.mark.parametrize("ta,tb,shape", EDGE_CASES)
def test_edge_split(ta, tb, shape, tmp_path, monkeypatch):
    """The library's choice splits these products: every entry of the
    remainders (rows M - M mod 256 .. M-1, columns N - N mod 256 .. N-1)
    against the oracle, a sample of the block, C's padding untouched, and
    the path taken."""
    M, N, K = shape
    logf = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", str(logf))
    c = synth.sgemm_case(44, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=3)
    log("f32 edge split %s %s%s" % (shape, ta, tb))
    got = run(c)
    assert "-> f32_edge_split " in logf.read_text()
    sampled_check(c, got, count=600)
    mm, nn = M - M % 256, N - N % 256
    rows = np.concatenate([np.repeat(np.arange(mm, M), N),
                           np.tile(np.arange(mm), N - nn)]).astype(np.int64)
    cols = np.concatenate([np.tile(np.arange(N), M - mm),
                           np.repeat(np.arange(nn, N), mm)]).astype(np.int64)
    args = (ta, tb, M, N, K, float(c["alpha"]), c["A"], c["lda"], c["B"], c["ldb"],
            float(c["beta"]), c["C"], c["ldc"])
    ref = oracle.sgemm_entries(*args, rows, cols)
    Cg = got.reshape(N, c["ldc"])
    edge = Cg[cols, rows].astype(np.float64)
    assert oracle.normwise_rel_err(edge, ref) <= 1e-5
    finite_abs = lambda x: np.abs(np.where(np.isfinite(x), x, 0)).astype(np.float32)
    absargs = (ta, tb, M, N, K, abs(float(c["alpha"])), finite_abs(c["A"]), c["lda"],
               finite_abs(c["B"]), c["ldb"], abs(float(c["beta"])), finite_abs(c["C"]), c["ldc"])
    scale = oracle.sgemm_entries(*absargs, rows, cols)
    assert np.all(np.abs(edge - ref) <= oracle.gamma(K + 2, 2.0 ** -23) * scale)


def test_edge_split_integers_bitwise():
    """Small integers: every partial sum is exact, so an entry computed with
    a wrong operand offset, twice or not at all would show."""
    M, N, K = 4100, 4097, 4096
    c = synth.sgemm_case(45, "T", "N", M, N, K, alpha=1.0, beta=1.0, dist="int16",
                         dist_c="int16", pad=3)
    log("f32 edge split integers")
    got = logical_c(run(c), c)
    rows, cols = synth.sample_entries(1, M, N, 4000)
    mm, nn = M - M % 256, N - N % 256
    rows = np.concatenate([rows, np.arange(mm, M), np.full(N - nn, mm - 1)]).astype(np.int64)
    cols = np.concatenate([cols, np.full(M - mm, N - 1), np.arange(nn, N)]).astype(np.int64)
    args = ("T", "N", M, N, K, 1.0, c["A"], c["lda"], c["B"], c["ldb"], 1.0, c["C"], c["ldc"])
    ref = oracle.sgemm_entries(*args, rows, cols)
    assert np.array_equal(got[rows, cols].astype(np.float64), ref)


@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 37, 5), (37, 1, 5), (33, 65, 7),
                                   (127, 129, 1), (130, 3, 300), (5, 300, 17),
                                   (257, 255, 33), (64, 64, 64)])
def test_ragged_shapes(ta, tb, shape):
    M, N, K = shape
    c = synth.sgemm_case(7, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=5)
    log("f32 ragged %s %s%s" % (shape, ta, tb))
    full_check(c, run(c))


@pytest.mark.parametrize("cfg", range(13))
@pytest.mark.parametrize("ta,tb", TRANS)
def test_every_config(cfg, ta, tb):
    c = synth.sgemm_case(3, ta, tb, 300, 270, 77, alpha=1.5, beta=-0.5, pad=3)
    log("f32 cfg %d %s%s" % (cfg, ta, tb))
    full_check(c, run(c, config=cfg))


@pytest.mark.parametrize("cfg", range(13))
@pytest.mark.parametrize("ta,tb", TRANS)
def test_every_config_sizes_multiple_of_4(cfg, ta, tb):
    """M and N multiples of 4 but of no tile edge, odd leading dimensions
    (rows of A, B and C start at 4-byte but not 16-byte boundaries) and a
    ragged K."""
    c = synth.sgemm_case(31, ta, tb, 292, 268, 83, alpha=1.5, beta=-0.5, pad=3)
    log("f32 sizes multiple of 4 cfg %d %s%s" % (cfg, ta, tb))
    full_check(c, run(c, config=cfg))


@pytest.mark.parametrize("cfg", range(13))
@pytest.mark.parametrize("K", [1, 17, 33])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "T")])
def test_short_k_every_config(cfg, K, ta, tb):
    """K shorter than one slab, one slab plus a ragged one, and so on, for
    every configuration (slab depths 16 and 32)."""
    c = synth.sgemm_case(27, ta, tb, 300, 270, K, alpha=1.5, beta=-0.5, pad=3)
    log("f32 short K cfg %d K %d %s%s" % (cfg, K, ta, tb))
    full_check(c, run(c, config=cfg))


@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 15, 3), (16, 16, 16), (33, 47, 17),
                                   (20, 40, 65), (100, 3, 129), (64, 64, 200), (48, 80, 1000)])
def test_small_product_kernel(ta, tb, shape):
    """Configuration 9 (16 x 16 tiles, k split over four waves): ragged
    tiles, k ranges from one group shared by four waves to many batches."""
    M, N, K = shape
    c = synth.sgemm_case(17, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=3)
    log("f32 small %s %s%s" % (shape, ta, tb))
    full_check(c, run(c, config=9))


@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("shape", [(600, 520, 333), (300, 700, 7), (257, 513, 1000)])
def test_big_tiles_with_small_tile_tail_full(ta, tb, shape):
    """Configuration 10 with fewer 256 x 256 tiles than CUs: every tile is
    the tail, computed as 128 x 128 quarters (those past the edge of C are
    skipped)."""
    M, N, K = shape
    c = synth.sgemm_case(23, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=3)
    log("f32 big+tail %s %s%s" % (shape, ta, tb))
    full_check(c, run(c, config=10))


@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("shape", [(300, 270, 5000), (64, 64, 20000), (257, 129, 3001),
                                   (1000, 1000, 4000)])
def test_split_k(ta, tb, shape):
    """Configuration 11 on products with a long k range: 64 x 64 tiles
    (few tiles) or 128 x 128 tiles (1000^2), k cut into pieces of a
    multiple of 32 with a shorter last piece, partial products added in a
    fixed order by the reduction kernel."""
    M, N, K = shape
    c = synth.sgemm_case(41, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=3)
    log("f32 split-K %s %s%s" % (shape, ta, tb))
    full_check(c, run(c, config=11))


def test_split_k_wide_ldc_runs_unsplit():
    """ldc above the buffer path's limit with a long k range: split-K does
    not apply (the 64-bit path runs 128 x 128 tiles) and the result is
    still correct."""
    c = wide_ldc_case(44, "N", "N", 200, 6, 5000, alpha=1.5, beta=-0.5)
    log("f32 split-K wide ldc")
    full_check(c, run(c, config=11))


def test_split_k_beta_zero_ignores_nan_in_c():
    c = synth.sgemm_case(42, "N", "T", 190, 200, 6000, pad=2)
    c["C"] = np.where(c["C"] == synth.C_SENTINEL, c["C"], np.float32(np.nan)).astype(np.float32)
    got = run(c, config=11)
    assert np.all(np.isfinite(logical_c(got, c)))
    assert padding_untouched(got, c)


def test_split_k_integer_inputs_bitwise():
    """Small integers: every partial sum, and the sum of the pieces, is an
    exact integer in FP32, so split-K equals the oracle bitwise."""
    c = synth.sgemm_case(43, "N", "N", 130, 120, 4100, alpha=1.0, beta=1.0, dist="int16",
                         dist_c="int16")
    got = logical_c(run(c, config=11), c)
    ref = oracle.sgemm(*(c[k] for k in ("transA", "transB", "M", "N", "K", "alpha", "A",
                                         "lda", "B", "ldb", "beta", "C", "ldc")))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "T")])
def test_big_tiles_whole_round_and_tail_sampled(ta, tb):
    """4097^3: 289 tiles of 256 x 256, one whole round on 256 CUs and a tail
    of 33 tiles as 128 x 128 quarters; checked on sampled entries, padding
    and finiteness everywhere."""
    n = 4097
    c = synth.sgemm_case(24, ta, tb, n, n, n, alpha=1.5, beta=-0.5, pad=16)
    log("f32 big+tail 4097 %s%s" % (ta, tb))
    sampled_check(c, run(c, config=10))


@pytest.mark.parametrize("cfg", [-1, 1, 5, 8, 9, 10, 11])
@pytest.mark.parametrize("ta,tb", TRANS)
def test_leading_dimension_beyond_32bit_offsets(cfg, ta, tb):
    """ldc above 2**21 floats: the 64-bit address path runs, whichever
    configuration is asked for.  K = 200 spans 12 full slabs and a partial one."""
    c = wide_ldc_case(13, ta, tb, 300, 6, 200, alpha=1.5, beta=-0.5)
    log("f32 wide ldc cfg %d %s%s" % (cfg, ta, tb))
    full_check(c, run(c, config=cfg))


def test_single_calls_captured_in_a_graph():
    """FP32 calls allocate nothing and never synchronise, so a caller can
    capture them in a HIP graph.  Two calls (the small-product kernel and a
    256 x 256 tile kernel) are captured; each of three replays, with eager
    work and a synchronisation between them, equals the eager result
    bitwise."""
    import torch
    from gpu_util import to_dev
    cases = [synth.sgemm_case(21, "N", "N", 256, 256, 256, alpha=1.5, beta=0.0, pad=0),
             synth.sgemm_case(22, "T", "N", 600, 520, 4100, alpha=1.0, beta=0.0, pad=3)]
    cfgs = [9, 8]
    bufs = [tuple(to_dev(c[k]) for k in ("A", "B", "C")) for c in cases]

    def calls():
        for c, cfg, (A, B, C) in zip(cases, cfgs, bufs):
            mg.sgemm(c["transA"], c["transB"], c["M"], c["N"], c["K"], float(c["alpha"]), A,
                     c["lda"], B, c["ldb"], float(c["beta"]), C, c["ldc"], config=cfg)

    log("f32 graph capture: eager")
    calls()
    torch.cuda.synchronize()
    eager = [C.clone() for (_, _, C) in bufs]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        calls()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    log("f32 graph capture: capture")
    with torch.cuda.graph(g):
        calls()
    for rep in range(3):
        for c, (_, _, C) in zip(cases, bufs):     # C's logical part only
            C[:c["N"] * c["ldc"]].view(c["N"], c["ldc"])[:, :c["M"]].fill_(float("nan"))
        torch.cuda.synchronize()
        log("f32 graph capture: replay %d" % rep)
        g.replay()
        torch.cuda.synchronize()
        for (_, _, C), ref in zip(bufs, eager):
            assert torch.equal(C, ref), "replay %d differs from the eager result" % rep


def test_split_k_captured_in_a_graph():
    """Split-K takes its workspace stream-ordered from the library's pool
    (hipMallocFromPoolAsync / hipFreeAsync), which a graph records as memory
    nodes: a captured split-K call replayed three times, with eager work and
    a synchronisation between replays, equals the eager result bitwise."""
    import torch
    from gpu_util import to_dev
    c = synth.sgemm_case(45, "N", "T", 300, 270, 5000, alpha=1.5, beta=0.0, pad=3)
    A, B, C = (to_dev(c[k]) for k in ("A", "B", "C"))

    def call():
        mg.sgemm(c["transA"], c["transB"], c["M"], c["N"], c["K"], 1.5, A, c["lda"], B,
                 c["ldb"], 0.0, C, c["ldc"], config=11)

    log("f32 split-K graph capture: eager")
    call()
    torch.cuda.synchronize()
    eager = C.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    log("f32 split-K graph capture: capture")
    with torch.cuda.graph(g):
        call()
    for rep in range(3):
        C[:c["N"] * c["ldc"]].view(c["N"], c["ldc"])[:, :c["M"]].fill_(float("nan"))
        torch.cuda.synchronize()
        log("f32 split-K graph capture: replay %d" % rep)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(C, eager), "replay %d differs from the eager result" % rep


@pytest.mark.parametrize("ta,tb", TRANS)
def test_integer_inputs_bitwise(ta, tb):
    """Integer inputs in [-16, 16]: every partial sum is an exact integer in
    FP32, so the GPU result equals the oracle bitwise in any order."""
    c = synth.sgemm_case(9, ta, tb, 200, 190, 260, alpha=1.0, beta=1.0, dist="int16",
                         dist_c="int16")
    got = logical_c(run(c), c)
    ref = oracle.sgemm(*(c[k] for k in ("transA", "transB", "M", "N", "K", "alpha", "A",
                                         "lda", "B", "ldb", "beta", "C", "ldc")))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("cfg", [-1, 1, 8, 9])
def test_identity_is_exact(cfg):
    n, N = 160, 70
    rng = np.random.default_rng(4)
    A = np.eye(n, dtype=np.float32).ravel(order="F")
    B = synth.matrix(rng, n, N, n + 4)
    C = synth.matrix(rng, n, N, n, pad=synth.C_SENTINEL)
    c = dict(transA="N", transB="N", M=n, N=N, K=n, alpha=np.float32(1), beta=np.float32(0),
             A=A, lda=n, B=B, ldb=n + 4, C=C, ldc=n)
    got = logical_c(run(c, config=cfg), c)
    assert np.array_equal(got, B.reshape(N, n + 4)[:, :n].T.astype(np.float64))


def test_k_zero_and_alpha_zero():
    for K, alpha, beta in ((0, 1.0, -0.5), (40, 0.0, 2.0), (40, 0.0, 0.0)):
        c = synth.sgemm_case(5, "N", "N", 70, 50, K, alpha=alpha, beta=beta, pad=2)
        got = run(c)
        want = np.float64(beta) * logical_c(c["C"], c) if beta != 0 else 0.0 * logical_c(c["C"], c)
        assert np.array_equal(logical_c(got, c), want)
        assert padding_untouched(got, c)


@pytest.mark.parametrize("cfg", [-1, 8, 9])
def test_beta_zero_ignores_nan_in_c(cfg):
    c = synth.sgemm_case(6, "T", "N", 90, 80, 70, pad=2)
    c["C"] = np.where(c["C"] == synth.C_SENTINEL, c["C"], np.float32(np.nan)).astype(np.float32)
    got = run(c, config=cfg)
    assert np.all(np.isfinite(logical_c(got, c)))


def test_alpha_zero_beta_one_leaves_c():
    c = synth.sgemm_case(6, "N", "N", 30, 20, 10, alpha=0.0, beta=1.0)
    got = run(c)
    assert np.array_equal(got, c["C"])


def test_side_stream_and_default_stream():
    import torch
    c = synth.sgemm_case(8, "N", "T", 500, 400, 300, alpha=1.5, beta=-0.5)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = run(c, stream=s)
    full_check(c, got)
    full_check(c, run(c, stream=0))


@pytest.mark.parametrize("cfg", [-1, 8, 9])
def test_nan_in_a_row_reaches_that_row_only(cfg):
    c = synth.sgemm_case(10, "N", "N", 100, 60, 50, pad=1)
    A = c["A"].copy()
    A[17 + 3 * c["lda"]] = np.nan       # op(A)[17, 3]
    c["A"] = A
    got = logical_c(run(c, config=cfg), c)
    assert np.all(np.isnan(got[17, :]))
    assert np.all(np.isfinite(np.delete(got, 17, axis=0)))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_tuner_records_a_valid_choice(prec):
    import torch
    c = synth.sgemm_case(12, "T", "N", 600, 500, 400, alpha=1.5, beta=-0.5)
    A, B = (torch.from_numpy(c[k]).cuda() for k in ("A", "B"))
    scratch = torch.from_numpy(c["C"]).cuda()
    try:
        cfg, ms = mg.tune_sgemm("T", "N", 600, 500, 400, 1.5, A, c["lda"], B, c["ldb"], -0.5,
                                scratch, c["ldc"], precision=prec, reps=2)
        assert 0 <= cfg < mg.config_count(prec) and ms > 0
        assert mg.default_config(prec, "T", "N", 600, 500, 400) == cfg
        tol = 1e-5
        got = run(c, precision=prec)            # config -1 now uses the tuned choice
        ref = oracle.sgemm(*(c[k] for k in ("transA", "transB", "M", "N", "K", "alpha", "A",
                                             "lda", "B", "ldb", "beta", "C", "ldc")))
        assert oracle.normwise_rel_err(logical_c(got, c), ref) <= tol
    finally:
        mg.clear_choices()


def test_tuner_on_an_edge_split_shape(tmp_path, monkeypatch):
    """4097^3: the library's own choice is the edge split, which the tuner
    must beat by 2% before it records a whole-product configuration; when
    the split stays, nothing is recorded (an earlier choice is dropped) and
    calls keep splitting."""
    import torch
    n = 4097
    c = synth.sgemm_case(13, "N", "N", n, n, n, alpha=1.0, beta=0.0, pad=3)
    A, B = (torch.from_numpy(c[k]).cuda() for k in ("A", "B"))
    scratch = torch.from_numpy(c["C"]).cuda()
    logf = tmp_path / "mgemm.log"
    try:
        mg.record_choice("fp32", "N", "N", n, n, n, 3)        # dropped by the tuner
        cfg, ms = mg.tune_sgemm("N", "N", n, n, n, 1.0, A, c["lda"], B, c["ldb"], 0.0,
                                scratch, c["ldc"], reps=2)
        log("tuner at 4097^3: config %d, %.3f ms" % (cfg, ms))
        assert ms > 0 and -1 <= cfg < mg.config_count("fp32")
        monkeypatch.setenv("MGEMM_LOG", str(logf))
        got = run(c)
        if cfg == -1:
            assert mg.default_config("fp32", "N", "N", n, n, n) == 12   # nothing recorded
            assert "-> f32_edge_split " in logf.read_text()
        else:
            assert mg.default_config("fp32", "N", "N", n, n, n) == cfg
            assert "-> f32_edge_split " not in logf.read_text()
        sampled_check(c, got, count=600)
    finally:
        mg.clear_choices()
