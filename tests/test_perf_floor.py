"""Loose performance floors: not measurements (bench.py makes those), but
regression guards far below the measured rates, so that a slow path taken by
mistake (a wrong tile choice, a fallback, a lost pipeline) fails here."""
import pytest

import paper_1912_04379_amd as mg
from gpu_util import log

pytestmark = pytest.mark.gpu


def time_ms(fn, reps=20, warmup=10):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def square_operands(n):
    import torch
    g = torch.Generator(device="cuda").manual_seed(0)
    ld = n + 16
    A = torch.rand(ld * n, device="cuda", generator=g) * 2 - 1
    B = torch.rand(ld * n, device="cuda", generator=g) * 2 - 1
    C = torch.zeros(ld * n, device="cuda")
    return A, B, C, ld


def test_fp32_and_forms_at_4096():
    """FP32 4096^3 NN measures about 143 TFLOP/s; BF16x3 about 2.7x and
    scaled FP16 about 4.5x its time."""
    n = 4096
    A, B, C, ld = square_operands(n)
    ms = {}
    for prec in ("fp32", "bf16x3", "fp16s"):
        ms[prec] = time_ms(lambda: mg.sgemm("N", "N", n, n, n, 1.0, A, ld, B, ld, 0.0, C, ld,
                                            precision=prec))
        log("perf floor 4096^3 %s: %.3f ms, %.1f TFLOP/s" % (prec, ms[prec], 2 * n ** 3 / ms[prec] / 1e9))
    assert 2 * n ** 3 / ms["fp32"] / 1e9 > 100.0
    assert ms["fp32"] / ms["bf16x3"] > 1.8
    assert ms["fp32"] / ms["fp16s"] > 3.0


def test_small_product_from_a_graph():
    """256^3 replayed from a graph measures about 5 us per call."""
    import torch
    n = 256
    A, B, C = (torch.rand(n * n, device="cuda") for _ in range(3))
    fn = lambda: mg.sgemm("N", "N", n, n, n, 1.0, A, n, B, n, 0.0, C, n)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(50):
            fn()
    us = 1000 * time_ms(g.replay, reps=5, warmup=2) / 50
    log("perf floor 256^3 from a graph: %.2f us per call" % us)
    assert us < 15.0


def test_fp32_one_tile_per_cu():
    """1024^3 NN (256 tiles of 64 x 64 x 32, about one per CU) measures 83-93
    TFLOP/s through the Python binding."""
    n = 1024
    A, B, C, ld = square_operands(n)
    assert mg.default_config("fp32", "N", "N", n, n, n) == 12
    ms = time_ms(lambda: mg.sgemm("N", "N", n, n, n, 1.0, A, ld, B, ld, 0.0, C, ld), reps=50)
    log("perf floor 1024^3 fp32: %.4f ms, %.1f TFLOP/s" % (ms, 2 * n ** 3 / ms / 1e9))
    assert 2 * n ** 3 / ms / 1e9 > 55.0


def test_grouped_batch_replay():
    """The 512-problem batch replayed from its graph measures 70-73 TFLOP/s
    (FP32) and about 100 (BF16x3) with the library's default plans."""
    from test_grouped import make_batch
    problems, data, arena, host = make_batch()
    flops = sum(2.0 * p["M"] * p["N"] * p["K"] for p in problems)
    for prec, floor in (("fp32", 45.0), ("bf16x3", 60.0)):
        with mg.GroupedPlan(problems, prec) as plan:
            ms = time_ms(plan.launch, reps=50, warmup=20)
        log("perf floor grouped %s: %.4f ms, %.1f TFLOP/s" % (prec, ms, flops / ms / 1e9))
        assert flops / ms / 1e9 > floor
