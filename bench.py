"""Benchmark: SGEMM TFLOP/s at M=N=K=8192 on one MI355X, the BF16x3 and
scaled-FP16 forms beside it, and the FP64 oracle on the host's cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one C <- alpha op(A) op(B) + beta C call at M=N=K=8192, NN,
lda=ldb=ldc=8208 (stored rows + 16, the padded-stride analogue of the
paper's Section 4 method), alpha=1.5, beta=-0.5, A/B/C uniform on [-1, 1)
from seed 0.  Inputs are resident in HBM before timing starts.  W untimed
steps, then exactly K steps between two synchronisations, timed with HIP
events on the stream the kernels run on.  One JSON line goes to stdout;
progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SGEMM TFLOP/s @N=8192 & % of peak; bf16x3-vs-fp32 speedup at equal error"
PEAK = {"fp32": 157.3, "bf16": 2516.6, "fp16": 2516.6}     # dense MFMA, TFLOP/s
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {
    "fp32": ["sgemm_f32.hip", "tile_f32.hpp", "tile_common.hpp"],
    "bf16x3": ["sgemm_lowp.hip", "tile_lowp.hpp", "tile_common.hpp"],
    "fp16s": ["sgemm_lowp.hip", "tile_lowp.hpp", "tile_common.hpp"],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(prec):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[prec]:
        p = os.path.join(ROOT, "paper_1912_04379_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(key, prec):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None
    when none exist or the kernel source changed since they were taken."""
    try:
        rec = json.load(open(TRAFFIC_FILE))[key]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_sha") != source_hash(prec):
        return None
    return rec.get("bytes_per_launch")


def timed(fn, steps, warmup, stream, min_ms=0.0):
    """Mean time per call of `steps` back-to-back calls after `warmup` calls.
    With min_ms > 0 (the sections other than the headline FP32 step), both
    the warm-up and the timed run are extended to at least min_ms of work
    each, so that short calls are timed at a steady engine clock."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if min_ms > 0:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        per = max(e0.elapsed_time(e1), 1e-3)
        reps = int(min_ms / per) + 1
        for _ in range(reps):
            fn()
        steps = max(steps, reps)
        torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def per_call_ms(fn, reps, stream):
    """Median of `reps` individually timed calls (after the timed region)."""
    import torch
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def prewarm(torch, seconds):
    """Back-to-back 4096^3 FP32 products through torch for about `seconds`,
    so that the engine clock has ramped up before the first library launch
    (the first few launches after an idle period otherwise run slower)."""
    if seconds <= 0:
        return
    x = torch.rand(4096, 4096, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.time()
    while time.time() - t0 < seconds:
        for _ in range(10):
            torch.mm(x, x, out=y)
        torch.cuda.synchronize()
    del x, y


def under_profiler():
    """True when a profiler's library is preloaded into this process: then
    no child program may be started (the preload would initialise the GPU
    in the child before it replaces itself with the new program)."""
    pre = os.environ.get("LD_PRELOAD", "")
    return "rocprof" in pre or any(k.startswith("ROCPROF") for k in os.environ)


def clock_under_load(fn, seconds=2.0):
    """Engine clock of each XCD, read with `amd-smi metric --clock --json`
    while `fn` runs back to back for about `seconds` (None if amd-smi is
    not there)."""
    import subprocess
    import threading
    import torch
    out = {}

    def sample():
        time.sleep(seconds / 2)
        try:
            r = subprocess.run(["amd-smi", "metric", "--clock", "--json"], capture_output=True,
                               text=True, timeout=30)
            out["json"] = r.stdout if r.returncode == 0 else None
        except (OSError, subprocess.SubprocessError):
            out["json"] = None

    th = threading.Thread(target=sample)
    th.start()
    t0 = time.perf_counter()
    while th.is_alive() or time.perf_counter() - t0 < seconds:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()
    th.join()
    try:
        gpu = json.loads(out["json"])["gpu_data"][0]["clock"]
        mhz = [v["clk"]["value"] for k, v in sorted(gpu.items()) if k.startswith("gfx_")]
        return {"mean_mhz": round(sum(mhz) / len(mhz), 1), "per_xcd_mhz": mhz,
                "max_mhz": gpu["gfx_0"]["max_clk"]["value"],
                "how": "amd-smi metric --clock, sampled once mid-way through %.0f s of "
                       "back-to-back calls" % seconds}
    except (KeyError, TypeError, ValueError, ZeroDivisionError):
        return None


def cold_time(fn, reps, stream, flush):
    """Median time of one call after writing a 512 MB buffer (evicts L2 and
    the MALL), as the paper flushes caches between calls."""
    import torch
    ts = []
    for _ in range(reps):
        flush.zero_()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="time only the FP32 path (for profiling runs)")
    ap.add_argument("--cold-reps", type=int, default=7)
    ap.add_argument("--no-grouped", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-mlp", action="store_true")
    ap.add_argument("--no-splitk", action="store_true")
    ap.add_argument("--no-thin", action="store_true")
    ap.add_argument("--no-prepacked", action="store_true")
    ap.add_argument("--grouped-defaults", action="store_true",
                    help="replay the library's default grouped plans instead of tuned ones "
                         "(profiling runs: every pass then runs the same kernels)")
    ap.add_argument("--no-vendor", action="store_true",
                    help="skip the ROCm BLAS (torch.addmm) comparison")
    ap.add_argument("--no-wide-range", action="store_true",
                    help="skip the three paths on wide-range (2^U[-8,8]) inputs")
    ap.add_argument("--no-clock", action="store_true",
                    help="do not sample the engine clock with amd-smi")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the size sweep (all trans pairs) and the 2048^3 forms")
    ap.add_argument("--no-single-calls", action="store_true",
                    help="skip the median of synchronised single FP32 calls (profiling runs: "
                         "the idle gaps between them let the engine clock dip)")
    ap.add_argument("--prewarm-s", type=float, default=1.0,
                    help="seconds of back-to-back torch FP32 products before anything is "
                         "timed, so that no library launch runs while the clock ramps up")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(asked for --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1912_04379_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    import oracle
    import paper_1912_04379_amd as mg
    import synth

    n = args.size
    alpha, beta = 1.5, -0.5
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    log("generating inputs %d^3 ..." % n)
    case = synth.sgemm_case(0, "N", "N", n, n, n, alpha=alpha, beta=beta, pad=16)
    ld = case["lda"]
    A = torch.from_numpy(case["A"]).to(dev)
    B = torch.from_numpy(case["B"]).to(dev)
    C0 = torch.from_numpy(case["C"]).to(dev)
    C = C0.clone()
    flops = 2.0 * n * n * n

    def call(prec, out):
        return lambda: mg.sgemm("N", "N", n, n, n, alpha, A, ld, B, ld, beta, out, ld,
                                precision=prec)

    # Error on sampled entries, from a fresh C0 each time (beta != 0).
    rows, cols = synth.sample_entries(1, n, n, 2048)
    log("oracle on %d sampled entries ..." % rows.size)
    ref = oracle.sgemm_entries("N", "N", n, n, n, alpha, case["A"], ld, case["B"], ld, beta,
                               case["C"], ld, rows, cols)

    def error_of(prec):
        C.copy_(C0)
        call(prec, C)()
        torch.cuda.synchronize()
        got = C.view(n, ld)[torch.from_numpy(cols).to(dev), torch.from_numpy(rows).to(dev)]
        return oracle.normwise_rel_err(got.double().cpu().numpy(), ref)

    prewarm(torch, args.prewarm_s)
    results = {}
    forms = ["fp32"] if args.no_forms else ["fp32", "bf16x3", "fp16s"]
    flush = torch.empty(512 * 2 ** 20 // 4, dtype=torch.float32, device=dev)
    for prec in forms:
        if mg.config_count(prec) == 0:
            continue
        # Timed first, right after the pre-warm or the previous form's
        # timing: the host work of the error check leaves the GPU idle long
        # enough for its clock to drop.
        log("%s: timing ..." % prec)
        ms = timed(call(prec, C), args.steps, args.warmup, stream)
        err = error_of(prec)
        log("%s: sampled normwise error %.3e" % (prec, err))
        cold = cold_time(call(prec, C), args.cold_reps, stream, flush) if args.cold_reps else None
        results[prec] = dict(ms=ms, cold_ms=cold, tflops=flops / ms / 1e9, err=err,
                             cfg=mg.default_config(prec, "N", "N", n, n, n))
        log("%s: %.3f ms/call warm, %s ms cold, %.1f TFLOP/s" %
            (prec, ms, "%.3f" % cold if cold else "-", results[prec]["tflops"]))

    if args.copy_calibration:
        src = torch.empty(2 ** 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    f32 = results["fp32"]
    f32_call = call("fp32", C)
    f32["median_ms"] = None if args.no_single_calls else \
        per_call_ms(f32_call, max(20, args.steps), stream)
    log("fp32: median of single calls %s ms; sampling the clock ..." % f32["median_ms"])
    f32["clock"] = None if (args.no_clock or under_profiler()) else clock_under_load(f32_call)
    line = {
        "metric": METRIC,
        "value": round(f32["tflops"], 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sgemm NN M=N=K=%d lda=ldb=ldc=%d alpha=1.5 beta=-0.5 "
                               "uniform[-1,1) seed 0" % (n, ld),
                   "M": n, "N": n, "K": n, "trans": "NN", "ld": ld,
                   "tile_config": f32["cfg"]},
        "pct_of_fp32_mfma_peak": round(100.0 * f32["tflops"] / PEAK["fp32"], 2),
        "fp32_normwise_err": f32["err"],
        "value_timing": "warm: K back-to-back launches between HIP events on the launch stream; "
                        "the cache-flushed median (L2 and MALL overwritten before each launch, "
                        "the paper's method) is fp32_cold_ms and roofline.cold; the 16-bit forms' "
                        "speedups likewise (speedup_vs_fp32 warm, speedup_vs_fp32_cold flushed)",
        "fp32_cold_ms": f32["cold_ms"],
        "fp32_median_ms": None if f32["median_ms"] is None else round(f32["median_ms"], 4),
        "gpu_clock": f32["clock"],
    }
    key = "sgemm_f32_nn_%d" % n
    traffic = measured_traffic(key, "fp32")
    line["roofline"] = {"bound": "mfma", "achieved": round(f32["tflops"], 3),
                        "peak": PEAK["fp32"], "unit": "TFLOP/s",
                        "frac": round(f32["tflops"] / PEAK["fp32"], 4),
                        "traffic": traffic,
                        "kernel": "sgemm_f32_kernel (one launch per step)",
                        "source": "2MNK / ms_per_step: HIP events on the launch stream around "
                                  "the K timed back-to-back launches (warm L2 and MALL)"}
    if f32["cold_ms"]:
        line["roofline"]["cold"] = {
            "ms": round(f32["cold_ms"], 4), "achieved": round(flops / f32["cold_ms"] / 1e9, 3),
            "frac": round(flops / f32["cold_ms"] / 1e9 / PEAK["fp32"], 4),
            "source": "median of %d single launches, each after 512 MB are written "
                      "(L2 and MALL flushed, the paper's cache-flushed method)" % args.cold_reps}
    if "bf16x3" in results:
        b = results["bf16x3"]
        line["bf16x3"] = {"tflops": round(b["tflops"], 3), "ms": round(b["ms"], 4),
                          "cold_ms": b["cold_ms"],
                          "speedup_vs_fp32": round(f32["ms"] / b["ms"], 3),
                          "speedup_vs_fp32_cold": (round(f32["cold_ms"] / b["cold_ms"], 3)
                                                   if f32["cold_ms"] and b["cold_ms"] else None),
                          "normwise_err": b["err"],
                          "both_within_1e-5": bool(b["err"] <= 1e-5 and f32["err"] <= 1e-5),
                          "mfma_frac": round(3 * b["tflops"] / PEAK["bf16"], 4)}
    if "fp16s" in results:
        h = results["fp16s"]
        line["fp16s"] = {"tflops": round(h["tflops"], 3), "ms": round(h["ms"], 4),
                         "cold_ms": h["cold_ms"],
                         "speedup_vs_fp32": round(f32["ms"] / h["ms"], 3),
                         "speedup_vs_fp32_cold": (round(f32["cold_ms"] / h["cold_ms"], 3)
                                                  if f32["cold_ms"] and h["cold_ms"] else None),
                         "normwise_err": h["err"],
                         "mfma_frac": round(h["tflops"] / PEAK["fp16"], 4)}

    if not (args.no_forms or args.no_wide_range):
        line["wide_range_inputs"] = bench_wide_range(args, mg, torch, oracle, synth, n)
    line["small_256"] = bench_small(args, mg, torch)
    if not (args.no_vendor or args.no_forms):
        line["vendor_blas"] = bench_vendor(args, torch, n, alpha, beta)
    if not args.no_grouped:
        line["grouped"] = bench_grouped(args, mg, torch)
    if not args.no_dense:
        line["dense_layer"] = bench_dense(args, mg, torch)
    if not args.no_mlp:
        line["mlp_training"] = bench_mlp(args, mg, torch)
    if not args.no_splitk:
        line["split_k"] = bench_splitk(args, mg, torch)
    if not args.no_thin:
        line["thin"] = bench_thin(args, mg, torch, oracle, synth)
    if not (args.no_prepacked or args.no_forms):
        line["prepacked_b"] = bench_prepacked(args, mg, torch, n)
    if not args.no_sweep:
        line["config2"] = bench_sweep(args, mg, torch, oracle, synth)
    if not (args.no_sweep or args.no_forms):
        line["config3_2048"] = bench_forms_2048(args, mg, torch, oracle, synth)

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(oracle, case, n, alpha, beta, ld)
        line["cpu_baseline"]["single_thread_1024"] = cpu_single_thread(oracle, synth)
    print(json.dumps(line), flush=True)


def cpu_baseline(oracle, case, n, alpha, beta, ld, target_s=12.0):
    """The FP64 oracle, as it is, on columns 0..J-1 of the same product:
    a 128-column pilot sets J for about `target_s` seconds of work, then
    the J-column run is timed (every output is one n-long FP64 dot)."""
    def run(J):
        t0 = time.perf_counter()
        oracle.sgemm("N", "N", n, J, n, alpha, case["A"], ld, case["B"], ld, beta,
                     case["C"], ld)
        return time.perf_counter() - t0
    pilot = min(n, 128)
    t_pilot = run(pilot)
    J = int(max(pilot, min(n, pilot * target_s / max(t_pilot, 1e-3))))
    log("cpu baseline: oracle on %d columns ..." % J)
    dt = run(J)
    return {"value": round(2.0 * n * n * J / dt / 1e12, 6), "unit": "TFLOP/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "FP64 oracle, columns 0..%d of the same %d^3 NN product "
                      "(%d x %d outputs), %.1f s" % (J - 1, n, n, J, dt),
            "host": host_info()}


def host_info():
    """The host the oracle ran on: CPU model, logical CPUs, the CPUs this
    process may run on, and the oracle's OpenMP thread count."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for l in f:
                if l.startswith("model name"):
                    model = l.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": affinity,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def oracle_gflops(oracle, c, target_s=0.6):
    """The FP64 oracle's rate on columns 0..J-1 of case c (J from a pilot
    for about target_s seconds); the whole op(A) is still converted."""
    M, N, K = c["M"], c["N"], c["K"]

    def run(J):
        t0 = time.perf_counter()
        oracle.sgemm(c["transA"], c["transB"], M, J, K, c["alpha"], c["A"], c["lda"], c["B"],
                     c["ldb"], c["beta"], c["C"], c["ldc"])
        return time.perf_counter() - t0
    pilot = min(N, 32)
    t = run(pilot)
    J = int(max(pilot, min(N, pilot * target_s / max(t, 1e-3))))
    dt = run(J)
    return round(2.0 * M * J * K / dt / 1e9, 3)


def cpu_single_thread(oracle, synth, n=1024):
    """The oracle on one thread at n^3 (NN, ld n+16, alpha 1.5, beta -0.5)."""
    c = synth.sgemm_case(0, "N", "N", n, n, n, alpha=1.5, beta=-0.5, pad=16)
    default = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.sgemm("N", "N", n, n, n, 1.5, c["A"], c["lda"], c["B"], c["ldb"], -0.5, c["C"],
                     c["ldc"])
        dt = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(default)
    return {"value": round(2.0 * n ** 3 / dt / 1e12, 6), "unit": "TFLOP/s", "cores": 1,
            "sample": "FP64 oracle, %d^3 NN, whole product, %.1f s" % (n, dt)}


def bench_small(args, mg, torch):
    """256^3 NN, ld 256, alpha 1, beta 0: the latency-bound end (one small
    grid of work-groups); reported in microseconds per call."""
    import numpy as np
    import synth
    n = 256
    c = synth.sgemm_case(0, "N", "N", n, n, n, pad=0)
    A, B, C = (torch.from_numpy(c[k]).cuda() for k in ("A", "B", "C"))
    fn = lambda: mg.sgemm("N", "N", n, n, n, 1.0, A, n, B, n, 0.0, C, n)
    stream = torch.cuda.current_stream()
    ms = timed(fn, 200, 20, stream, min_ms=50)
    med = per_call_ms(fn, 50, stream)
    # The same calls replayed from a HIP graph: the device-side rate, without
    # the Python binding's per-call cost.
    graph_us = None
    if not under_profiler():
        try:
            graph_us = graph_us_per_call(fn, torch, stream)
        except Exception as e:      # context only: never lose the bench line
            log("256^3 graph timing skipped: %r" % (e,))
    return {"workload": "sgemm NN 256^3 ld 256 alpha 1 beta 0 fp32",
            "us_per_call": round(1000 * ms, 2), "median_us": round(1000 * med, 2),
            "graph_us_per_call": graph_us,
            "tflops": round(2.0 * n ** 3 / ms / 1e9, 3),
            "tile_config": mg.default_config("fp32", "N", "N", n, n, n)}


def graph_us_per_call(fn, torch, stream, reps=100):
    """Microseconds per call of `reps` calls of fn captured in one graph
    (a warm-up call on a side stream first, as torch's capture expects)."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    return round(1000 * timed(g.replay, 10, 2, stream) / reps, 2)


def bench_wide_range(args, mg, torch, oracle, synth, n):
    """The three paths on sign-random inputs of magnitude 2**U[-8, 8] (NN,
    lda = rows + 16, alpha 1, beta 0): time and sampled normwise error, so
    that the 16-bit forms' speedups are stated at equal error on inputs
    spanning 16 binades."""
    c = synth.sgemm_case(0, "N", "N", n, n, n, dist="loguni")
    ld = c["lda"]
    dev = torch.device("cuda:0")
    A = torch.from_numpy(c["A"]).to(dev)
    B = torch.from_numpy(c["B"]).to(dev)
    C = torch.zeros(c["C"].size, dtype=torch.float32, device=dev)
    rows, cols = synth.sample_entries(2, n, n, 2048)
    ref = oracle.sgemm_entries("N", "N", n, n, n, 1.0, c["A"], ld, c["B"], ld, 0.0, c["C"], ld,
                               rows, cols)
    stream = torch.cuda.current_stream()
    out = {"workload": "sgemm NN %d^3 lda=ldb=ldc=%d alpha=1 beta=0, sign-random 2**U[-8,8], "
                       "seed 0" % (n, ld)}
    for prec in ("fp32", "bf16x3", "fp16s"):
        fn = lambda: mg.sgemm("N", "N", n, n, n, 1.0, A, ld, B, ld, 0.0, C, ld, precision=prec)
        fn()
        torch.cuda.synchronize()
        got = C.view(n, ld)[torch.from_numpy(cols).to(dev), torch.from_numpy(rows).to(dev)]
        err = oracle.normwise_rel_err(got.double().cpu().numpy(), ref)
        ms = timed(fn, args.steps, args.warmup, stream, min_ms=50)
        out[prec] = {"ms": round(ms, 4), "tflops": round(2.0 * n ** 3 / ms / 1e9, 3),
                     "normwise_err": err}
        log("wide-range inputs %s: %.3f ms, sampled normwise error %.3e" % (prec, ms, err))
    for prec in ("bf16x3", "fp16s"):
        out[prec]["speedup_vs_fp32"] = round(out["fp32"]["ms"] / out[prec]["ms"], 3)
    out["bf16x3"]["both_within_1e-5"] = bool(out["bf16x3"]["normwise_err"] <= 1e-5 and
                                             out["fp32"]["normwise_err"] <= 1e-5)
    return out


def bench_vendor(args, torch, n, alpha, beta):
    """Context, not a target: the same FP32 products through torch.addmm
    (ROCm's BLAS libraries), TF32-style reduced precision disabled, on
    unpadded square operands."""
    torch.backends.cuda.matmul.allow_tf32 = False
    stream = torch.cuda.current_stream()
    out = {"library": "torch.addmm %s (ROCm BLAS), fp32" % torch.__version__}
    for size, steps, warmup in ((n, args.steps, args.warmup), (256, 200, 20)):
        g = torch.Generator(device="cuda").manual_seed(0)
        A = torch.rand(size, size, device="cuda", generator=g) * 2 - 1
        B = torch.rand(size, size, device="cuda", generator=g) * 2 - 1
        C = torch.rand(size, size, device="cuda", generator=g) * 2 - 1
        D = torch.empty_like(C)
        fn = lambda: torch.addmm(C, A, B, beta=beta, alpha=alpha, out=D)
        ms = timed(fn, steps, warmup, stream, min_ms=50)
        out["n%d" % size] = {"ms": round(ms, 4), "tflops": round(2.0 * size ** 3 / ms / 1e9, 3)}
        del A, B, C, D
    log("vendor fp32: %s" % out)
    return out


def bench_grouped(args, mg, torch):
    """512 independent GEMMs, M, N, K uniform on {16..512}, transA N/T, alpha
    = beta = 1: a tuned plan replayed from its HIP graph against one library
    launch per GEMM."""
    import ctypes
    import numpy as np
    import synth
    shapes = synth.grouped_problems(0, 512, 16, 512)
    data = synth.grouped_data(shapes, seed=1)
    sizes = [d[k].size for d in data for k in ("A", "B", "C")]
    offs, tot = [], 0
    for sz in sizes:
        offs.append(tot)
        tot += (sz + 63) // 64 * 64
    host = np.zeros(tot, dtype=np.float32)
    for k, (d, key) in enumerate((d, key) for d in data for key in ("A", "B", "C")):
        host[offs[k]:offs[k] + d[key].size] = d[key]
    init = torch.from_numpy(host).cuda()
    arena = init.clone()
    base = arena.data_ptr()
    probs = []
    for i, (sh, d) in enumerate(zip(shapes, data)):
        probs.append(dict(sh, alpha=1.0, beta=1.0, A=base + 4 * offs[3 * i], lda=d["lda"],
                          B=base + 4 * offs[3 * i + 1], ldb=d["ldb"],
                          C=base + 4 * offs[3 * i + 2], ldc=d["ldc"]))
    flops = sum(2.0 * p["M"] * p["N"] * p["K"] for p in probs)
    # Algorithmic bytes: A and B read once, C read (beta = 1) and written once.
    nbytes = sum(4.0 * (p["M"] * p["K"] + p["K"] * p["N"] + 2 * p["M"] * p["N"]) for p in probs)
    stream = torch.cuda.current_stream()
    L = mg.lib()
    h = stream.cuda_stream
    out = {"workload": "512 GEMMs, M,N,K ~ U{16..512}, transA N/T, alpha=beta=1, seed 0",
           "gflop_per_step": round(flops / 1e9, 3), "gbytes_per_step": round(nbytes / 1e9, 4)}
    for prec in ("fp32", "bf16x3"):
        cfg = None if args.grouped_defaults else mg.tune_grouped(probs, prec, reps=3)[0]
        arena.copy_(init)
        plan = mg.GroupedPlan(probs, prec, bucket_configs=cfg)
        ms_graph = timed(lambda: plan.launch(stream), args.steps, args.warmup, stream, min_ms=50)
        pcode = mg.PRECISIONS[prec]
        calls = [(p["transA"].encode(), p["transB"].encode(), p["M"], p["N"], p["K"],
                  ctypes.c_float(p["alpha"]), p["A"], p["lda"], p["B"], p["ldb"],
                  ctypes.c_float(p["beta"]), p["C"], p["ldc"], h, pcode, -1) for p in probs]

        def eager():
            for c in calls:
                L.mgemm_sgemm_ex(*c)
        ms_eager = timed(eager, max(3, args.steps // 4), 2, stream)
        info = plan.info()
        plan.close()
        out[prec] = {"bucket_configs": cfg if cfg is not None else "library defaults",
                     "tiles": info["tiles"],
                     "workgroups": info["workgroups"],
                     "graph_ms": round(ms_graph, 4), "tflops": round(flops / ms_graph / 1e9, 3),
                     "gbs": round(nbytes / ms_graph / 1e6, 1),
                     "hbm_frac": round(nbytes / ms_graph / 1e6 / HBM_PEAK_GBS, 4),
                     "eager_ms": round(ms_eager, 4),
                     "eager_tflops": round(flops / ms_eager / 1e9, 3),
                     "speedup_vs_eager": round(ms_eager / ms_graph, 3)}
        log("grouped %s: graph %.3f ms (%.1f TFLOP/s), one launch per GEMM %.3f ms" %
            (prec, ms_graph, flops / ms_graph / 1e9, ms_eager))
    return out


def bench_dense(args, mg, torch):
    """Dense layer Y = X W (X 8192 x 1024, W 1024 x 4096) forward + hand-written
    backward (dX = G W^T, dW = X^T G): three GEMMs per step."""
    import synth
    X, W, G = synth.dense_layer(0, 8192, 1024, 4096)
    Xd = torch.from_numpy(X).cuda().requires_grad_()
    Wd = torch.from_numpy(W).cuda().requires_grad_()
    Gd = torch.from_numpy(G).cuda()
    flops = 3 * 2.0 * 8192 * 1024 * 4096
    out = {"workload": "X 8192x1024, W 1024x4096, fwd + bwd (3 GEMMs)"}
    stream = torch.cuda.current_stream()
    for prec in ("fp32", "bf16x3"):
        def step():
            Xd.grad = None
            Wd.grad = None
            mg.linear(Xd, Wd, precision=prec).backward(Gd)
        ms = timed(step, max(5, args.steps // 2), 2, stream, min_ms=50)
        out[prec] = {"ms": round(ms, 4), "tflops": round(flops / ms / 1e9, 3)}
        log("dense layer %s: %.3f ms per fwd+bwd (%.1f TFLOP/s)" % (prec, ms, flops / ms / 1e9))
    return out


def bench_mlp(args, mg, torch):
    """Sustained rate of multilayer-perceptron training (the paper's
    application, Section 4): batch 8192, widths 1024 -> 4096 -> 4096 ->
    1024, tanh hidden layers, squared-error loss, one gradient-descent step
    per batch with the update fused into the weight-gradient products.  The
    rate counts the products' flops; the step's time includes the
    elementwise work."""
    import synth
    batch, widths, lr = 8192, [1024, 4096, 4096, 1024], 1e-3
    X, T, Ws = synth.mlp_case(0, batch, widths)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    flops = mg.mlp_step_flops(batch, widths)
    out = {"workload": "MLP batch 8192, widths 1024-4096-4096-1024, tanh, MSE, SGD lr 1e-3",
           "gflop_per_step": round(flops / 1e9, 3)}
    stream = torch.cuda.current_stream()
    for prec in ("fp32", "bf16x3"):
        net = mg.MLP([torch.from_numpy(W).cuda() for W in Ws], precision=prec)
        first = float(net.step(Xd, Td, lr))
        ms = timed(lambda: net.step(Xd, Td, lr), max(5, args.steps // 2), 2, stream, min_ms=50)
        last = float(net.step(Xd, Td, lr))
        out[prec] = {"ms_per_step": round(ms, 4), "tflops": round(flops / ms / 1e9, 3),
                     "loss_first": round(first, 6), "loss_last": round(last, 6)}
        log("mlp %s: %.3f ms per step (%.1f TFLOP/s), loss %.5f -> %.5f"
            % (prec, ms, flops / ms / 1e9, first, last))
        del net
    return out


def bench_splitk(args, mg, torch):
    """Products with few tiles and a long k range (NN, ld = rows + 16, alpha
    1.5, beta -0.5, uniform inputs): the library's choice (split-K) against
    the same product unsplit on 64 x 64 x 32 tiles (configuration 12, the
    rule's pick without split-K) and, at 256^2, the small-product kernel
    (configuration 9); the same for the two 16-bit forms."""
    import synth
    stream = torch.cuda.current_stream()
    out = {}
    for (M, N, K), other in (((1024, 1024, 8192), 12), ((512, 512, 16384), 12),
                             ((256, 256, 65536), 9)):
        c = synth.sgemm_case(0, "N", "N", M, N, K, alpha=1.5, beta=-0.5)
        A, B, C = (torch.from_numpy(c[k]).cuda() for k in ("A", "B", "C"))
        res = {"default_config": mg.default_config("fp32", "N", "N", M, N, K)}
        for name, cfg in (("default", -1), ("unsplit_config_%d" % other, other)):
            ms = timed(lambda: mg.sgemm("N", "N", M, N, K, 1.5, A, c["lda"], B, c["ldb"], -0.5, C,
                                        c["ldc"], config=cfg), max(10, args.steps), 3, stream,
                       min_ms=50)
            res[name] = {"ms": round(ms, 4), "tflops": round(2.0 * M * N * K / ms / 1e9, 3)}
        res["speedup"] = round(res["unsplit_config_%d" % other]["ms"] / res["default"]["ms"], 3)
        # The 16-bit forms: the library's choice (split-K) against the
        # fastest unsplit configuration the library had chosen before
        # split-K existed (BF16x3 in-staging 64 x 64, FP16 packed 128 x 128).
        for prec, unsplit in (("bf16x3", 3), ("fp16s", 11)):
            r = {"default_config": mg.default_config(prec, "N", "N", M, N, K)}
            for name, cfg in (("default", -1), ("unsplit_config_%d" % unsplit, unsplit)):
                ms = timed(lambda: mg.sgemm("N", "N", M, N, K, 1.5, A, c["lda"], B, c["ldb"], -0.5,
                                            C, c["ldc"], precision=prec, config=cfg),
                           max(10, args.steps), 3, stream, min_ms=50)
                r[name] = {"ms": round(ms, 4), "tflops": round(2.0 * M * N * K / ms / 1e9, 3)}
            r["speedup"] = round(r["unsplit_config_%d" % unsplit]["ms"] / r["default"]["ms"], 3)
            res[prec] = r
        out["%dx%dx%d" % (M, N, K)] = res
        log("split-K %dx%dx%d: %.1f TFLOP/s (config %d), unsplit %.1f; bf16x3 %.1f (%.2fx), "
            "fp16s %.1f (%.2fx)" %
            (M, N, K, res["default"]["tflops"], res["default_config"],
             res["unsplit_config_%d" % other]["tflops"], res["bf16x3"]["default"]["tflops"],
             res["bf16x3"]["speedup"], res["fp16s"]["default"]["tflops"],
             res["fp16s"]["speedup"]))
        del A, B, C
    return out


def bench_thin(args, mg, torch, oracle, synth):
    """FP32 products with at most 8 columns (or rows) of C (ld = rows + 16,
    alpha 1.5, beta -0.5, uniform inputs): the library's choice (the thin
    path) against split-K (configuration 11, the choice before it); rate in
    algorithmic bytes (op(A), op(B) read once, C read and written once) and
    the normwise error of the whole product against the oracle."""
    import numpy as np
    stream = torch.cuda.current_stream()
    out = {"workload": "FP32, ld = rows + 16, alpha 1.5, beta -0.5, uniform[-1,1) seed 0; "
                       "bytes = 4 (MK + KN + 2MN)"}
    for (M, N, K, ta, tb) in ((8192, 1, 8193, "N", "N"), (8192, 8, 8193, "N", "N"),
                              (8192, 1, 8193, "T", "N"), (8192, 1, 8193, "T", "T"),
                              (8192, 8, 8193, "T", "T"),
                              (1, 8193, 8193, "N", "N"),
                              (4096, 1, 4097, "N", "N")):
        c = synth.sgemm_case(0, ta, tb, M, N, K, alpha=1.5, beta=-0.5)
        A, B, C0 = (torch.from_numpy(c[k]).cuda() for k in ("A", "B", "C"))
        C = C0.clone()
        nbytes = 4.0 * (M * K + K * N + 2 * M * N)
        res = {}
        for name, cfg in (("thin", -1), ("split_k_config_11", 11)):
            fn = lambda: mg.sgemm(ta, tb, M, N, K, 1.5, A, c["lda"], B, c["ldb"], -0.5, C,
                                  c["ldc"], config=cfg)
            C.copy_(C0)
            fn()
            torch.cuda.synchronize()
            ref = oracle.sgemm(ta, tb, M, N, K, 1.5, c["A"], c["lda"], c["B"], c["ldb"], -0.5,
                               c["C"], c["ldc"])
            flat, ldc = C.cpu().numpy(), c["ldc"]
            got = np.stack([flat[j * ldc:j * ldc + M] for j in range(N)], axis=1)
            err = oracle.normwise_rel_err(got.astype(np.float64), ref)
            ms = timed(fn, max(10, args.steps), 3, stream, min_ms=50)
            res[name] = {"us": round(ms * 1e3, 2), "gbs": round(nbytes / ms / 1e6, 1),
                         "normwise_err": float("%.3e" % err)}
        res["speedup"] = round(res["split_k_config_11"]["us"] / res["thin"]["us"], 3)
        key = "%s%s %dx%dx%d" % (ta, tb, M, N, K)
        out[key] = res
        log("thin %s: %.1f us (%.0f GB/s), split-K %.1f us" %
            (key, res["thin"]["us"], res["thin"]["gbs"], res["split_k_config_11"]["us"]))
        del A, B, C0, C
    return out


def bench_sweep(args, mg, torch, oracle, synth):
    """The FP32 path over the sweep of square sizes {1000, 1024, 2048, 3001,
    4096, 4097} in all four trans pairs: ld = stored rows + 16 (the fixed
    stride of the paper's Section 4 method), alpha 1.5, beta -0.5, uniform
    inputs from seed 0 (square operands, so one set of arrays serves every
    trans pair).  Per product: warm TFLOP/s over a few launches, sampled
    normwise error against the oracle; per size: the oracle's own rate on
    this host."""
    import numpy as np
    stream = torch.cuda.current_stream()
    out = {"workload": "sgemm M=N=K in {1000,1024,2048,3001,4096,4097} x NN/NT/TN/TT, "
                       "ld = rows + 16, alpha 1.5, beta -0.5, uniform[-1,1) seed 0",
           "tile_config": "mgemm_default_config for the whole product; 4097 runs as its "
                          "4096^2 whole-tile block (configuration 8) plus one-row and "
                          "one-column remainders on the thin path"}
    steps, warmup = max(5, args.steps // 2), 3
    for n in (1000, 1024, 2048, 3001, 4096, 4097):
        c = synth.sgemm_case(0, "N", "N", n, n, n, alpha=1.5, beta=-0.5)
        ld = c["lda"]
        A, B, C0 = (torch.from_numpy(c[k]).cuda() for k in ("A", "B", "C"))
        C = C0.clone()
        rows, cols = synth.sample_entries(3, n, n, 256)
        res = {"oracle_gflops": oracle_gflops(oracle, c)}
        for ta, tb in (("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")):
            fn = lambda: mg.sgemm(ta, tb, n, n, n, 1.5, A, ld, B, ld, -0.5, C, ld)
            C.copy_(C0)
            fn()
            torch.cuda.synchronize()
            got = C.view(n, ld)[torch.from_numpy(cols).cuda(), torch.from_numpy(rows).cuda()]
            ref = oracle.sgemm_entries(ta, tb, n, n, n, 1.5, c["A"], ld, c["B"], ld, -0.5, c["C"],
                                       ld, rows, cols)
            err = oracle.normwise_rel_err(got.double().cpu().numpy(), ref)
            ms = timed(fn, steps, warmup, stream, min_ms=50)
            res[ta + tb] = {"ms": round(ms, 4), "tflops": round(2.0 * n ** 3 / ms / 1e9, 3),
                            "normwise_err": float("%.3e" % err),
                            "tile_config": mg.default_config("fp32", ta, tb, n, n, n)}
        out[str(n)] = res
        log("sweep %d: %s" % (n, " ".join("%s %.1f" % (k, v["tflops"]) for k, v in res.items()
                                          if isinstance(v, dict))))
        del A, B, C0, C
    return out


def bench_forms_2048(args, mg, torch, oracle, synth):
    """The precision-form shapes at 2048^3: NN, ld 2064, alpha 1, beta 0,
    sign-random magnitudes 2**U[-8, 8]; the three paths' time and sampled
    normwise error, and the oracle's rate on the same product."""
    n = 2048
    c = synth.sgemm_case(0, "N", "N", n, n, n, dist="loguni")
    ld = c["lda"]
    A, B = torch.from_numpy(c["A"]).cuda(), torch.from_numpy(c["B"]).cuda()
    C = torch.zeros(c["C"].size, dtype=torch.float32, device="cuda")
    rows, cols = synth.sample_entries(4, n, n, 1024)
    ref = oracle.sgemm_entries("N", "N", n, n, n, 1.0, c["A"], ld, c["B"], ld, 0.0, c["C"], ld,
                               rows, cols)
    stream = torch.cuda.current_stream()
    out = {"workload": "sgemm NN 2048^3 ld 2064 alpha 1 beta 0, sign-random 2**U[-8,8], seed 0",
           "oracle_gflops": oracle_gflops(oracle, c)}
    for prec in ("fp32", "bf16x3", "fp16s"):
        fn = lambda: mg.sgemm("N", "N", n, n, n, 1.0, A, ld, B, ld, 0.0, C, ld, precision=prec)
        fn()
        torch.cuda.synchronize()
        got = C.view(n, ld)[torch.from_numpy(cols).cuda(), torch.from_numpy(rows).cuda()]
        err = oracle.normwise_rel_err(got.double().cpu().numpy(), ref)
        ms = timed(fn, max(10, args.steps), args.warmup, stream, min_ms=50)
        out[prec] = {"ms": round(ms, 4), "tflops": round(2.0 * n ** 3 / ms / 1e9, 3),
                     "normwise_err": float("%.3e" % err)}
    for prec in ("bf16x3", "fp16s"):
        out[prec]["speedup_vs_fp32"] = round(out["fp32"]["ms"] / out[prec]["ms"], 3)
    log("forms 2048^3: %s" % {k: v for k, v in out.items() if isinstance(v, dict)})
    del A, B, C
    return out


def bench_prepacked(args, mg, torch, n):
    """BF16x3 at n^3 NN with op(B) packed once (mgemm_pack_b) against the
    ordinary call, which packs both operands every time; same inputs as the
    headline product (alpha 1.5, beta -0.5).  Then scaled FP16 the same way,
    and FP32 TT with op(B) transposed once."""
    import synth
    c = synth.sgemm_case(0, "N", "N", n, n, n, alpha=1.5, beta=-0.5)
    A, B, C = (torch.from_numpy(c[k]).cuda() for k in ("A", "B", "C"))
    stream = torch.cuda.current_stream()
    ld = c["lda"]
    ms_call = timed(lambda: mg.sgemm("N", "N", n, n, n, 1.5, A, ld, B, ld, -0.5, C, ld,
                                     precision="bf16x3"), args.steps, args.warmup, stream,
                    min_ms=50)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    pb = mg.PackedB("N", n, n, B, ld)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_pack = e0.elapsed_time(e1)
    ms_packed = timed(lambda: pb.sgemm("N", n, 1.5, A, ld, -0.5, C, ld), args.steps,
                      args.warmup, stream, min_ms=50)
    pb.close()
    flops = 2.0 * n ** 3
    out = {"workload": "bf16x3 NN %d^3, op(B) packed once" % n,
           "ordinary_ms": round(ms_call, 4), "packed_b_ms": round(ms_packed, 4),
           "packed_b_tflops": round(flops / ms_packed / 1e9, 3),
           "speedup": round(ms_call / ms_packed, 3), "pack_once_ms": round(ms_pack, 4)}
    log("pre-packed B bf16x3 %d^3: %.3f ms per call against %.3f (pack once %.3f ms)"
        % (n, ms_packed, ms_call, ms_pack))
    # Scaled FP16: the handle also keeps op(B)'s panel exponents.
    ms_f16 = timed(lambda: mg.sgemm("N", "N", n, n, n, 1.5, A, ld, B, ld, -0.5, C, ld,
                                    precision="fp16s"), args.steps, args.warmup, stream,
                   min_ms=50)
    with mg.PackedB("N", n, n, B, ld, precision="fp16s") as pf:
        ms_f16p = timed(lambda: pf.sgemm("N", n, 1.5, A, ld, -0.5, C, ld), args.steps,
                        args.warmup, stream, min_ms=50)
    out["fp16s"] = {"ordinary_ms": round(ms_f16, 4), "packed_b_ms": round(ms_f16p, 4),
                    "packed_b_tflops": round(flops / ms_f16p / 1e9, 3),
                    "speedup": round(ms_f16 / ms_f16p, 3)}
    log("pre-packed B fp16s %d^3: %.3f ms per call against %.3f" % (n, ms_f16p, ms_f16))
    # FP32: op(B) stored transposed ('T', the same buffer read as N x K),
    # transposed once into the k-contiguous layout; A 'T' too, so the
    # ordinary call is the TT product and the packed one runs as TN.
    ms_tt = timed(lambda: mg.sgemm("T", "T", n, n, n, 1.5, A, ld, B, ld, -0.5, C, ld),
                  args.steps, args.warmup, stream, min_ms=50)
    with mg.PackedB("T", n, n, B, ld, precision="fp32") as p32:
        ms_ttp = timed(lambda: p32.sgemm("T", n, 1.5, A, ld, -0.5, C, ld), args.steps,
                       args.warmup, stream, min_ms=50)
    out["fp32_tt"] = {"ordinary_ms": round(ms_tt, 4), "packed_b_ms": round(ms_ttp, 4),
                      "packed_b_tflops": round(flops / ms_ttp / 1e9, 3),
                      "speedup": round(ms_tt / ms_ttp, 3)}
    log("pre-packed B fp32 TT %d^3: %.3f ms per call against %.3f" % (n, ms_ttp, ms_tt))
    del A, B, C
    return out


if __name__ == "__main__":
    main()
