"""Grouped persistent launch: many uneven GEMMs in one kernel, replayed
from a HIP graph, with per-bucket tile variants from the tuner."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1912_04379_amd as mg
import synth
from form_bars import stat_bar
from paper_1912_04379_amd import _lib
from paper_1912_04379_amd import grouped as gp

FA, FB, FC = 0x10000000, 0x20000000, 0x30000000


def fake(ta="N", M=8, N=8, K=8, A=FA, B=FB, C=FC, alpha=1.0, beta=0.0, lda=None):
    return dict(transA=ta, transB="N", M=M, N=N, K=K, alpha=alpha, beta=beta, A=A,
                lda=lda if lda is not None else (K if ta == "T" else M), B=B, ldb=K, C=C, ldc=M)


def create(problems, precision=0, configs=None):
    arr = gp._problem_array(problems)
    cfg = (ctypes.c_int * 4)(*configs) if configs else None
    plan = ctypes.c_void_p()
    bad, bst = ctypes.c_int64(), ctypes.c_int()
    st = mg.lib().mgemm_grouped_plan_create_ex(arr, len(problems), precision, cfg, None,
                                               ctypes.byref(plan), ctypes.byref(bad),
                                               ctypes.byref(bst))
    return st, bad.value, bst.value


# ---- CPU: validation happens before any device work -------------------------

def test_bad_problem_is_reported_with_its_index():
    probs = [fake(), fake(A=FA + 4096, C=FC + 4096), fake(M=-3, C=FC + 8192)]
    st, bad, bst = create(probs)
    assert st == _lib.ERR_BAD_PROBLEM and bad == 2 and bst == -3
    probs[2] = fake(C=FC + 8192, lda=2)            # lda < M
    st, bad, bst = create(probs)
    assert (st, bad, bst) == (_lib.ERR_BAD_PROBLEM, 2, -8)


def test_overlapping_outputs_are_rejected():
    st, bad, bst = create([fake(), fake(A=FA + 4096, C=FC + 128)])
    assert st == _lib.ERR_BAD_PROBLEM and bst == _lib.ERR_ALIAS
    # one problem's C over another problem's A
    st, bad, bst = create([fake(), fake(A=FA + 4096, C=FA + 64)])
    assert st == _lib.ERR_BAD_PROBLEM and bst == _lib.ERR_ALIAS


def test_unsupported_precision_and_variant():
    assert create([fake()], precision=2)[0] == _lib.ERR_UNSUPPORTED
    assert create([fake()], configs=[0, 0, 9, 0])[0] == _lib.ERR_UNSUPPORTED
    assert gp.variant_count("fp32") == 3 and gp.variant_count("fp16s") == 0
    assert gp.variant_info("bf16x3", 1)["bm"] > 0


def test_buckets():
    assert [gp.bucket(m, n) for m, n in ((16, 64), (65, 10), (200, 256), (257, 16))] == \
        [0, 1, 2, 3]


def test_destroy_null_plan():
    assert mg.lib().mgemm_grouped_plan_destroy(None) == _lib.ERR_BAD_PLAN


# ---- GPU --------------------------------------------------------------------

def make_batch(count=512, seed=0, lo=16, hi=512):
    """Problems and host data; every matrix sits 256-byte aligned in one
    device arena."""
    import torch
    shapes = synth.grouped_problems(seed, count, lo, hi)
    data = synth.grouped_data(shapes, seed=seed + 1)
    sizes = []
    for d in data:
        sizes += [d["A"].size, d["B"].size, d["C"].size]
    offs, tot = [], 0
    for s in sizes:
        offs.append(tot)
        tot += (s + 63) // 64 * 64
    host = np.zeros(tot, dtype=np.float32)
    k = 0
    for d in data:
        for key in ("A", "B", "C"):
            host[offs[k]:offs[k] + d[key].size] = d[key]
            k += 1
    arena = torch.from_numpy(host).cuda()
    base = arena.data_ptr()
    problems = []
    k = 0
    for s, d in zip(shapes, data):
        p = dict(s, alpha=1.0, beta=1.0, lda=d["lda"], ldb=d["ldb"], ldc=d["ldc"])
        p["A"], p["B"], p["C"] = base + 4 * offs[k], base + 4 * offs[k + 1], base + 4 * offs[k + 2]
        p["_c_off"], p["_c_size"] = offs[k + 2], d["C"].size
        k += 3
        problems.append(p)
    return problems, data, arena, host


def c_of(arena_host, p):
    return arena_host[p["_c_off"]:p["_c_off"] + p["_c_size"]]


def check_batch(problems, data, out_host, precision, tol):
    worst = 0.0
    for p, d in zip(problems, data):
        args = (p["transA"], p["transB"], p["M"], p["N"], p["K"], p["alpha"], d["A"], d["lda"],
                d["B"], d["ldb"], p["beta"], d["C"], d["ldc"])
        ref = oracle.sgemm(*args)
        got = c_of(out_host, p).reshape(p["N"], p["ldc"])[:, :p["M"]].T.astype(np.float64)
        err = oracle.normwise_rel_err(got, ref)
        worst = max(worst, err)
        assert err <= tol, "problem %s: %.3e" % ((p["M"], p["N"], p["K"], p["transA"]), err)
        if precision == "fp32":
            bound = oracle.gamma(p["K"] + 2, 2.0 ** -23) * oracle.abs_product(*args)
            assert np.all(np.abs(got - ref) <= bound)
        else:
            # Against the split form's FP64 emulation: FP32 accumulation
            # error only, elementwise and (statistically) normwise.
            emu = oracle.bf16x3(*args)
            bound = oracle.gamma(3 * p["K"] + 2, 2.0 ** -23) * (1 + 2.0 ** -6) * \
                oracle.abs_product(*args)
            assert np.all(np.abs(got - emu) <= bound)
            assert oracle.normwise_rel_err(got, emu) <= stat_bar(p["K"])
    return worst


@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16x3", 1e-5)])
@pytest.mark.parametrize("buckets", [None, [0, 1, 2, 2], [2, 2, 2, 2]])
def test_512_uneven_problems_against_oracle(precision, tol, buckets):
    """Library defaults (one launch), every variant at once (three
    launches) and the largest tile throughout."""
    import torch
    print("grouped 512 problems", precision, buckets, flush=True)
    problems, data, arena, host = make_batch()
    with mg.GroupedPlan(problems, precision, bucket_configs=buckets) as plan:
        info = plan.info()
        assert info["tiles"] > 512 and info["workgroups"] > 0
        plan.launch()
        torch.cuda.synchronize()
    worst = check_batch(problems, data, arena.cpu().numpy(), precision, tol)
    print("worst normwise error %.3e" % worst, flush=True)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_graph_replay_equals_direct_launch_bitwise(precision):
    """Several replays, with eager work and synchronisations in between,
    each from the same initial C: every replay equals the direct launch."""
    import torch
    problems, data, arena, host = make_batch(count=96, seed=5)
    init = torch.from_numpy(host).cuda()
    with mg.GroupedPlan(problems, precision) as plan:
        plan.run()
        torch.cuda.synchronize()
        direct = arena.clone()
        for r in range(4):
            arena.copy_(init)
            scratch = torch.randn(1 << 20, device="cuda")
            scratch.mul_(2.0).sum().item()          # unrelated eager work
            plan.launch()
            torch.cuda.synchronize()
            assert torch.equal(arena, direct), "replay %d differs" % r


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_back_to_back_launches_find_the_queues_reset(precision):
    """Work-groups take tiles from counters that the last work-group of a
    launch puts back to zero.  Launches queued back to back on one stream
    (graph replays and direct runs, C restored between them on the same
    stream, no host synchronisation) must each compute every tile: a tile
    left out would keep C's initial value."""
    import torch
    problems, data, arena, host = make_batch(count=64, seed=9)
    init = torch.from_numpy(host).cuda()
    with mg.GroupedPlan(problems, precision) as plan:
        plan.run()
        torch.cuda.synchronize()
        direct = arena.clone()
        outs = []
        for r in range(12):
            arena.copy_(init)
            plan.launch() if r % 3 else plan.run()
            outs.append(arena.clone())
        torch.cuda.synchronize()
    for r, o in enumerate(outs):
        assert torch.equal(o, direct), "launch %d differs" % r
    check_batch(problems, data, direct.cpu().numpy(), precision, 1e-5)


@pytest.mark.gpu
@pytest.mark.parametrize("shapes", [[(20, 30, 40)], [(64, 64, 16)], [(130, 70, 50), (5, 5, 5)]])
def test_batches_with_fewer_tiles_than_queues(shapes):
    """One queue per XCD, but never more queues than work-groups: one tile,
    or a handful, still runs to completion."""
    import torch
    rng = np.random.default_rng(21)
    probs, keep, hosts = [], [], []
    for (M, N, K) in shapes:
        A, B, C = (synth.matrix(rng, r, c, r) for r, c in ((M, K), (K, N), (M, N)))
        t = [torch.from_numpy(x.copy()).cuda() for x in (A, B, C)]
        keep.append(t)
        hosts.append((A, B, C))
        probs.append(dict(transA="N", transB="N", M=M, N=N, K=K, alpha=1.25, beta=-0.5, A=t[0],
                          lda=M, B=t[1], ldb=K, C=t[2], ldc=M))
    for precision in ("fp32", "bf16x3"):
        for t, (A, B, C) in zip(keep, hosts):
            t[2].copy_(torch.from_numpy(C))
        with mg.GroupedPlan(probs, precision) as plan:
            for _ in range(3):
                for t, (A, B, C) in zip(keep, hosts):
                    t[2].copy_(torch.from_numpy(C))
                plan.launch()
            torch.cuda.synchronize()
        for p, (A, B, C), t in zip(probs, hosts, keep):
            ref = oracle.sgemm("N", "N", p["M"], p["N"], p["K"], p["alpha"], A, p["lda"], B,
                               p["ldb"], p["beta"], C, p["ldc"])
            got = t[2].cpu().numpy().reshape(p["N"], p["ldc"])[:, :p["M"]].T.astype(np.float64)
            assert oracle.normwise_rel_err(got, ref) <= 1e-5, (precision, p["M"], p["N"], p["K"])


@pytest.mark.gpu
def test_grouped_equals_single_calls_with_same_tile():
    """Variant 1 (128x128x16) is the single-call configuration 0: the same
    tile code, so the results are bitwise equal."""
    import torch
    problems, data, arena, host = make_batch(count=40, seed=7)
    init = torch.from_numpy(host).cuda()
    assert gp.variant_info("fp32", 1) == {"bm": 128, "bn": 128, "bk": 16}
    assert mg.config_info("fp32", 0)["bk"] == 16
    with mg.GroupedPlan(problems, "fp32", bucket_configs=[1, 1, 1, 1]) as plan:
        plan.launch()
        torch.cuda.synchronize()
    grouped = arena.clone()
    arena.copy_(init)
    for p in problems:
        mg.sgemm(p["transA"], p["transB"], p["M"], p["N"], p["K"], p["alpha"], p["A"], p["lda"],
                 p["B"], p["ldb"], p["beta"], p["C"], p["ldc"], config=0)
    torch.cuda.synchronize()
    assert torch.equal(arena, grouped)


# Grouped variant -> single-call configuration with the same tile code.
SAME_TILE = {"fp32": {0: 1, 1: 0, 2: 12}, "bf16x3": {0: 3, 1: 1}}


def check_variant(precision, variant, shapes, seed):
    """One plan of `shapes` ((M, N, K, transA, transB), padded leading
    dimensions, alpha 1.5, beta -0.75) with every bucket on `variant`:
    each C within the oracle's bar with its padding rows untouched and,
    where a single-call configuration runs the same tile, bitwise equal
    to that call."""
    import torch
    rng = np.random.default_rng(seed)
    probs, keep, hosts = [], [], []
    for (M, N, K, ta, tb) in shapes:
        lda = K + 3 if ta == "T" else M + 5
        ldb = N + 2 if tb == "T" else K + 1
        A = synth.matrix(rng, K, M, lda) if ta == "T" else synth.matrix(rng, M, K, lda)
        B = synth.matrix(rng, N, K, ldb) if tb == "T" else synth.matrix(rng, K, N, ldb)
        C = synth.matrix(rng, M, N, M + 2)
        t = [torch.from_numpy(x.copy()).cuda() for x in (A, B, C)]
        keep.append(t)
        hosts.append((A, B, C))
        probs.append(dict(transA=ta, transB=tb, M=M, N=N, K=K, alpha=1.5, beta=-0.75, A=t[0],
                          lda=lda, B=t[1], ldb=ldb, C=t[2], ldc=M + 2))
    with mg.GroupedPlan(probs, precision, bucket_configs=[variant] * 4) as plan:
        plan.launch()
        torch.cuda.synchronize()
    grouped = [t[2].clone() for t in keep]
    for p, (A, B, C), g in zip(probs, hosts, grouped):
        args = (p["transA"], p["transB"], p["M"], p["N"], p["K"], p["alpha"], A, p["lda"], B,
                p["ldb"], p["beta"], C, p["ldc"])
        ref = oracle.sgemm(*args)
        out = g.cpu().numpy().reshape(p["N"], p["ldc"])
        got = out[:, :p["M"]].T.astype(np.float64)
        case = (precision, variant, p["M"], p["N"], p["K"], p["transA"], p["transB"])
        assert oracle.normwise_rel_err(got, ref) <= 1e-5, case
        # the rows between M and ldc are not C: untouched
        assert np.array_equal(out[:, p["M"]:], C.reshape(p["N"], p["ldc"])[:, p["M"]:],
                              equal_nan=True), case
    cfg = SAME_TILE[precision].get(variant)
    if cfg is None:
        return
    vi = gp.variant_info(precision, variant)
    ci = mg.config_info(precision, cfg)
    assert (vi["bm"], vi["bn"], vi["bk"]) == (ci["bm"], ci["bn"], ci["bk"])
    for p, (A, B, C), t, g in zip(probs, hosts, keep, grouped):
        t[2].copy_(torch.from_numpy(C))
        mg.sgemm(p["transA"], p["transB"], p["M"], p["N"], p["K"], p["alpha"], p["A"], p["lda"],
                 p["B"], p["ldb"], p["beta"], p["C"], p["ldc"], precision=precision, config=cfg)
        torch.cuda.synchronize()
        # bit patterns: the NaN rows between M and ldc compare equal too
        assert torch.equal(t[2].view(torch.int32), g.view(torch.int32)), \
            (precision, variant, p["M"], p["N"], p["K"], p["transA"], p["transB"])


# Problems whose edge tiles leave whole 32-row or 32-column wave blocks (64
# for the 128 x 128 tiles) outside C: those waves stage their share of each
# slab but issue no MFMAs and store nothing.
SKIP_SHAPES = [(1, 300, 40, "N"), (300, 1, 40, "T"), (32, 97, 64, "N"), (97, 32, 33, "T"),
               (33, 160, 17, "N"), (160, 33, 100, "T"), (64, 65, 31, "N"), (65, 64, 48, "T"),
               (129, 129, 64, "N"), (16, 16, 16, "T"), (200, 70, 7, "N")]


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_waves_outside_c_skip_their_work(precision, variant):
    """Every variant on edge-heavy problems."""
    print("skipped waves", precision, variant, flush=True)
    check_variant(precision, variant, [sh + ("N",) for sh in SKIP_SHAPES], 31 + variant)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_every_trans_pair_in_one_batch(precision, variant):
    """A batch mixing all four (transA, transB) pairs, so every operand
    layout of the persistent kernel runs, on ragged shapes."""
    print("trans pairs", precision, variant, flush=True)
    rng = np.random.default_rng(41 + variant)
    shapes = []
    for i in range(24):
        M, N, K = (int(v) for v in rng.integers(1, 300, size=3))
        shapes.append((M, N, K, "NT"[i % 2], "NT"[(i // 2) % 2]))
    check_variant(precision, variant, shapes, 51 + variant)


@pytest.mark.gpu
def test_edge_problems_in_a_batch():
    """alpha = 0 (C = beta C, A holds NaN and is not read), beta = 0 with
    NaN in C, K = 0, an empty problem, and 1 x 1 x 1."""
    import torch
    rng = np.random.default_rng(3)
    specs = [(50, 40, 30, 0.0, 2.0), (70, 33, 20, 1.0, 0.0), (20, 20, 0, 1.5, -1.0),
             (0, 10, 10, 1.0, 1.0), (1, 1, 1, 1.0, 1.0), (300, 129, 65, -1.0, 0.5)]
    probs, keep, hosts = [], [], []
    for (M, N, K, al, be) in specs:
        A = synth.matrix(rng, M, K, max(1, M)) if K else np.zeros(1, np.float32)
        if al == 0.0:
            A = np.full_like(A, np.nan)
        B = synth.matrix(rng, K, N, max(1, K)) if K else np.zeros(1, np.float32)
        C = synth.matrix(rng, M, N, max(1, M)) if M else np.zeros(1, np.float32)
        if be == 0.0:
            C = np.full_like(C, np.nan)
        t = [torch.from_numpy(x.copy()).cuda() for x in (A, B, C)]
        keep.append(t)
        hosts.append((A, B, C))
        probs.append(dict(transA="N", transB="N", M=M, N=N, K=K, alpha=al, beta=be, A=t[0],
                          lda=max(1, M), B=t[1], ldb=max(1, K), C=t[2], ldc=max(1, M)))
    with mg.GroupedPlan(probs, "fp32") as plan:
        plan.launch()
        torch.cuda.synchronize()
    for p, (A, B, C), t in zip(probs, hosts, keep):
        M, N = p["M"], p["N"]
        if M == 0:
            continue
        ref = oracle.sgemm("N", "N", M, N, p["K"], p["alpha"], A, p["lda"], B, p["ldb"],
                           p["beta"], C, p["ldc"])
        got = t[2].cpu().numpy().reshape(N, p["ldc"])[:, :M].T.astype(np.float64)
        assert np.all(np.isfinite(got))
        assert oracle.normwise_rel_err(got, ref) <= 1e-6


@pytest.mark.gpu
def test_tuner_returns_valid_configs_and_plan_stays_correct():
    import torch
    problems, data, arena, host = make_batch(count=64, seed=11)
    init = torch.from_numpy(host).cuda()
    cfg, ms = mg.tune_grouped(problems, "fp32", reps=2)
    assert len(cfg) == 4 and all(0 <= c < 3 for c in cfg) and ms > 0
    arena.copy_(init)
    with mg.GroupedPlan(problems, "fp32", bucket_configs=cfg) as plan:
        plan.launch()
        torch.cuda.synchronize()
    check_batch(problems, data, arena.cpu().numpy(), "fp32", 1e-5)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_tune_cache_through_the_c_abi(tmp_path, monkeypatch, precision):
    """A plan made with a tune_cache path: the first call tunes (every C is
    kept as it was) and appends the choice for this device, version,
    precision and batch; the second reads it back without tuning; the plan
    computes the batch correctly."""
    import torch
    print("tune cache", precision, flush=True)
    problems, data, arena, host = make_batch(count=48, seed=12)
    init = torch.from_numpy(host).cuda()
    arena.copy_(init)
    cache = tmp_path / "tune.txt"
    log = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", str(log))
    plan = mg.GroupedPlan(problems, precision, tune_cache=str(cache))
    torch.cuda.synchronize()
    assert torch.equal(arena, init), "tuning left a C changed"
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    f = lines[0].split()
    assert f[:3] == ["mgemm-tune", "v1", "grouped"] and f[3].startswith("gfx950")
    assert int(f[4]) == torch.cuda.get_device_properties(0).multi_processor_count
    assert int(f[5]) == mg.version() and int(f[6]) == mg.PRECISIONS[precision]
    configs = [int(v) for v in f[8].split(",")]
    plan.close()
    plan = mg.GroupedPlan(problems, precision, tune_cache=str(cache))
    assert len(cache.read_text().splitlines()) == 1          # read, not tuned again
    text = log.read_text()
    assert "source=tuned" in text and "source=cache configs=%d,%d,%d,%d" % tuple(configs) in text
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    check_batch(problems, data, arena.cpu().numpy(), precision, 1e-5)


@pytest.mark.gpu
def test_plan_destroyed_twice_is_detected():
    problems, data, arena, host = make_batch(count=4, seed=2)
    plan = mg.GroupedPlan(problems, "fp32")
    handle = plan._plan
    plan.close()
    assert mg.lib().mgemm_grouped_plan_destroy(handle) == _lib.ERR_BAD_PLAN
    assert mg.lib().mgemm_grouped_plan_launch(handle, None) == _lib.ERR_BAD_PLAN
