"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Two executables are built with ``-fsanitize=address,undefined`` and
``-fno-sanitize-recover=all`` (any report aborts the run):

* ``tests/sanitize/host_checks.cpp`` with the library's HIP-free host
  sources (argument validation, operand overlap, default tile rules, the
  split-K plan, the grouped list schedule and batch aliasing).  Its answers
  are compared with the library itself (through the C ABI, for calls that
  never reach a device), with the BLAS rules as the header states them, and
  with brute force.
* ``tests/sanitize/oracle_check.c`` with the FP64 oracle, every operand in a
  heap block of exactly its referenced extent (an unreferenced operand is
  NULL).  Its results must equal the ordinary oracle build bitwise.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import paper_1912_04379_amd as mg
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1912_04379_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")

I64_MAX = 2 ** 63 - 1


@pytest.fixture(scope="module")
def bins(tmp_path_factory):
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("gcc / g++ not available")
    d = tmp_path_factory.mktemp("sanitized")
    host = str(d / "host_checks")
    subprocess.run(["g++", "-std=c++17", *SAN, "-I" + os.path.join(ROOT, "include"),
                    "-I" + CSRC, os.path.join(HERE, "sanitize", "host_checks.cpp"),
                    os.path.join(CSRC, "validate.cpp"), os.path.join(CSRC, "defaults.cpp"),
                    os.path.join(CSRC, "schedule.cpp"), "-o", host], check=True)
    orc = str(d / "oracle_check")
    subprocess.run(["gcc", "-std=c11", *SAN, "-fopenmp", "-ffp-contract=off",
                    os.path.join(HERE, "sanitize", "oracle_check.c"),
                    os.path.join(ROOT, "oracle", "oracle.c"), "-o", orc], check=True)
    return {"host": host, "oracle": orc, "dir": d}


def _host(bins, lines):
    r = subprocess.run([bins["host"]], input="\n".join(lines) + "\n", capture_output=True,
                       text=True, env=ENV, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]
    out = r.stdout.strip().splitlines()
    assert len(out) == len(lines)
    return out


# ---- argument validation -----------------------------------------------------

def _blas_status(ta, tb, M, N, K, alpha, A, lda, B, ldb, C, ldc):
    """The BLAS argument rules of the C ABI, restated: the number of the
    first illegal argument (negated), or 0."""
    is_t = {"N": 0, "n": 0, "T": 1, "t": 1, "C": 1, "c": 1}
    if ta not in is_t:
        return -1
    if tb not in is_t:
        return -2
    if M < 0:
        return -3
    if N < 0:
        return -4
    if K < 0:
        return -5
    rows_a = K if is_t[ta] else M
    rows_b = N if is_t[tb] else K
    reads = alpha != 0 and K > 0 and M > 0 and N > 0
    if reads and A == 0:
        return -7
    if lda < max(1, rows_a):
        return -8
    if reads and B == 0:
        return -9
    if ldb < max(1, rows_b):
        return -10
    if M > 0 and N > 0 and C == 0:
        return -12
    if ldc < max(1, M):
        return -13
    return 0


def _extent(p, rows, cols, ld):
    return p, min(p + ((cols - 1) * ld + rows) * 4, 2 ** 64 - 1)


def _overlap(ta, tb, M, N, K, alpha, A, lda, B, ldb, C, ldc):
    if alpha == 0 or K == 0 or M == 0 or N == 0:
        return 0
    t = lambda x: x in "TtCc"
    clo, chi = _extent(C, M, N, ldc)
    for p, r, c, ld in ((A, K if t(ta) else M, M if t(ta) else K, lda),
                        (B, N if t(tb) else K, K if t(tb) else N, ldb)):
        lo, hi = _extent(p, r, c, ld)
        if lo < chi and clo < hi:
            return 1
    return 0


def _random_calls(seed, n):
    rng = np.random.default_rng(seed)
    trans = list("NnTtCcX")
    sizes = [-1, 0, 1, 5, 37, 4096, 2 ** 40]
    calls = []
    for _ in range(n):
        ta, tb = rng.choice(trans), rng.choice(trans)
        M, N, K = (int(rng.choice(sizes)) for _ in range(3))
        alpha = float(rng.choice([0.0, 1.5]))
        beta = float(rng.choice([0.0, 1.0, -0.5]))
        base = [0, 1 << 32, 1 << 40, 3 << 40]
        A, B, C = (int(rng.choice(base)) for _ in range(3))

        def ld(rows):
            return int(rng.choice([0, 1, max(rows - 1, 0), max(rows, 1), max(rows, 1) + 16,
                                   2 ** 62, I64_MAX]))
        is_t = lambda x: x in "TtCc"
        lda = ld(K if is_t(ta) else M)
        ldb = ld(N if is_t(tb) else K)
        ldc = ld(M)
        calls.append((str(ta), str(tb), M, N, K, alpha, A, lda, B, ldb, beta, C, ldc))
    return calls


def test_validation_and_overlap_match_the_library_and_the_blas_rules(bins):
    calls = _random_calls(0, 4000)
    lines = []
    for (ta, tb, M, N, K, al, A, lda, B, ldb, be, C, ldc) in calls:
        lines.append("V %s %s %d %d %d %r %d %d %d %d %r %d %d" %
                     (ta, tb, M, N, K, al, A, lda, B, ldb, be, C, ldc))
        lines.append("O %s %s %d %d %d %r %d %d %d %d %d %d" %
                     (ta, tb, M, N, K, al, A, lda, B, ldb, C, ldc))
    out = _host(bins, lines)
    L = mg.lib()
    checked_lib = 0
    for i, (ta, tb, M, N, K, al, A, lda, B, ldb, be, C, ldc) in enumerate(calls):
        v, o = int(out[2 * i]), int(out[2 * i + 1])
        assert v == _blas_status(ta, tb, M, N, K, al, A, lda, B, ldb, C, ldc), calls[i]
        if v == 0:
            assert o == _overlap(ta, tb, M, N, K, al, A, lda, B, ldb, C, ldc), calls[i]
        # The library's own answer, for calls that stop before any device
        # work: an illegal argument, a quick return, or an overlap.
        quick = M == 0 or N == 0 or ((al == 0 or K == 0) and be == 1.0)
        if v != 0 or quick or o:
            st = L.mgemm_sgemm_ex(ta.encode(), tb.encode(), M, N, K, al, A, lda, B, ldb, be, C,
                                  ldc, None, 0, -1)
            assert st == (v if v else (0 if quick else 105)), (calls[i], st)
            checked_lib += 1
    assert checked_lib > 1000


# ---- default rules and split-K plan -----------------------------------------

def test_default_rules_match_the_library(bins):
    dims = [1, 64, 100, 256, 300, 512, 1000, 1024, 2048, 3001, 4096, 4097, 4608, 6144, 8192,
            12288, 65536]
    rng = np.random.default_rng(1)
    shapes = [(int(rng.choice(dims)), int(rng.choice(dims)), int(rng.choice(dims)))
              for _ in range(600)]
    cases = [(p, ta, tb, M, N, K) for (M, N, K) in shapes for p in (0, 1, 2)
             for ta, tb in (("N", "N"), ("T", "T"), ("N", "T"))]
    out = _host(bins, ["D %d %s %s %d %d %d" % c for c in cases])
    L = mg.lib()
    assert L.mgemm_clear_choices() == 0
    for c, got in zip(cases, out):
        p, ta, tb, M, N, K = c
        want = L.mgemm_default_config(p, ta.encode(), tb.encode(), M, N, K)
        assert int(got) == want, c
        assert 0 <= want < L.mgemm_config_count(p)


def test_edge_split_rule(bins):
    """The FP32 edge split as documented: M and N each a multiple of 256 or
    at most 64 past one (at least one past), a whole-tile block of at least
    256 x 256 holding at least 2^37 flops; otherwise the product stays whole
    and Mm, Nm are left alone."""
    dims = [1, 255, 256, 257, 300, 320, 321, 1024, 1025, 2048, 2049, 4096, 4097, 4100, 4160,
            4161, 6145, 8192, 8193, 8256, 8257]
    rng = np.random.default_rng(5)
    cases = [("N", "N", 4097, 4097, 4097), ("T", "T", 8193, 8193, 8193),
             ("N", "T", 4096, 4096, 4096), ("N", "N", 4161, 4097, 4097),
             ("N", "N", 4097, 4097, 1024)]
    cases += [(str(rng.choice(list("NT"))), str(rng.choice(list("NT"))), int(rng.choice(dims)),
               int(rng.choice(dims)), int(rng.choice([512, 4096, 4097, 8193])))
              for _ in range(800)]
    out = _host(bins, ["E %s %s %d %d %d" % c for c in cases])
    split_seen = 0
    for c, line in zip(cases, out):
        ta, tb, M, N, K = c
        flag, mm, nn = (int(x) for x in line.split())
        rm, rn = M % 256, N % 256
        want = (rm <= 64 and rn <= 64 and (rm or rn) and M - rm >= 256 and N - rn >= 256
                and 2 * (M - rm) * (N - rn) * K >= 2 ** 37)
        assert bool(flag) == bool(want), (c, line)
        if flag:
            split_seen += 1
            assert (mm, nn) == (M - rm, N - rn), c
        else:
            assert (mm, nn) == (-1, -1), c
    assert split_seen >= 20
    assert out[0].split() == ["1", "4096", "4096"] and out[1].split() == ["1", "8192", "8192"]
    assert out[2].split()[0] == "0" and out[3].split()[0] == "0" and out[4].split()[0] == "0"


def test_split_k_plan_invariants(bins):
    rng = np.random.default_rng(2)
    cases = [(int(rng.integers(1, 9000)), int(rng.integers(1, 9000)),
              int(rng.integers(1, 70000)), int(rng.choice([1, 80, 256, 304])))
             for _ in range(3000)]
    cases += [(1, 1, 2 ** 40, 256), (2 ** 31, 2 ** 31, 2 ** 40, 256), (0, 5, 5, 256),
              (5, 5, 0, 256), (5, 5, 5, 0)]
    out = _host(bins, ["S %d %d %d %d" % c for c in cases])
    for (M, N, K, cus), line in zip(cases, out):
        small, splits, kc, ws = (int(x) for x in line.split())
        if splits == 0:
            continue
        assert splits >= 2 and kc % 32 == 0 and kc >= 256
        assert (splits - 1) * kc < K <= splits * kc
        assert ws == splits * M * N * 4
        bm = 64 if small else 128
        tiles = -(-M // bm) * -(-N // bm)
        assert tiles * splits <= 0xffffffff


# ---- grouped schedule and batch aliasing --------------------------------------

def test_list_schedule_is_longest_first_to_least_loaded(bins):
    rng = np.random.default_rng(3)
    cases = []
    for _ in range(200):
        n = int(rng.integers(0, 400))
        G = int(rng.integers(1, 70))
        cost = np.sort(rng.integers(1, 50, n).astype(float) * 32.0)[::-1]
        cases.append((G, cost))
    lines = ["L %d %d %s" % (G, len(c), " ".join("%.17g" % float(x) for x in c)) for G, c in cases]
    out = _host(bins, lines)
    for (G, cost), line in zip(cases, out):
        got = [int(x) for x in line.split()]
        load = [0.0] * G
        for i, c in enumerate(cost):
            w = min(range(G), key=lambda g: (load[g], g))
            assert got[i] == w
            load[w] += c
        if len(cost):
            assert max(load) <= cost.sum() / G + cost.max() + 1e-9


def test_queue_partition_covers_every_tile_once(bins):
    """The grouped plan's work queues: every tile of every problem in exactly
    one queue, each queue costliest first, the queues balanced within one
    chunk, and a problem costing more than a queue's share spread over
    several queues."""
    rng = np.random.default_rng(5)
    cases = []
    for _ in range(150):
        n = int(rng.integers(0, 60))
        nq = int(rng.integers(1, 9))
        nt = rng.integers(0, 70, n)
        cost = rng.integers(1, 40, n).astype(float) * 16.0
        cases.append((nq, nt, cost))
    cases.append((8, np.array([1000]), np.array([5.0])))          # one large problem
    cases.append((8, np.array([3, 1]), np.array([7.0, 100.0])))   # fewer chunks than queues
    lines = ["Q %d %d %s %s" % (nq, len(nt), " ".join(str(int(x)) for x in nt),
                                " ".join("%.17g" % x for x in cost)) for nq, nt, cost in cases]
    out = _host(bins, lines)
    for (nq, nt, cost), line in zip(cases, out):
        queues = []
        for part in line.split(";"):
            f = [int(x) for x in part.split()]
            assert f[0] * 2 == len(f) - 1
            queues.append(list(zip(f[1::2], f[2::2])))
        assert len(queues) == nq
        seen = sorted(pt for q in queues for pt in q)
        assert seen == sorted((p, t) for p in range(len(nt)) for t in range(int(nt[p])))
        total = float(sum(nt[p] * cost[p] for p in range(len(nt))))
        loads = []
        for q in queues:
            c = [cost[p] for p, _ in q]
            assert all(c[i] >= c[i + 1] for i in range(len(c) - 1))
            loads.append(sum(c))
        if total > 0:
            # a chunk costs at most a queue's share plus one tile
            assert max(loads) <= 2 * total / nq + cost.max() + 1e-9
    line = out[-2]
    assert all(int(part.split()[0]) == 125 for part in line.split(";"))


def test_batch_aliasing_against_brute_force(bins):
    rng = np.random.default_rng(4)
    cases, lines = [], []
    for _ in range(400):
        nc, na = int(rng.integers(0, 12)), int(rng.integers(0, 12))

        def iv():
            lo = int(rng.integers(0, 4000)) * 4
            return lo, lo + int(rng.integers(1, 300)) * 4
        cs = [(*iv(), i) for i in range(nc)]
        ab = [(*iv(), int(rng.integers(0, max(nc, 1)))) for _ in range(na)]
        cases.append((cs, ab))
        lines.append("B %d %d %s" % (nc, na, " ".join("%d %d %d" % e for e in cs + ab)))
    out = _host(bins, lines)
    for (cs, ab), line in zip(cases, out):
        who, kind = (int(x) for x in line.split())
        cc = [c for c in cs if any(c is not d and c[0] < d[1] and d[0] < c[1] for d in cs)]
        ca = [c for c in cs if any(c[0] < x[1] and x[0] < c[1] for x in ab)]
        if not cc and not ca:
            assert who == -1 and kind == 0
        elif cc:
            assert kind == 1 and who in [c[2] for c in cc]
        else:
            assert kind == 2 and who in [c[2] for c in ca]


# ---- the oracle ---------------------------------------------------------------

def _extent_n(rows, cols, ld):
    return 0 if rows <= 0 or cols <= 0 else (cols - 1) * ld + rows


ORACLE_CASES = [
    ("N", "N", 37, 29, 53, 1.5, -0.5, 3),
    ("T", "N", 16, 17, 18, 1.0, 0.0, 0),
    ("N", "T", 40, 1, 70, -2.0, 1.0, 5),
    ("T", "T", 1, 33, 9, 1.5, -0.5, 1),
    ("N", "N", 1, 1, 1, 1.0, 0.0, 0),
    ("N", "N", 8, 6, 0, 1.5, -0.5, 2),      # K = 0: C <- beta C, A and B unread
    ("T", "N", 8, 6, 5, 0.0, 2.0, 2),       # alpha = 0
    ("N", "T", 0, 6, 5, 1.0, 0.0, 2),       # M = 0
    ("T", "T", 7, 0, 5, 1.0, 0.0, 2),       # N = 0
    ("C", "c", 25, 31, 64, 1.5, -0.5, 7),
]


@pytest.mark.parametrize("case", ORACLE_CASES, ids=lambda c: "%s%s_%dx%dx%d" % c[:5])
def test_oracle_under_sanitizers_matches_the_ordinary_build(bins, case):
    ta, tb, M, N, K, alpha, beta, pad = case
    c = synth.sgemm_case(5, ta, tb, M, N, K, alpha=alpha, beta=beta, pad=pad)
    t = lambda x: x in "TtCc"
    use_product = alpha != 0 and K > 0
    na = _extent_n(K if t(ta) else M, M if t(ta) else K, c["lda"]) if use_product else 0
    nb = _extent_n(N if t(tb) else K, K if t(tb) else N, c["ldb"]) if use_product else 0
    nc = _extent_n(M, N, c["ldc"]) if beta != 0 else 0
    rng = np.random.default_rng(6)
    count = 5 if M > 0 and N > 0 else 0
    rows = rng.integers(0, max(M, 1), count).astype(np.int64)
    cols = rng.integers(0, max(N, 1), count).astype(np.int64)
    f = bins["dir"] / ("case_%s%s_%d_%d_%d.bin" % case[:5])
    o = bins["dir"] / ("out_%s%s_%d_%d_%d.bin" % case[:5])
    with open(f, "wb") as fh:
        fh.write(("%s %s %d %d %d %r %r %d %d %d %d %d %d %d\n%d %d %d\n" %
                  (ta, tb, M, N, K, float(np.float32(alpha)), float(np.float32(beta)),
                   c["lda"], c["ldb"], c["ldc"], count, int(use_product), int(use_product),
                   int(beta != 0), na, nb, nc)).encode())
        if use_product:
            fh.write(c["A"][:na].tobytes())
            fh.write(c["B"][:nb].tobytes())
        if beta != 0:
            fh.write(c["C"][:nc].tobytes())
        fh.write(rows.tobytes())
        fh.write(cols.tobytes())
    r = subprocess.run([bins["oracle"], str(f), str(o)], capture_output=True, text=True,
                       env=ENV, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]
    out = np.fromfile(o, np.float64)
    ldo = max(1, M)
    full = out[:ldo * N].reshape(N, ldo)[:, :M].T if N > 0 else np.zeros((M, 0))
    ent = out[ldo * N: ldo * N + count]
    dfull = out[ldo * N + count:].reshape(N, ldo)[:, :M].T if N > 0 else np.zeros((M, 0))
    args = (ta, tb, M, N, K, alpha, c["A"], c["lda"], c["B"], c["ldb"], beta, c["C"], c["ldc"])
    assert np.array_equal(full, oracle.sgemm(*args), equal_nan=True)
    if count:
        assert np.array_equal(ent, oracle.sgemm_entries(*args, rows, cols), equal_nan=True)
    wide = (ta, tb, M, N, K, float(np.float32(alpha)), c["A"].astype(np.float64), c["lda"],
            c["B"].astype(np.float64), c["ldb"], float(np.float32(beta)),
            c["C"].astype(np.float64), c["ldc"])
    assert np.array_equal(dfull, oracle.dgemm(*wide), equal_nan=True)


def test_thin_plan_rule(bins):
    """The thin-product plan as documented: at most 8 columns of C (else at
    most 8 rows, through the transpose), at least 256 on the other side,
    K >= 256, leading dimensions and M within the buffer path's limit and
    the referenced extents of A and B below 2^31 bytes, and with a
    k-contiguous large operand and more than 4 of them, 2^25 elements of it; the k pieces are
    multiples of 64, at most 64 of them, every one non-empty, for about
    eight work-groups per CU; a small operand with non-adjacent k elements
    is gathered first when the large one is k-contiguous and r >= 2 or it
    holds at least 2^25 elements; the
    workspace holds S partial products and the gathered operand."""
    lim, rng_bytes = (1 << 21) - 64, 0x7ffffff0
    rng = np.random.default_rng(7)
    cases = [("N", "N", 8192, 1, 8193, 8192, 8193, 8192, 256),
             ("N", "N", 1, 8193, 8193, 1, 8193, 1, 256),
             ("N", "T", 4096, 8, 4097, 4096, 8, 4096, 256),
             ("N", "N", 4096, 9, 4097, 4096, 4097, 4096, 256),
             ("N", "N", 255, 1, 4096, 255, 4096, 255, 256),
             ("N", "N", 4096, 1, 255, 4096, 255, 4096, 256),
             ("N", "N", 4096, 1, 4096, lim + 1, 4096, 4096, 256),
             ("N", "N", 4096, 1, 4096, 4096, 4096, lim + 1, 256),
             ("T", "N", 300000, 2, 2000, 2000, 2000, 300000, 256),
             ("N", "N", 4096, 1, 4096, 4096, 4096, 4096, 0)]
    dims = [1, 2, 3, 5, 8, 9, 16, 255, 256, 257, 1000, 4097, 8193]
    for _ in range(1500):
        ta, tb = str(rng.choice(list("NT"))), str(rng.choice(list("NT")))
        M, N = int(rng.choice(dims)), int(rng.choice(dims))
        K = int(rng.choice([64, 255, 256, 300, 4097, 65536, 1 << 20]))
        lda = (K if ta == "T" else M) + int(rng.choice([0, 3, 64]))
        ldb = (N if tb == "T" else K) + int(rng.choice([0, 5]))
        cases.append((ta, tb, M, N, K, lda, ldb, M + int(rng.choice([0, 7])),
                      int(rng.choice([1, 80, 256]))))
    out = _host(bins, ["T %s %s %d %d %d %d %d %d %d" % c for c in cases])
    seen, seen_gather = {0: 0, 1: 0}, {0: 0, 1: 0}
    for c, line in zip(cases, out):
        ta, tb, M, N, K, lda, ldb, ldc, cus = c
        ok, rows, S, kc, nbytes, gather = (int(x) for x in line.split())
        cols = N <= 8
        few_rows = not cols and M <= 8
        P = M if cols else N
        aext = K + (M - 1) * lda if ta == "T" else M + (K - 1) * lda
        bext = N + (K - 1) * ldb if tb == "T" else K + (N - 1) * ldb
        kcontig = (ta == "T") if cols else (tb == "N")
        r = N if cols else M
        want = ((cols or few_rows) and P >= 256 and K >= 256 and cus >= 1
                and max(lda, ldb, ldc, M) <= lim and 4 * aext < rng_bytes and 4 * bext < rng_bytes
                and not (kcontig and r > 4 and P * K < 2 ** 25))
        assert bool(ok) == want, (c, line)
        if not ok:
            assert (rows, S, kc, nbytes, gather) == (0, 0, 0, 0, 0), (c, line)
            continue
        seen[rows] += 1
        assert rows == int(few_rows), c
        assert kc % 64 == 0 and 1 <= S <= 64, (c, line)
        assert (S - 1) * kc < K <= S * kc, (c, line)        # every piece non-empty
        strided = (tb == "T" and ldb != 1) if cols else (ta == "N" and lda != 1)
        assert gather == int(strided and kcontig and (r >= 2 or P * K >= 2 ** 25)), (c, line)
        seen_gather[gather] += 1
        assert nbytes == 4 * (S * M * N + (K * r if gather else 0)), (c, line)
        blocks = -(-P // (16 if kcontig else 64))
        target = min(64, -(-8 * cus // blocks))
        assert S <= target, (c, line)                      # at most the target pieces
        assert S == -(-K // kc) and kc == -(-(-(-K // target)) // 64) * 64, (c, line)
    assert seen[0] >= 30 and seen[1] >= 30, seen
    assert seen_gather[0] >= 30 and seen_gather[1] >= 8, seen_gather
    assert out[0].split()[:2] == ["1", "0"] and out[1].split()[:2] == ["1", "1"]
    assert out[2].split()[0] == "1"
    for line in out[3:10]:
        assert line.split()[0] == "0", line
