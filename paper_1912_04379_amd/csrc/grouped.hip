// grouped.hip -- many independent GEMMs in one persistent launch.
//
// A plan holds, in device memory, one descriptor per problem (operands,
// sizes, trans flags, the tile variant chosen for its size bucket, its tile
// grid) and, per launch (one per tile variant in use), up to eight work
// queues of (problem, tile) references, one per XCD.  The host fills the
// queues: whole problems (a large one cut into runs of tiles) go to the
// queue with the least work so far, and each queue holds its tiles
// costliest first (cost ~ k slabs + a fixed per-tile share).  The kernel
// starts (CUs x work-groups per CU) work-groups; work-group w serves the
// queue of its XCD (w mod 8) by taking the next tile with an atomic
// counter, then helps the other queues in turn once its own is empty.  A
// tile's result does not depend on which work-group computes it or when,
// and every tile is written by exactly one work-group, so results are
// bitwise reproducible run to run and between the graph replay and a
// direct launch.  Taking tiles as work-groups free up balances the load
// against the tiles' real durations, which a static schedule could only
// estimate; keeping a problem on one XCD keeps its operands in that XCD's
// L2.  The last work-group to finish puts the counters back to zero, so
// every launch finds them zeroed.
//
// The plan records its launch into a HIP graph once; mgemm_grouped_plan_launch
// replays it.  mgemm_grouped_tune picks the variant of each size bucket by
// timing the whole batch (coordinate descent over buckets).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <string>
#include <tuple>
#include <unordered_set>
#include <vector>

#include "host_common.hpp"
#include "mgemm.h"
#include "rules.hpp"
#include "tile_f32.hpp"
#include "tile_lowp.hpp"

namespace mgemm {

// ---- tile variants of the persistent kernel (all 256 threads) -------------
using GF0 = CfgF32<64, 64, 16, 2, 2>;
using GF1 = CfgF32<128, 128, 16, 2, 2>;
using GF2 = CfgF32<64, 64, 32, 2, 2>;   // 32-deep slabs: half the barriers per MFMA
using GL0 = CfgLP<64, 64, 2, 2>;
using GL1 = CfgLP<128, 128, 2, 2>;
using GL2 = CfgLP<128, 64, 2, 2>;
constexpr int NUM_VARIANTS = 3;
constexpr int NUM_BUCKETS = 4;

struct VariantShape {
    int bm, bn, bk;
};

static VariantShape variant_shape(int precision, int v) {
    if (precision == MGEMM_PREC_FP32) {
        const VariantShape s[NUM_VARIANTS] = {{GF0::BM, GF0::BN, GF0::BK},
                                              {GF1::BM, GF1::BN, GF1::BK},
                                              {GF2::BM, GF2::BN, GF2::BK}};
        return s[v];
    }
    const VariantShape s[NUM_VARIANTS] = {{GL0::BM, GL0::BN, GL0::BK},
                                          {GL1::BM, GL1::BN, GL1::BK},
                                          {GL2::BM, GL2::BN, GL2::BK}};
    return s[v];
}

template <class Cfg>
constexpr int f32_lds() { return Cfg::SMEM_FLOATS * 4; }
template <class Cfg>
constexpr int lp_lds() { return 2 * 2 * (Cfg::BM + Cfg::BN) * Cfg::ROW_BYTES; }

// Default variant per size bucket (bucket = by max(M, N)): one variant for
// every bucket, so an untuned batch is one launch (measured fastest on a
// batch of 512 problems with M, N, K uniform on 16..512: FP32 64x64x32, 2%
// ahead of 64x64x16; BF16x3 128x128, level with 128x64).
static const int DEFAULT_F32[NUM_BUCKETS] = {2, 2, 2, 2};
static const int DEFAULT_LP[NUM_BUCKETS] = {1, 1, 1, 1};

// A tile's fixed cost (prologue, epilogue, the hand-over to the next tile)
// in units of one k slab of its own variant: least-squares fits of measured
// tile durations against their slab counts on the 512-problem batch (M, N,
// K uniform on 16..512).
static double tile_overhead_slabs(int precision, int v) {
    static const double f32[NUM_VARIANTS] = {0.5, 0.5, 0.5};
    static const double lp[NUM_VARIANTS] = {2.0, 4.0, 3.0};
    return precision == MGEMM_PREC_FP32 ? f32[v] : lp[v];
}

static int bucket_of(int64_t M, int64_t N) {
    const int64_t s = M > N ? M : N;
    return s <= 64 ? 0 : s <= 128 ? 1 : s <= 256 ? 2 : 3;
}

// ---- device descriptors ----------------------------------------------------
struct GroupedProblem {
    GemmDesc d;
    uint32_t tiles_m, tiles_n;
    int32_t ta, tb, variant, pad;
};

struct TileRef {
    uint32_t problem, tile;
};

template <int V>
using VariantF32 = typename std::tuple_element<V, std::tuple<GF0, GF1, GF2>>::type;
template <int V>
using VariantLP = typename std::tuple_element<V, std::tuple<GL0, GL1, GL2>>::type;

template <int PREC, int V>
constexpr int variant_lds() {
    if constexpr (PREC == MGEMM_PREC_FP32) return f32_lds<VariantF32<V>>();
    else return lp_lds<VariantLP<V>>();
}

// One persistent kernel per (precision, tile variant).  The queues of the
// launch are qstarts[q] .. qstarts[q+1]-1 of `tiles` (q < nq); counter q
// (counters[q * CTR_STRIDE]) is queue q's next ticket and counter nq counts
// finished work-groups.  Each counter has a 256-byte line of its own:
// atomics on one line are served one at a time, so counters sharing a line
// would serialise every work-group's draw.
// Thread 0 draws the ticket for the next tile when a tile starts, so the
// atomic's round trip overlaps the tile; the ticket is resolved, and handed
// to the work-group through LDS, when the tile is done.  The table pointers
// are kernel arguments, so every field of a problem is a wave-uniform
// scalar load, and the four operand layouts are inlined tile code, as in
// the single-call kernels.
constexpr uint32_t NO_TILE = 0xffffffffu;
constexpr uint32_t CTR_STRIDE = 64;

template <int PREC, int V>
__global__ __launch_bounds__(256, 2) void grouped_kernel(const GroupedProblem* __restrict__ probs,
                                                      const TileRef* __restrict__ tiles,
                                                      const uint32_t* __restrict__ qstarts,
                                                      uint32_t* __restrict__ counters, uint32_t nq) {
    extern __shared__ __attribute__((aligned(16))) char grouped_smem[];
    __shared__ uint32_t next_tile;
    // Thread 0's cursor: the queue it draws from and how many queues it has
    // not yet found empty.  Each queue is found empty at most once, so a
    // work-group draws at most (its tiles + nq) tickets.
    uint32_t q = blockIdx.x % nq, left = nq;
    auto resolve = [&](uint32_t ticket) -> uint32_t {
        for (;;) {
            if (ticket < qstarts[q + 1] - qstarts[q]) return qstarts[q] + ticket;
            q = q + 1 == nq ? 0 : q + 1;
            if (--left == 0) return NO_TILE;
            ticket = atomicAdd(&counters[q * CTR_STRIDE], 1u);
        }
    };
    if (threadIdx.x == 0) next_tile = resolve(atomicAdd(&counters[q * CTR_STRIDE], 1u));
    __syncthreads();
    uint32_t t = next_tile;
    while (t != NO_TILE) {
        uint32_t ticket = 0;
        if (threadIdx.x == 0) ticket = atomicAdd(&counters[q * CTR_STRIDE], 1u);
        const TileRef tr = tiles[t];
        const GroupedProblem& gp = probs[tr.problem];
        const GemmDesc d = gp.d;
        const uint32_t tm = tr.tile % gp.tiles_m, tn = tr.tile / gp.tiles_m;
        // The work-item index, opaque to the compiler in every iteration:
        // otherwise it hoists the tile code's per-lane addresses out of this
        // loop and keeps them all live across it (about 45 more VGPRs for
        // the 64 x 64 tile, and lower occupancy).
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        // op(A) is K-contiguous for A 'T'; op(B) is K-contiguous for B 'N'.
        if constexpr (PREC == MGEMM_PREC_FP32) {
            using Cfg = VariantF32<V>;
            const int64_t m0 = (int64_t)tm * Cfg::BM, n0 = (int64_t)tn * Cfg::BN;
            float* sm = reinterpret_cast<float*>(grouped_smem);
            if (!gp.ta && !gp.tb) tile_f32<Cfg, false, true, true, true>(d, m0, n0, sm, tid);
            else if (!gp.ta)      tile_f32<Cfg, false, false, true, true>(d, m0, n0, sm, tid);
            else if (!gp.tb)      tile_f32<Cfg, true, true, true, true>(d, m0, n0, sm, tid);
            else                  tile_f32<Cfg, true, false, true, true>(d, m0, n0, sm, tid);
        } else {
            using Cfg = VariantLP<V>;
            const int64_t m0 = (int64_t)tm * Cfg::BM, n0 = (int64_t)tn * Cfg::BN;
            if (!gp.ta && !gp.tb) tile_lowp<Cfg, Form::BF16X3, false, true, true, true>(d, m0, n0, grouped_smem, tid);
            else if (!gp.ta)      tile_lowp<Cfg, Form::BF16X3, false, false, true, true>(d, m0, n0, grouped_smem, tid);
            else if (!gp.tb)      tile_lowp<Cfg, Form::BF16X3, true, true, true, true>(d, m0, n0, grouped_smem, tid);
            else                  tile_lowp<Cfg, Form::BF16X3, true, false, true, true>(d, m0, n0, grouped_smem, tid);
        }
        __syncthreads();  // LDS is reused by the next tile; next_tile was read
        if (threadIdx.x == 0) next_tile = resolve(ticket);
        __syncthreads();
        t = next_tile;
    }
    // Every ticket this work-group drew has returned; the last work-group
    // out zeroes the counters for the next launch.
    if (threadIdx.x == 0 && atomicAdd(&counters[nq * CTR_STRIDE], 1u) == gridDim.x - 1) {
        for (uint32_t i = 0; i <= nq; ++i) atomicExch(&counters[i * CTR_STRIDE], 0u);
    }
}

template <int PREC, int V>
static const void* kernel_ptr() { return (const void*)grouped_kernel<PREC, V>; }

static const void* kernel_of(int precision, int v) {
    if (precision == MGEMM_PREC_FP32)
        return v == 0 ? kernel_ptr<MGEMM_PREC_FP32, 0>()
                      : v == 1 ? kernel_ptr<MGEMM_PREC_FP32, 1>() : kernel_ptr<MGEMM_PREC_FP32, 2>();
    return v == 0 ? kernel_ptr<MGEMM_PREC_BF16X3, 0>()
                  : v == 1 ? kernel_ptr<MGEMM_PREC_BF16X3, 1>() : kernel_ptr<MGEMM_PREC_BF16X3, 2>();
}

static int lds_of(int precision, int v) {
    if (precision == MGEMM_PREC_FP32)
        return v == 0 ? variant_lds<MGEMM_PREC_FP32, 0>()
                      : v == 1 ? variant_lds<MGEMM_PREC_FP32, 1>() : variant_lds<MGEMM_PREC_FP32, 2>();
    return v == 0 ? variant_lds<MGEMM_PREC_BF16X3, 0>()
                  : v == 1 ? variant_lds<MGEMM_PREC_BF16X3, 1>() : variant_lds<MGEMM_PREC_BF16X3, 2>();
}

// One launch of a plan: the kernel of one variant over its own queues.
struct VariantLaunch {
    int variant;
    uint32_t grid;
    uint32_t nq;          // queues (at most one per XCD, at most grid)
    int64_t starts_off;   // first of its nq + 1 offsets in the plan's starts table
    int64_t counters_off; // first of its (nq + 1) x CTR_STRIDE counter words
};

}  // namespace mgemm

// ---- the plan object ---------------------------------------------------------
struct mgemm_plan {
    int device = 0;
    int precision = 0;
    int64_t nprob = 0, ntiles = 0;
    uint32_t grid = 0;   // work-groups of the largest launch
    std::vector<mgemm::VariantLaunch> launches;   // in launch order
    mgemm::GroupedProblem* d_probs = nullptr;
    mgemm::TileRef* d_tiles = nullptr;
    uint32_t* d_starts = nullptr;   // per launch, nq + 1 queue offsets into d_tiles
    uint32_t* d_counters = nullptr; // per launch, nq tickets + 1 finished count, one line each
                                    // (zero between launches)
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace mgemm {

static std::mutex g_plans_mu;
static std::unordered_set<mgemm_plan*> g_plans;

static bool plan_live(const mgemm_plan* p) {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    return p && g_plans.count(const_cast<mgemm_plan*>(p));
}

static void plan_free(mgemm_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->capture) (void)hipStreamDestroy(p->capture);
    if (p->d_probs) (void)hipFree(p->d_probs);
    if (p->d_tiles) (void)hipFree(p->d_tiles);
    if (p->d_starts) (void)hipFree(p->d_starts);
    if (p->d_counters) (void)hipFree(p->d_counters);
    delete p;
}

static int hip_err(hipError_t e, const char* where) {
    (void)hipGetLastError();
    return fail(MGEMM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

static hipError_t launch_plan_kernel(const mgemm_plan* p, hipStream_t s) {
    for (const VariantLaunch& l : p->launches) {
        const void* k = kernel_of(p->precision, l.variant);
        const GroupedProblem* probs = p->d_probs;
        const TileRef* tiles = p->d_tiles;
        const uint32_t* starts = p->d_starts + l.starts_off;
        uint32_t* counters = p->d_counters + l.counters_off;
        uint32_t nq = l.nq;
        void* args[] = {&probs, &tiles, &starts, &counters, &nq};
        hipError_t e = hipLaunchKernel(k, dim3(l.grid), dim3(256), args,
                                       (size_t)lds_of(p->precision, l.variant), s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// Build (without a graph) the plan for a batch.  Shared by plan_create and
// the tuner.
static int build_plan(const mgemm_problem* probs, int64_t count, int precision,
                      const int* bucket_configs, mgemm_plan** out, int64_t* bad_index,
                      int* bad_status) {
    if (bad_index) *bad_index = -1;
    if (bad_status) *bad_status = 0;
    if (!out) return fail(MGEMM_ERR_BAD_PLAN, "out_plan is NULL");
    *out = nullptr;
    if (count < 0 || (count > 0 && !probs))
        return fail(MGEMM_ERR_BAD_PROBLEM, "problem array is NULL or count < 0");
    if (precision != MGEMM_PREC_FP32 && precision != MGEMM_PREC_BF16X3)
        return fail(MGEMM_ERR_UNSUPPORTED, "grouped plans support FP32 and BF16x3");
    int cfg[NUM_BUCKETS];
    for (int b = 0; b < NUM_BUCKETS; ++b) {
        cfg[b] = bucket_configs ? bucket_configs[b]
                                : (precision == MGEMM_PREC_FP32 ? DEFAULT_F32[b] : DEFAULT_LP[b]);
        if (cfg[b] < 0 || cfg[b] >= NUM_VARIANTS)
            return fail(MGEMM_ERR_UNSUPPORTED, "bucket configuration out of range");
    }
    // Validate every problem (BLAS rules) and collect the live ones.
    std::vector<GroupedProblem> live;
    std::vector<int64_t> live_index;
    std::vector<Extent> cs, ab;
    for (int64_t i = 0; i < count; ++i) {
        const mgemm_problem& q = probs[i];
        std::string why;
        int st = validate(q.transA, q.transB, q.M, q.N, q.K, q.alpha, q.A, q.lda, q.B, q.ldb,
                          q.beta, q.C, q.ldc, why);
        const int ta = trans_code(q.transA), tb = trans_code(q.transB);
        if (st == 0 && (q.lda > MAX_BUF_LD || q.ldb > MAX_BUF_LD || q.ldc > MAX_BUF_LD)) {
            st = MGEMM_ERR_UNSUPPORTED;
            why = "leading dimension above the grouped kernel's limit";
        }
        if (st == 0 && overlaps(ta, tb, q.M, q.N, q.K, q.alpha, q.A, q.lda, q.B, q.ldb, q.C,
                                q.ldc)) {
            st = MGEMM_ERR_ALIAS;
            why = "C overlaps A or B";
        }
        if (st) {
            if (bad_index) *bad_index = i;
            if (bad_status) *bad_status = st;
            return fail(MGEMM_ERR_BAD_PROBLEM, "problem " + std::to_string(i) + ": " + why);
        }
        if (q.M == 0 || q.N == 0) continue;
        const bool no_product = q.alpha == 0.0f || q.K == 0;
        if (no_product && q.beta == 1.0f) continue;
        GroupedProblem g{};
        // alpha == 0: K = 0 so that A and B are never read.
        g.d = GemmDesc{q.A, q.B, q.C, q.M, q.N, no_product ? 0 : q.K, q.lda, q.ldb, q.ldc,
                       q.alpha, q.beta, nullptr, nullptr};
        g.ta = ta;
        g.tb = tb;
        g.variant = cfg[bucket_of(q.M, q.N)];
        const VariantShape vs = variant_shape(precision, g.variant);
        g.tiles_m = (uint32_t)((q.M + vs.bm - 1) / vs.bm);
        g.tiles_n = (uint32_t)((q.N + vs.bn - 1) / vs.bn);
        live.push_back(g);
        live_index.push_back(i);
        cs.push_back(extent_of(q.C, q.M, q.N, q.ldc, i));
        if (!no_product) {
            ab.push_back(extent_of(q.A, ta ? q.K : q.M, ta ? q.M : q.K, q.lda, i));
            ab.push_back(extent_of(q.B, tb ? q.N : q.K, tb ? q.K : q.N, q.ldb, i));
        }
    }
    // No C may overlap another C, or any A or B of the batch.
    int kind = 0;
    const int64_t culprit = batch_alias(cs, ab, &kind);
    if (culprit >= 0) {
        if (bad_index) *bad_index = culprit;
        if (bad_status) *bad_status = MGEMM_ERR_ALIAS;
        return fail(MGEMM_ERR_BAD_PROBLEM,
                    "problem " + std::to_string(culprit) +
                        (kind == 1 ? ": C overlaps another problem's C"
                                   : ": C overlaps an operand of the batch"));
    }
    // Tiles per problem, and the cost of one: its k slabs plus a fixed share
    // for its prologue and epilogue, times the tile's MFMA area (edge tiles
    // run the whole tile's MFMAs).
    std::vector<uint32_t> ntile(live.size());
    std::vector<double> tcost(live.size());
    uint64_t total_tiles = 0;
    for (size_t i = 0; i < live.size(); ++i) {
        const VariantShape vs = variant_shape(precision, live[i].variant);
        const uint64_t n = (uint64_t)live[i].tiles_m * live[i].tiles_n;
        if (n > 0xffffffffULL) return fail(MGEMM_ERR_UNSUPPORTED, "too many tiles");
        ntile[i] = (uint32_t)n;
        total_tiles += n;
        const double slabs = (double)((live[i].d.K + vs.bk - 1) / vs.bk) +
                             tile_overhead_slabs(precision, live[i].variant);
        tcost[i] = slabs * vs.bk * vs.bm * vs.bn;
    }
    if (total_tiles > 0xffffffffULL) return fail(MGEMM_ERR_UNSUPPORTED, "too many tiles");
    int st = check_device(nullptr);
    if (st) return st;
    mgemm_plan* p = new mgemm_plan();
    hipError_t e = hipGetDevice(&p->device);
    p->precision = precision;
    p->nprob = (int64_t)live.size();
    p->ntiles = (int64_t)total_tiles;
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                                   p->device);

    // One launch per variant in use, the costliest first, each with
    // min(8, work-groups) queues.  All launches share one tile table, one
    // offsets table and one counters table.
    double vcost[NUM_VARIANTS] = {0.0, 0.0, 0.0};
    uint64_t vtiles[NUM_VARIANTS] = {0, 0, 0};
    for (size_t i = 0; i < live.size(); ++i) {
        vcost[live[i].variant] += ntile[i] * tcost[i];
        vtiles[live[i].variant] += ntile[i];
    }
    int vorder[NUM_VARIANTS] = {0, 1, 2};
    std::stable_sort(vorder, vorder + NUM_VARIANTS,
                     [&](int a2, int b2) { return vcost[a2] > vcost[b2]; });
    std::vector<TileRef> sched;
    std::vector<uint32_t> starts;
    int64_t ncounters = 0;
    sched.reserve(total_tiles);
    for (int vi = 0; vi < NUM_VARIANTS && e == hipSuccess; ++vi) {
        const int v = vorder[vi];
        if (vtiles[v] == 0) continue;
        const void* k = kernel_of(precision, v);
        const int lds = lds_of(precision, v);
        int per_cu = 0;
        e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, lds);
        if (e != hipSuccess) break;
        const int64_t slots = (int64_t)(per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
        const uint32_t G = (uint32_t)std::max<int64_t>(1, std::min<int64_t>(slots, (int64_t)vtiles[v]));
        const uint32_t nq = std::min<uint32_t>(NUM_XCD, G);
        std::vector<uint32_t> pid, nt;
        std::vector<double> pc;
        for (size_t i = 0; i < live.size(); ++i) {
            if (live[i].variant != v || ntile[i] == 0) continue;
            pid.push_back((uint32_t)i);
            nt.push_back(ntile[i]);
            pc.push_back(tcost[i]);
        }
        const auto queues = queue_partition(nt, pc, nq);
        p->launches.push_back(VariantLaunch{v, G, nq, (int64_t)starts.size(), ncounters});
        for (uint32_t q = 0; q < nq; ++q) {
            starts.push_back((uint32_t)sched.size());
            for (const auto& pt : queues[q]) sched.push_back(TileRef{pid[pt.first], pt.second});
        }
        starts.push_back((uint32_t)sched.size());
        ncounters += (int64_t)(nq + 1) * CTR_STRIDE;
        p->grid = std::max(p->grid, G);
    }
    if (e != hipSuccess) {
        plan_free(p);
        return hip_err(e, "grouped plan set-up");
    }
    if (starts.empty()) starts.push_back(0);
    const std::vector<uint32_t> zeros((size_t)std::max<int64_t>(1, ncounters), 0u);

    if (fault_injected()) e = hipErrorOutOfMemory;
    if (e == hipSuccess && !live.empty())
        e = hipMalloc((void**)&p->d_probs, live.size() * sizeof(GroupedProblem));
    if (e == hipSuccess && !sched.empty())
        e = hipMalloc((void**)&p->d_tiles, sched.size() * sizeof(TileRef));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_starts, starts.size() * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_counters, zeros.size() * sizeof(uint32_t));
    if (e != hipSuccess) {
        plan_free(p);
        (void)hipGetLastError();
        return fail(MGEMM_ERR_ALLOC, "device memory for the plan's tables");
    }
    if (!live.empty())
        e = hipMemcpy(p->d_probs, live.data(), live.size() * sizeof(GroupedProblem),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !sched.empty())
        e = hipMemcpy(p->d_tiles, sched.data(), sched.size() * sizeof(TileRef),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_starts, starts.data(), starts.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice);
    // The counters start at zero (an upload, not a memset: the plan's
    // launches may run on streams that do not wait for the null stream).
    if (e == hipSuccess)
        e = hipMemcpy(p->d_counters, zeros.data(), zeros.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_err(e, "grouped plan upload");
    }
    *out = p;
    return MGEMM_OK;
}

static void plan_register(mgemm_plan* p) {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    g_plans.insert(p);
}

static bool plan_unregister(mgemm_plan* p) {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    return g_plans.erase(p) > 0;
}

}  // namespace mgemm

using namespace mgemm;

extern "C" {

int mgemm_grouped_bucket(int64_t M, int64_t N, int64_t K) {
    (void)K;
    return bucket_of(M, N);
}

int mgemm_grouped_variant_count(int precision) {
    return precision == MGEMM_PREC_FP32 || precision == MGEMM_PREC_BF16X3 ? NUM_VARIANTS : 0;
}

int mgemm_grouped_variant_info(int precision, int variant, int* bm, int* bn, int* bk) {
    if (mgemm_grouped_variant_count(precision) == 0 || variant < 0 || variant >= NUM_VARIANTS)
        return fail(MGEMM_ERR_UNSUPPORTED, "unknown grouped variant");
    const VariantShape s = variant_shape(precision, variant);
    if (bm) *bm = s.bm;
    if (bn) *bn = s.bn;
    if (bk) *bk = s.bk;
    return MGEMM_OK;
}

int mgemm_grouped_plan_create_ex(const mgemm_problem* problems, int64_t count, int precision,
                                 const int* bucket_configs, void* stream, mgemm_plan** out_plan,
                                 int64_t* bad_index, int* bad_status) {
    (void)stream;
    mgemm_plan* p = nullptr;
    int st = build_plan(problems, count, precision, bucket_configs, out_plan ? &p : nullptr,
                        bad_index, bad_status);
    if (st) return st;
    // Record the launch once into a graph, on a private non-blocking stream
    // of default priority (the legacy default stream cannot be captured).
    hipError_t e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = launch_plan_kernel(p, p->capture);
        e = hipStreamEndCapture(p->capture, &p->graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_err(e, "grouped plan graph capture");
    }
    plan_register(p);
    *out_plan = p;
    return MGEMM_OK;
}

}  // extern "C"

namespace mgemm {

// Runs the tuner on the batch with every C saved before and put back after
// (the tuner runs the problems), on `s`; waits for `s`.
static int tune_keeping_c(const mgemm_problem* problems, int64_t count, int precision,
                          hipStream_t s, int* configs) {
    std::vector<std::pair<int64_t, int64_t>> spans;   // (problem, bytes)
    int64_t total = 0;
    for (int64_t i = 0; i < count; ++i) {
        const mgemm_problem& q = problems[i];
        if (q.M <= 0 || q.N <= 0) continue;
        const int64_t bytes = ((q.N - 1) * q.ldc + q.M) * (int64_t)sizeof(float);
        spans.emplace_back(i, bytes);
        total += (bytes + 255) / 256 * 256;
    }
    char* save = nullptr;
    hipError_t e = hipSuccess;
    if (total > 0) e = fault_injected() ? hipErrorOutOfMemory : hipMalloc((void**)&save, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MGEMM_ERR_ALLOC, "device memory to keep C while tuning");
    }
    auto copy_all = [&](bool to_save) {
        int64_t off = 0;
        for (const auto& sp : spans) {
            char* c = reinterpret_cast<char*>(problems[sp.first].C);
            if (e == hipSuccess)
                e = to_save ? hipMemcpyAsync(save + off, c, sp.second, hipMemcpyDeviceToDevice, s)
                            : hipMemcpyAsync(c, save + off, sp.second, hipMemcpyDeviceToDevice, s);
            off += (sp.second + 255) / 256 * 256;
        }
    };
    copy_all(true);
    int st = e == hipSuccess ? mgemm_grouped_tune(problems, count, precision, s, 3, configs, nullptr)
                             : hip_err(e, "saving C");
    copy_all(false);
    const hipError_t e2 = hipStreamSynchronize(s);
    if (save) (void)hipFree(save);
    if (st == MGEMM_OK && (e != hipSuccess || e2 != hipSuccess))
        st = hip_err(e != hipSuccess ? e : e2, "restoring C after tuning");
    return st;
}

}  // namespace mgemm

extern "C" {

int mgemm_grouped_plan_create(const mgemm_problem* problems, int64_t count, int precision,
                              const char* tune_cache, void* stream, mgemm_plan** out_plan,
                              int64_t* bad_index) {
    int bad_status = 0;
    const char* source = tune_cache ? "cache" : "defaults";
    int configs[NUM_BUCKETS];
    const int* use = nullptr;
    uint64_t key = 0;
    if (tune_cache) {
        key = batch_key(problems && count > 0 ? problems : nullptr, problems ? count : 0);
        if (grouped_cache_lookup(tune_cache, precision, key, configs)) use = configs;
    }
    int st = mgemm_grouped_plan_create_ex(problems, count, precision, use, stream, out_plan,
                                          bad_index, &bad_status);
    if (st == MGEMM_OK && tune_cache && !use) {
        // Not in the cache: tune now (keeping every C), store, and rebuild
        // the plan if the tuned assignment differs from the defaults.
        source = "tuned";
        st = tune_keeping_c(problems, count, precision, (hipStream_t)stream, configs);
        if (st == MGEMM_OK && !grouped_cache_store(tune_cache, precision, key, configs))
            st = fail(MGEMM_ERR_UNSUPPORTED, std::string("cannot write ") + tune_cache);
        bool same = true;
        for (int b = 0; b < NUM_BUCKETS; ++b)
            same &= configs[b] == (precision == MGEMM_PREC_FP32 ? DEFAULT_F32[b] : DEFAULT_LP[b]);
        if (st == MGEMM_OK && !same) {
            mgemm_grouped_plan_destroy(*out_plan);
            *out_plan = nullptr;
            st = mgemm_grouped_plan_create_ex(problems, count, precision, configs, stream,
                                              out_plan, bad_index, &bad_status);
        } else if (st != MGEMM_OK) {
            const std::string why = mgemm_last_error();
            mgemm_grouped_plan_destroy(*out_plan);
            *out_plan = nullptr;
            fail(st, why);
        }
        use = configs;
    }
    if (log_enabled())
        log_line("grouped_plan_create precision=%d count=%lld tune_cache=%s source=%s "
                 "configs=%d,%d,%d,%d status=%d%s%s",
                 precision, (long long)count, tune_cache ? tune_cache : "(none)", source,
                 use ? use[0] : -1, use ? use[1] : -1, use ? use[2] : -1, use ? use[3] : -1, st,
                 st ? " " : "", st ? mgemm_last_error() : "");
    return st;
}

int mgemm_grouped_plan_launch(mgemm_plan* plan, void* stream) {
    if (!plan_live(plan)) return fail(MGEMM_ERR_BAD_PLAN, "plan is NULL or destroyed");
    if (plan->ntiles == 0) return MGEMM_OK;
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    return e == hipSuccess ? MGEMM_OK : hip_err(e, "hipGraphLaunch");
}

int mgemm_grouped_plan_run(mgemm_plan* plan, void* stream) {
    if (!plan_live(plan)) return fail(MGEMM_ERR_BAD_PLAN, "plan is NULL or destroyed");
    hipError_t e = launch_plan_kernel(plan, (hipStream_t)stream);
    return e == hipSuccess ? MGEMM_OK : hip_err(e, "grouped kernel launch");
}

int mgemm_grouped_plan_info(const mgemm_plan* plan, int64_t* tiles, int64_t* workgroups) {
    if (!plan_live(plan)) return fail(MGEMM_ERR_BAD_PLAN, "plan is NULL or destroyed");
    if (tiles) *tiles = plan->ntiles;
    if (workgroups) *workgroups = plan->grid;
    return MGEMM_OK;
}

int mgemm_grouped_plan_destroy(mgemm_plan* plan) {
    if (!plan || !plan_unregister(plan))
        return fail(MGEMM_ERR_BAD_PLAN, "plan is NULL or already destroyed");
    plan_free(plan);
    return MGEMM_OK;
}

int mgemm_grouped_tune(const mgemm_problem* problems, int64_t count, int precision, void* stream,
                       int reps, int* bucket_configs, float* best_ms) {
    if (!bucket_configs) return fail(MGEMM_ERR_UNSUPPORTED, "bucket_configs is NULL");
    if (reps < 1) reps = 1;
    hipStream_t s = (hipStream_t)stream;
    for (int b = 0; b < NUM_BUCKETS; ++b)
        bucket_configs[b] = precision == MGEMM_PREC_FP32 ? DEFAULT_F32[b] : DEFAULT_LP[b];
    bool used[NUM_BUCKETS] = {false, false, false, false};
    for (int64_t i = 0; i < count && problems; ++i)
        used[bucket_of(problems[i].M, problems[i].N)] = true;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_err(hipGetLastError(), "hipEventCreate");
    }
    // Time the whole batch with the given bucket assignment: the best of
    // `reps` rounds, each the mean of LAUNCHES back-to-back launches, after
    // two warm-up launches (one launch of a few hundred microseconds is too
    // short to time against the clock's drift).
    constexpr int LAUNCHES = 8;
    auto time_of = [&](const int* cfg, float& ms) -> int {
        mgemm_plan* p = nullptr;
        int st = build_plan(problems, count, precision, cfg, &p, nullptr, nullptr);
        if (st) return st;
        hipError_t e = launch_plan_kernel(p, s);   // warm-up
        if (e == hipSuccess) e = launch_plan_kernel(p, s);
        float best = 1e30f;
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            e = hipEventRecord(e0, s);
            for (int l = 0; l < LAUNCHES && e == hipSuccess; ++l) e = launch_plan_kernel(p, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e == hipSuccess && t / LAUNCHES < best) best = t / LAUNCHES;
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        plan_free(p);
        if (e != hipSuccess) return hip_err(e, "grouped tuning run");
        ms = best;
        return MGEMM_OK;
    };
    // Start from the fastest of the defaults and the single-variant
    // assignments (one launch for the whole batch: no launch waits behind
    // another's last work-groups), then descend one bucket at a time, in two
    // passes so that an early bucket is revisited once the later ones moved.
    // A change is taken only when it is faster by more than TUNE_MARGIN:
    // of two assignments within timing noise of each other, the earlier one
    // stays.
    constexpr float TUNE_MARGIN = 0.98f;
    int defaults[NUM_BUCKETS];
    for (int b = 0; b < NUM_BUCKETS; ++b) defaults[b] = bucket_configs[b];
    float cur = 0.0f;
    int st = time_of(bucket_configs, cur);   // brings the clock up; timed again below
    if (st == MGEMM_OK) st = time_of(bucket_configs, cur);
    for (int v = 0; v < NUM_VARIANTS && st == MGEMM_OK; ++v) {
        int uni[NUM_BUCKETS];
        for (int b = 0; b < NUM_BUCKETS; ++b) uni[b] = v;
        float t = 0.0f;
        st = time_of(uni, t);
        if (st == MGEMM_OK && t < cur * TUNE_MARGIN) {
            cur = t;
            for (int b = 0; b < NUM_BUCKETS; ++b) bucket_configs[b] = v;
        }
    }
    for (int pass = 0; pass < 2 && st == MGEMM_OK; ++pass) {
        for (int b = 0; b < NUM_BUCKETS && st == MGEMM_OK; ++b) {
            if (!used[b]) continue;
            const int keep = bucket_configs[b];
            int best_v = keep;
            for (int v = 0; v < NUM_VARIANTS && st == MGEMM_OK; ++v) {
                if (v == keep) continue;
                bucket_configs[b] = v;
                float t = 0.0f;
                st = time_of(bucket_configs, t);
                if (st == MGEMM_OK && t < cur * TUNE_MARGIN) {
                    cur = t;
                    best_v = v;
                }
            }
            bucket_configs[b] = best_v;
        }
    }
    // The descent compares assignments timed at different moments.  The
    // winner replaces the defaults only if it also wins a head-to-head
    // against them, timed alternately, by the same margin.
    bool moved = false;
    for (int b = 0; b < NUM_BUCKETS; ++b) moved |= bucket_configs[b] != defaults[b];
    if (moved && st == MGEMM_OK) {
        float td = 1e30f, tc = 1e30f;
        for (int r = 0; r < 3 && st == MGEMM_OK; ++r) {
            float t = 0.0f;
            st = time_of(defaults, t);
            if (st == MGEMM_OK) td = std::min(td, t);
            if (st == MGEMM_OK) st = time_of(bucket_configs, t);
            if (st == MGEMM_OK) tc = std::min(tc, t);
        }
        if (st == MGEMM_OK) {
            if (tc < td * TUNE_MARGIN) {
                cur = tc;
            } else {
                for (int b = 0; b < NUM_BUCKETS; ++b) bucket_configs[b] = defaults[b];
                cur = td;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == MGEMM_OK && best_ms) *best_ms = cur;
    return st;
}

}  // extern "C"
