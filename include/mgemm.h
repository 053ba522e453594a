/*
 * mgemm.h -- C ABI of libmgemm, a single-precision general matrix-matrix
 * multiply for AMD Instinct MI355X (gfx950).
 *
 * The operation is the Level-3 BLAS SGEMM routine (Aberdeen & Baxter,
 * Section 1: the paper's library offers the BLAS SGEMM calling interface;
 * A is M x K, B is K x N and the product costs 2MNK flops):
 *
 *     C <- alpha * op(A) * op(B) + beta * C
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Storage.  Column-major, as in BLAS: element (r, c) of a stored array X
 *   with leading dimension ldX is X[r + c*ldX].  op(X) is X for trans 'N'
 *   or 'n', and X^T for 'T', 't', 'C' or 'c' (real data: the conjugate
 *   transpose is the transpose).  A is stored M x K ('N') or K x M ('T');
 *   B is stored K x N ('N') or N x K ('T'); C is stored M x N.  Only the
 *   leading stored-rows x columns part of each array is referenced.
 * Pointers.  A, B and C are DEVICE pointers owned by the caller (for
 *   example torch tensors).  The library never frees or keeps them.  C must
 *   not overlap the referenced part of A or B.
 * Scalars.  alpha == 0 or K == 0: A and B are not read and C <- beta*C.
 *   beta == 0: C is not read, so NaN or Inf in C do not propagate.
 *   M == 0, N == 0, or ((alpha == 0 or K == 0) and beta == 1): nothing is
 *   launched and the call returns MGEMM_OK.
 * Sizes.  64-bit.  Leading dimensions: lda >= max(1, stored rows of A),
 *   ldb >= max(1, stored rows of B), ldc >= max(1, M).
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Calls
 *   enqueue work and return; a fault inside a kernel is reported by the
 *   caller's next synchronisation, as usual for HIP.  Calls on different
 *   streams may be made from different threads.
 * Errors.  Return value 0 (MGEMM_OK) on success.  A negative value -i
 *   names the illegal argument by its position in the BLAS SGEMM argument
 *   list: 1 transA, 2 transB, 3 M, 4 N, 5 K, 7 A, 8 lda, 9 B, 10 ldb,
 *   12 C, 13 ldc (a NULL A, B or C is illegal only when it would be
 *   read or written).  Arguments are checked in that order, before any
 *   HIP call, so a bad call launches nothing.  Positive values are the
 *   MGEMM_ERR_* codes below.  mgemm_last_error() gives a text for the last
 *   failing call on the calling thread.
 */
#ifndef MGEMM_H
#define MGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGEMM_OK              0
#define MGEMM_ERR_HIP         100 /* a HIP runtime call failed */
#define MGEMM_ERR_NO_DEVICE   101 /* no HIP device is visible */
#define MGEMM_ERR_ARCH        102 /* the current device is not gfx950 */
#define MGEMM_ERR_ALLOC       103 /* device memory for a workspace or plan */
#define MGEMM_ERR_ALIAS       105 /* C overlaps the referenced part of A or B */
#define MGEMM_ERR_UNSUPPORTED 106 /* unknown precision or tile configuration */
#define MGEMM_ERR_BAD_PLAN    107 /* NULL or already destroyed plan */
#define MGEMM_ERR_BAD_PROBLEM 108 /* a grouped problem failed validation */

/* Arithmetic used for the product (the result is always FP32). */
#define MGEMM_PREC_FP32        0 /* FP32 operands, FP32 MFMA, FP32 accumulate */
#define MGEMM_PREC_BF16X3      1 /* x = hi + lo in BF16 (round to nearest even);
                                    hi*hi + hi*lo + lo*hi on BF16 MFMA,
                                    FP32 accumulate; lo*lo is dropped */
#define MGEMM_PREC_FP16_SCALED 2 /* power-of-two scale per 32-row panel of
                                    op(A) and per 32-column panel of op(B),
                                    FP16 MFMA, FP32 accumulate, exact unscale */

/*
 * The SGEMM operation above (paper, Section 1), computed in FP32 on FP32
 * MFMA with a tile configuration the library chooses.  The 14 arguments
 * follow the BLAS SGEMM order, plus the stream.
 */
int mgemm_sgemm(char transA, char transB, int64_t M, int64_t N, int64_t K,
                float alpha, const float *A, int64_t lda,
                const float *B, int64_t ldb,
                float beta, float *C, int64_t ldc, void *stream);

/*
 * The same operation in one of the MGEMM_PREC_* arithmetics, with an
 * explicit tile configuration `config` (0 .. mgemm_config_count(precision)-1)
 * or -1 for the library's choice.
 *
 * Workspace.  The two 16-bit forms take one stream-ordered workspace per
 * call (hipMallocFromPoolAsync on `stream`, freed with hipFreeAsync on it
 * after the call's kernels) from a memory pool the library keeps per
 * device.  The pool keeps freed memory across synchronisations (release
 * threshold: unlimited), so later calls reuse it; mgemm_trim_workspace()
 * hands it back.  The workspace holds:
 *   - MGEMM_PREC_FP16_SCALED: the panel exponents, (M+N)/32 ints, and the
 *     per-panel partial maxima of the exponent pass;
 *   - configurations 4 and up of either form (the library's choice for
 *     large products): the operands packed once, 2 bytes per element of A
 *     and of B for FP16, 4 bytes (hi and lo) for BF16x3 -- 512 MB at
 *     M = N = K = 8192.
 * FP32 configuration 11 (split-K: the k range cut into S pieces whose
 * partial products are added in a fixed order by a second kernel), which
 * the library's choice takes for products with at most one 128 x 128 tile
 * per CU and K of about 2048 and up, takes S*M*N*4 bytes from the same
 * pool (at most 1 GiB; larger products, and leading dimensions beyond the
 * 32-bit buffer path, run configuration 0 instead).  The other FP32
 * configurations take no workspace; mgemm_config_info describes each
 * (configuration 12, 64 x 64 tiles with 32-deep slabs, is the library's
 * choice for products of one to a few such tiles per CU).  The last
 * configuration of either
 * 16-bit form (13) is split-K in the same way: the pieces are in-staging
 * tiles (128 x 128, or 64 x 64 for few tiles), their S*M*N*4 bytes of
 * partial products come from the pool too (the FP16 unscale is applied per
 * piece, exactly), and where splitting does not apply configuration 1 runs.
 * The FP16 form's 128 x 128 pieces run on packed copies of op(A) and op(B)
 * (2(M + N)K more bytes of workspace) where those fit, with the same
 * results bitwise.  The library's choice takes it for BF16x3 products with
 * at most 128 tiles of 128 x 128 and K >= 2048, or at most 256 and
 * K >= 8192, and for FP16 products with at most 64 such tiles and
 * K >= 2048, or at most 160 and K >= 3072.
 * An allocation failure returns MGEMM_ERR_ALLOC before anything runs.  A
 * packed configuration that the product cannot use (K too long for 32-bit
 * block offsets, or an LDS ring larger than a CU) runs configuration 0.
 * FP32 with config = -1, no choice recorded for the shape and no
 * activation: a product whose M and N are each a multiple of 256 or at most
 * 64 past one (at least one past), with a whole-tile block Mm x Nm of at
 * least 2^37 flops, runs as three products on the same stream, each with
 * its own default configuration: the block, rows Mm..M-1 of C (all
 * columns), and columns Nm..N-1 of its first Mm rows (4097^3: 136 against
 * 124 TFLOP/s whole).  FP32 with config = -1 and no choice recorded: a
 * product with at most 8 columns (or rows) of C, at least 256 rows (or
 * columns), K >= 256 and leading dimensions (and M) below 2^21 - 64
 * (with a k-contiguous large operand, i.e. op(A) stored transposed or op(B)
 * not, and more than 4 such columns or rows: at least 2^25 elements of it)
 * streams the large operand once in k pieces whose
 * partial sums (S*M*N*4 bytes of workspace from the pool) are added in a
 * fixed order, as for split-K.  mgemm_default_config reports the
 * configuration the product would otherwise take.
 */
int mgemm_sgemm_ex(char transA, char transB, int64_t M, int64_t N, int64_t K,
                   float alpha, const float *A, int64_t lda,
                   const float *B, int64_t ldb,
                   float beta, float *C, int64_t ldc, void *stream,
                   int precision, int config);

/*
 * Activations that mgemm_sgemm_act applies to v = alpha op(A) op(B) + beta C
 * before C is written (the paper's application, Section 4, trains a neural
 * network whose layers are these products):
 *   MGEMM_ACT_TANH       C <- tanh(v)                (a tanh layer's output)
 *   MGEMM_ACT_TANH_GRAD  C <- v * (1 - aux^2)        (the gradient through a
 *                        tanh layer whose output is aux)
 */
#define MGEMM_ACT_NONE      0
#define MGEMM_ACT_TANH      1
#define MGEMM_ACT_TANH_GRAD 2

/*
 * mgemm_sgemm_ex with an activation fused into the epilogue, so that the
 * product is stored once, already activated.  `aux` (device, caller-owned)
 * is read only by MGEMM_ACT_TANH_GRAD: an M x N column-major array with C's
 * leading dimension ldc, which must not overlap C (MGEMM_ERR_ALIAS); it may
 * be NULL otherwise.  An unknown activation, or a NULL aux that would be
 * read, returns MGEMM_ERR_UNSUPPORTED before anything runs.  Everything
 * else is as for mgemm_sgemm_ex, except that with an activation the quick
 * return for (alpha == 0 or K == 0) and beta == 1 does not apply: C <-
 * act(C) is still computed.  Split-K configurations apply the activation
 * once, in their reduction.  tanh is the device library's tanhf.
 */
int mgemm_sgemm_act(char transA, char transB, int64_t M, int64_t N, int64_t K,
                    float alpha, const float *A, int64_t lda,
                    const float *B, int64_t ldb,
                    float beta, float *C, int64_t ldc, void *stream,
                    int precision, int config, int activation,
                    const float *aux);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as mgemm_sgemm_ex, arguments and results alike, whose workspace is
 * a device array of MGEMM_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on, from load until the process ends.  The call makes
 * no hipMalloc, hipFree or pool allocation; its device address is looked
 * up once per device, on the first call there.
 *
 * The array is shared by every call on one GPU and keeps what the last call
 * left in it (nothing needs it cleared: every call writes what it reads).
 * Calls that overlap in time on one GPU -- on different streams, or from
 * different threads -- race on it and give wrong results; serialise them
 * (one stream, or events).
 *
 * Workspace beyond the array: a named `config` whose workspace exceeds it
 * (the split-K configurations with S*M*N*4 bytes of partial products, a
 * packed 16-bit configuration with its packed operands) returns
 * MGEMM_ERR_UNSUPPORTED and launches nothing; with config = -1 the library
 * takes its usual choice when it fits, else a configuration that needs
 * less (unsplit tiles; 16-bit operands split or scaled while staging).
 * Scaled-FP16 split-K whose packed operands do not fit beside its partial
 * products runs its pieces scaling while staging, with the same results
 * bitwise.  Scaled FP16 always needs its panel exponents and partial maxima
 * (about (M+N)/32 * (4 + 4*ceil(K/2048)) bytes); a product whose exponents
 * exceed the array returns MGEMM_ERR_UNSUPPORTED.
 */
#define MGEMM_NOALLOC_SCRATCH_BYTES (64LL << 20)
int mgemm_sgemm_ex_noalloc(char transA, char transB, int64_t M, int64_t N,
                           int64_t K, float alpha, const float *A,
                           int64_t lda, const float *B, int64_t ldb,
                           float beta, float *C, int64_t ldc, void *stream,
                           int precision, int config);

/*
 * Return the memory the workspace pools keep (freed workspaces of earlier
 * 16-bit calls) to the device.  Calls still in flight keep theirs.
 */
int mgemm_trim_workspace(void);

/* Number of tile configurations for a precision (0 for an unknown one). */
int mgemm_config_count(int precision);

/*
 * Description of one configuration: BM, BN, BK (the work-group tile of C
 * and the K depth of one staged slab) and the number of threads per
 * work-group.  Returns MGEMM_ERR_UNSUPPORTED for an unknown pair.
 */
int mgemm_config_info(int precision, int config, int *bm, int *bn, int *bk,
                      int *threads);

/* The configuration mgemm_sgemm_ex(..., config = -1) would use: a choice
 * recorded for exactly this (precision, trans pair, M, N, K), else the
 * built-in size heuristic.  -1 for a bad trans flag. */
int mgemm_default_config(int precision, char transA, char transB,
                         int64_t M, int64_t N, int64_t K);

/*
 * Autotuner for single calls: runs the product once per configuration as a
 * warm-up and then `reps` timed rounds (HIP events on `stream`; a round is
 * one call, or as many back-to-back calls as fill about a millisecond, at
 * most 64), keeps the fastest (best round) and records it as the choice for
 * this exact (precision, trans pair, M, N, K), so later calls with
 * config = -1 use it.  A choice other than the built-in rule's is kept only
 * if it also beats that rule's choice by more than 2% in a head-to-head,
 * the two timed alternately three times.  For an FP32 product that the
 * library's choice splits at its ragged edges or runs on the thin path (see
 * mgemm_sgemm_ex), that choice is the one to beat; when it stays, nothing is
 * recorded (any earlier choice for the shape is dropped) and *best_config
 * is -1.
 * Arguments as for mgemm_sgemm_ex; C is overwritten (with beta != 0 it is
 * updated once per run), so tune on scratch output.  Synchronises `stream`.
 * *best_config and *best_ms (either may be NULL) receive the result.
 */
int mgemm_tune_sgemm(char transA, char transB, int64_t M, int64_t N, int64_t K,
                     float alpha, const float *A, int64_t lda,
                     const float *B, int64_t ldb,
                     float beta, float *C, int64_t ldc, void *stream,
                     int precision, int reps, int *best_config, float *best_ms);

/* Record a choice without timing (e.g. replayed from a saved tuning run);
 * returns MGEMM_ERR_UNSUPPORTED for an unknown precision or configuration. */
int mgemm_record_choice(int precision, char transA, char transB,
                        int64_t M, int64_t N, int64_t K, int config);

/* Forget every recorded choice. */
int mgemm_clear_choices(void);

/*
 * Persist the recorded single-call choices: mgemm_save_choices appends one
 * line per choice, `mgemm-tune v1 single <arch> <cus> <version>
 * <precision> <trans pair> <M> <N> <K> <config>`, stamped with the current
 * device's architecture and CU count ("nodevice" and 0 when none is
 * visible) and the library version; mgemm_load_choices records every line
 * of the file that matches the current device and version (the last of
 * several for one product wins) and writes how many to *loaded (may be
 * NULL).  A file that cannot be written or read returns
 * MGEMM_ERR_UNSUPPORTED.  The same file may hold grouped entries
 * (mgemm_grouped_plan_create).
 */
int mgemm_save_choices(const char *path);
int mgemm_load_choices(const char *path, int64_t *loaded);

/* ---- many independent products in one persistent launch ---------------- */

/*
 * One problem of a batch: C_i <- alpha_i op(A_i) op(B_i) + beta_i C_i with
 * the conventions above (device pointers, column-major).
 */
typedef struct mgemm_problem {
    char transA, transB;
    int64_t M, N, K;
    float alpha, beta;
    const float *A; int64_t lda;
    const float *B; int64_t ldb;
    float *C; int64_t ldc;
} mgemm_problem;

typedef struct mgemm_plan mgemm_plan;

/*
 * Build a plan for `count` problems (host array, copied).  Precision is
 * MGEMM_PREC_FP32 or MGEMM_PREC_BF16X3.  Every problem is validated with
 * the rules above; on failure the call returns MGEMM_ERR_BAD_PROBLEM with
 * *bad_index (may be NULL) set to the problem; mgemm_last_error() names
 * the rule.  No C may overlap another problem's C, A or B.  Leading
 * dimensions must not exceed 2^21 - 64.
 *
 * Problems are sorted into four size buckets (mgemm_grouped_bucket); each
 * bucket uses one tile variant.  `tune_cache` chooses them:
 *   - NULL: the library defaults (one variant for every bucket: FP32
 *     64x64x32, BF16x3 128x128);
 *   - a file path: the variants recorded in that file for this device
 *     (architecture and CU count), library version, precision and batch
 *     (the problems' trans flags and sizes, in order).  When the file has
 *     no such entry (or does not exist), the batch is tuned on `stream` as
 *     by mgemm_grouped_tune (best of 3 timed runs per assignment), with
 *     every C saved before and restored after (device memory of the C
 *     extents, freed before return), and the result is appended to the
 *     file.  That first call synchronises `stream`; later calls only read
 *     the file.  File format: lines of `mgemm-tune v1 grouped <arch>
 *     <cus> <version> <precision> <batch hash> <c0>,<c1>,<c2>,<c3>`; the
 *     last matching line wins; other lines are ignored.  A file that
 *     cannot be written returns MGEMM_ERR_UNSUPPORTED.
 * The paper sets its block sizes by experiment on the target machine
 * (Section 3); the cache keeps such experiments across processes.
 *
 * The plan uploads to device memory it owns a descriptor table and, per
 * tile variant in use, up to eight work queues of tiles (one per XCD:
 * whole problems to the least-loaded queue, each queue costliest tile
 * first) with one counter each.  The variant's persistent work-groups take
 * tiles from their XCD's queue with an atomic counter and then help the
 * other queues; the last work-group to finish zeroes the counters.  It
 * records the launches (one per variant in use, costliest first) into a
 * HIP graph on a private stream.  Results are bitwise reproducible: a
 * tile's result does not depend on which work-group computes it, and
 * every tile of C is written by one work-group.  Launches of one plan must
 * not overlap in time (they share the counters, as well as C): launch it
 * on one stream, or order the streams.
 */
int mgemm_grouped_plan_create(const mgemm_problem *problems, int64_t count,
                              int precision, const char *tune_cache,
                              void *stream, mgemm_plan **out_plan,
                              int64_t *bad_index);

/*
 * The same with the variants given explicitly: `bucket_configs` holds 4
 * entries (0 .. mgemm_grouped_variant_count()-1, e.g. from
 * mgemm_grouped_tune; NULL = the library defaults), and on a bad problem
 * *bad_status (may be NULL) also receives its BLAS-style code (or
 * MGEMM_ERR_ALIAS / MGEMM_ERR_UNSUPPORTED).  `stream` is unused and may be
 * NULL.
 */
int mgemm_grouped_plan_create_ex(const mgemm_problem *problems, int64_t count,
                                 int precision, const int *bucket_configs,
                                 void *stream, mgemm_plan **out_plan,
                                 int64_t *bad_index, int *bad_status);

/* Replay the plan's graph on `stream` (hipGraphLaunch). */
int mgemm_grouped_plan_launch(mgemm_plan *plan, void *stream);

/* Launch the plan's persistent kernels directly on `stream` (no graph). */
int mgemm_grouped_plan_run(mgemm_plan *plan, void *stream);

/* Number of tiles of the plan, and work-groups of its largest launch. */
int mgemm_grouped_plan_info(const mgemm_plan *plan, int64_t *tiles,
                            int64_t *workgroups);

/* Free the plan and its device memory (the caller synchronises first:
 * nothing waits for launches in flight).  A NULL or already destroyed plan
 * returns MGEMM_ERR_BAD_PLAN. */
int mgemm_grouped_plan_destroy(mgemm_plan *plan);

/* Size bucket (0..3) of a grouped problem: max(M, N) <= 64, <= 128,
 * <= 256, > 256. */
int mgemm_grouped_bucket(int64_t M, int64_t N, int64_t K);

/* Number of tile variants of the grouped kernel for a precision (0 when
 * grouped plans do not support it), and the tile shape of one variant. */
int mgemm_grouped_variant_count(int precision);
int mgemm_grouped_variant_info(int precision, int variant, int *bm, int *bn,
                               int *bk);

/*
 * Autotuner: choose the variant of every size bucket present in the batch
 * by timing the whole grouped launch on `stream` (HIP events; the best of
 * `reps` rounds, each the mean of 8 back-to-back launches, after two
 * warm-up launches): the defaults and each assignment of one variant to
 * every bucket are timed, then, from the fastest, each bucket in turn
 * tries every variant (two passes).  A change is kept only when it is more
 * than 2% faster than the assignment it replaces, so near ties keep the
 * earlier choice; a result other than the defaults must also beat them by
 * 2% in a final head-to-head, the two timed alternately three times.
 * Writes 4 entries to
 * bucket_configs and the best time in
 * milliseconds to *best_ms (may be NULL).  The problems are RUN: every C
 * is overwritten with unspecified values, so tune on scratch outputs or
 * re-initialise C afterwards.  Synchronises `stream`.
 */
int mgemm_grouped_tune(const mgemm_problem *problems, int64_t count,
                       int precision, void *stream, int reps,
                       int *bucket_configs, float *best_ms);

/* ---- pre-packed B -------------------------------------------------------- */

/*
 * op(B) converted once and kept in the library's packed layout, for calls
 * that reuse one B with many A (layer weights, a fixed operand).  The
 * paper re-orders blocks of B into a buffer laid out for the kernel's
 * accesses (Section 3, re-buffering); here that step runs once for the
 * whole operand and its result is kept, so a call with a packed B packs
 * only op(A).
 *
 * Built for MGEMM_PREC_BF16X3 (the hi and lo bf16 halves of every
 * element, 4 bytes per element of op(B), K rounded up to 16 and N to 32)
 * and MGEMM_PREC_FP16_SCALED (2 bytes per element, scaled by the panel
 * exponents of op(B), which the handle keeps).  Their products run on the
 * pipelined packed 256 x 256 tile when there are at least 144 such tiles,
 * else on the pipelined 128 x 128 tile (16-bit configurations 10 and 11):
 * their results equal mgemm_sgemm_ex with the same precision and
 * configuration bitwise.  MGEMM_PREC_FP32 keeps op(B) transposed once into
 * the layout the FP32 kernels load with 16-byte loads (a column-major K x N
 * array, k contiguous, leading dimension K rounded up to 4; 4 bytes per
 * element); its products are the ordinary FP32 call with that array as a
 * 'N' operand (library's choice of configuration for op(A) and 'N'), and
 * equal that call bitwise.
 *
 * Argument errors are reported with the SGEMM number of the same argument
 * (transB -2, N -4, K -5, B -9, ldb -10; transA -1, M -3, A -7, lda -8,
 * C -12, ldc -13); a NULL or destroyed handle gives MGEMM_ERR_BAD_PLAN.
 */
typedef struct mgemm_packed_b mgemm_packed_b;

/*
 * Pack op(B) (K x N; B stored K x N for 'N', N x K for 'T'/'C', column-
 * major at ldb) on `stream`.  The handle owns hipMalloc'ed device memory on
 * the current device.  Packing is asynchronous on `stream`: calls on that
 * stream may use the handle at once; B may change once that work is done.
 * *out is NULL on any error; out == NULL returns MGEMM_ERR_UNSUPPORTED.
 */
int mgemm_pack_b(char transB, int64_t K, int64_t N, const float *B, int64_t ldb,
                 int precision, void *stream, mgemm_packed_b **out);

/* K, N, precision and device bytes of a packed B (any pointer may be NULL). */
int mgemm_packed_b_info(const mgemm_packed_b *Bp, int64_t *K, int64_t *N,
                        int *precision, int64_t *bytes);

/*
 * C <- alpha op(A) op(B) + beta C with op(B) from Bp (K and N are Bp's).
 * op(A) is M x K.  Same rules as mgemm_sgemm_ex for A, C, alpha, beta and
 * the quick returns; op(A) is packed into a stream-ordered workspace from
 * the library's pool (4 bytes per element for BF16x3, 2 for FP16, which
 * also computes op(A)'s panel exponents there).  Bp must stay alive until
 * the call's work has run.
 */
int mgemm_sgemm_packed_b(char transA, int64_t M, float alpha, const float *A,
                         int64_t lda, const mgemm_packed_b *Bp, float beta,
                         float *C, int64_t ldc, void *stream);

/* Free a packed B; waits for device work still reading it. */
int mgemm_packed_b_destroy(mgemm_packed_b *Bp);

/* ---- status ------------------------------------------------------------ */

/* Static text for a status code. */
const char *mgemm_status_string(int status);

/* Text for the last failing call on this thread ("" if none). */
const char *mgemm_last_error(void);

/* Library version as 10000*major + 100*minor + patch. */
int mgemm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MGEMM_H */
