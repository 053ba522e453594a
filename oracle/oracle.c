/*
 * oracle.c -- plain FP64 reference for the single-precision general
 * matrix-matrix product
 *
 *     C <- alpha * op(A) * op(B) + beta * C
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the ground truth that the GPU
 * library is checked against.  It shares no code, header, table or helper
 * with the GPU library and is never called by it.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * What it follows:
 *   - Section 1 (Introduction) of Aberdeen & Baxter: the operation is the
 *     SGEMM routine of Level-3 BLAS, A is M x K, B is K x N, and a dense
 *     product costs 2MNK floating point operations (no Strassen).
 *   - Section 4 (Results) compares against a plain multiply of three nested
 *     loops.  This is that loop, with the accumulation done in
 *     FP64 instead of FP32 so that it is far more accurate than anything it
 *     checks.
 *
 * BLAS conventions (the paper only says "the SGEMM interface"; these are
 * the reference-BLAS reading):
 *   - column-major storage: element (r, c) of a stored array X with leading
 *     dimension ld is X[r + c*ld];
 *   - op(X) = X for 'N'/'n', X^T for 'T'/'t'/'C'/'c' (real data, so the
 *     conjugate transpose is the transpose);
 *   - alpha == 0 or K == 0: the product term is absent and A, B are not read;
 *   - beta == 0: C0 is not read (NaN/Inf in C0 do not reach the result).
 *
 * Arithmetic: every op(A)[i,k] * op(B)[k,j] product of two FP32 values is
 * exact in FP64 (24 + 24 significant bits <= 53), so the only roundings are
 * the K-1 additions, done in increasing k with one sequential accumulator
 * per output element, then one multiply by alpha and one add of beta*C0
 * (itself an exact product).  Build with -ffp-contract=off so that no fused
 * multiply-add changes those two final roundings.  Work is split over
 * output elements only, so the result is bitwise the same for any thread
 * count.
 *
 * Return value of every entry point: 0 on success, -1 for an argument that
 * is not a legal BLAS argument (bad trans flag, negative size, leading
 * dimension too small, sampled index out of range), -2 when host memory
 * for the FP64 copies of the operands cannot be allocated.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

static int trans_code(char t)
{
    if (t == 'N' || t == 'n') return 0;
    if (t == 'T' || t == 't' || t == 'C' || t == 'c') return 1;
    return -1;
}

static int64_t max1(int64_t v) { return v > 1 ? v : 1; }

static int check_args(int ta, int tb, int64_t M, int64_t N, int64_t K,
                      int64_t lda, int64_t ldb, int64_t ldc)
{
    if (ta < 0 || tb < 0) return -1;
    if (M < 0 || N < 0 || K < 0) return -1;
    if (lda < max1(ta ? K : M)) return -1;   /* stored rows of A */
    if (ldb < max1(tb ? N : K)) return -1;   /* stored rows of B */
    if (ldc < max1(M)) return -1;
    return 0;
}

/* Element (r, c) of op(X), X column-major with leading dimension ld. */
static double op_elem(const void *X, int is_double, int64_t ld, int trans,
                      int64_t r, int64_t c)
{
    int64_t off = trans ? (c + r * ld) : (r + c * ld);
    return is_double ? ((const double *)X)[off] : (double)((const float *)X)[off];
}

/*
 * Copy op(X) (rows x cols) into a dense FP64 array, each ROW contiguous when
 * row_major != 0 and each COLUMN contiguous otherwise.  This only changes
 * where the values sit in memory, not the order in which they are summed.
 */
static double *materialise(const void *X, int is_double, int64_t ld, int trans,
                           int64_t rows, int64_t cols, int row_major)
{
    size_t n = (size_t)rows * (size_t)cols;
    double *out = (double *)malloc((n ? n : 1) * sizeof(double));
    if (!out) return NULL;
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t c = 0; c < cols; ++c) {
            double v = op_elem(X, is_double, ld, trans, r, c);
            if (row_major) out[(size_t)r * cols + c] = v;
            else           out[(size_t)c * rows + r] = v;
        }
    return out;
}

/* alpha * sum_k a[k]*b[k] (k increasing) + beta * c0, with the BLAS rule
 * that an absent product term or a zero beta is not evaluated. */
static double finish(double dot, int use_product, double alpha,
                     double beta, double c0)
{
    double v = use_product ? alpha * dot : 0.0;
    if (beta != 0.0) v += beta * c0;
    return v;
}

static int gemm_full(char transA, char transB, int64_t M, int64_t N, int64_t K,
                     double alpha, const void *A, int64_t lda,
                     const void *B, int64_t ldb, double beta,
                     const void *C0, int64_t ldc, int is_double,
                     double *out, int64_t ldo)
{
    int ta = trans_code(transA), tb = trans_code(transB);
    if (check_args(ta, tb, M, N, K, lda, ldb, ldc) || ldo < max1(M)) return -1;
    int use_product = (alpha != 0.0 && K > 0);
    double *Ar = NULL, *Bc = NULL;
    if (use_product) {
        Ar = materialise(A, is_double, lda, ta, M, K, 1);   /* rows of op(A) */
        Bc = materialise(B, is_double, ldb, tb, K, N, 0);   /* cols of op(B) */
        if (!Ar || !Bc) { free(Ar); free(Bc); return -2; }
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t i = 0; i < M; ++i) {
            double dot = 0.0;
            if (use_product) {
                const double *a = Ar + (size_t)i * K;
                const double *b = Bc + (size_t)j * K;
                for (int64_t k = 0; k < K; ++k)
                    dot += a[k] * b[k];
            }
            double c0 = 0.0;
            if (beta != 0.0)
                c0 = is_double ? ((const double *)C0)[i + j * ldc]
                               : (double)((const float *)C0)[i + j * ldc];
            out[i + j * ldo] = finish(dot, use_product, alpha, beta, c0);
        }
    }
    free(Ar);
    free(Bc);
    return 0;
}

static int gemm_entries(char transA, char transB, int64_t M, int64_t N, int64_t K,
                        double alpha, const void *A, int64_t lda,
                        const void *B, int64_t ldb, double beta,
                        const void *C0, int64_t ldc, int is_double,
                        int64_t count, const int64_t *rows, const int64_t *cols,
                        double *out)
{
    int ta = trans_code(transA), tb = trans_code(transB);
    if (check_args(ta, tb, M, N, K, lda, ldb, ldc) || count < 0) return -1;
    for (int64_t e = 0; e < count; ++e)
        if (rows[e] < 0 || rows[e] >= M || cols[e] < 0 || cols[e] >= N) return -1;
    int use_product = (alpha != 0.0 && K > 0);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t e = 0; e < count; ++e) {
        int64_t i = rows[e], j = cols[e];
        double dot = 0.0;
        if (use_product)
            for (int64_t k = 0; k < K; ++k)
                dot += op_elem(A, is_double, lda, ta, i, k) *
                       op_elem(B, is_double, ldb, tb, k, j);
        double c0 = 0.0;
        if (beta != 0.0)
            c0 = is_double ? ((const double *)C0)[i + j * ldc]
                           : (double)((const float *)C0)[i + j * ldc];
        out[e] = finish(dot, use_product, alpha, beta, c0);
    }
    return 0;
}

/* ---- exported entry points (plain C ABI, host pointers only) ---------- */

/* Whole result: out[i + j*ldo] for 0 <= i < M, 0 <= j < N.  A, B, C0 are
 * FP32 arrays; alpha and beta are the FP32 scalars widened to FP64. */
int oracle_sgemm(char transA, char transB, int64_t M, int64_t N, int64_t K,
                 double alpha, const float *A, int64_t lda,
                 const float *B, int64_t ldb, double beta,
                 const float *C0, int64_t ldc, double *out, int64_t ldo)
{
    return gemm_full(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta,
                     C0, ldc, 0, out, ldo);
}

/* Selected entries: out[e] = C[rows[e], cols[e]], e < count. */
int oracle_sgemm_entries(char transA, char transB, int64_t M, int64_t N, int64_t K,
                         double alpha, const float *A, int64_t lda,
                         const float *B, int64_t ldb, double beta,
                         const float *C0, int64_t ldc, int64_t count,
                         const int64_t *rows, const int64_t *cols, double *out)
{
    return gemm_entries(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta,
                        C0, ldc, 0, count, rows, cols, out);
}

/* The same product with FP64 operands (used for finite differences, where
 * perturbed inputs are not FP32 values).  Products of FP64 values are
 * rounded here, so this form is as accurate as FP64 allows, not exact. */
int oracle_dgemm(char transA, char transB, int64_t M, int64_t N, int64_t K,
                 double alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb, double beta,
                 const double *C0, int64_t ldc, double *out, int64_t ldo)
{
    return gemm_full(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta,
                     C0, ldc, 1, out, ldo);
}

/* Number of threads the parallel loops above use (OpenMP's maximum). */
int oracle_num_threads(void)
{
    return omp_get_max_threads();
}

/* Set that number (n >= 1) for later calls from this thread.  Results do
 * not depend on it: every output is one sequential dot product. */
void oracle_set_num_threads(int n)
{
    omp_set_num_threads(n < 1 ? 1 : n);
}
