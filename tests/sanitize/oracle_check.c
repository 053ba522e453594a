/*
 * oracle_check.c -- runs the FP64 oracle (oracle/oracle.c, linked in) on
 * one product read from a file, with every operand in a heap block of
 * exactly its referenced extent, so that AddressSanitizer reports any read
 * outside it and UndefinedBehaviorSanitizer any undefined operation.  Built
 * and run by tests/test_host_sanitized.py (test infrastructure checking
 * test infrastructure).
 *
 * Input file: one text line
 *     ta tb M N K alpha beta lda ldb ldc count a_refd b_refd c_refd
 * then, as raw little-endian data, the referenced extent of A, of B and of
 * C0 as FP32 (each only when its *_refd flag is 1; an unreferenced operand
 * is passed as NULL), then count row and count column indices as int64.
 * Output file: the M x N result (FP64, column-major, ld max(1, M)), then the
 * count sampled entries, then the same product with FP64 operands
 * (oracle_dgemm on the widened inputs).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_sgemm(char, char, int64_t, int64_t, int64_t, double, const float *, int64_t,
                 const float *, int64_t, double, const float *, int64_t, double *, int64_t);
int oracle_sgemm_entries(char, char, int64_t, int64_t, int64_t, double, const float *,
                         int64_t, const float *, int64_t, double, const float *, int64_t,
                         int64_t, const int64_t *, const int64_t *, double *);
int oracle_dgemm(char, char, int64_t, int64_t, int64_t, double, const double *, int64_t,
                 const double *, int64_t, double, const double *, int64_t, double *, int64_t);

static void *take(FILE *f, size_t n, size_t size)
{
    void *p = malloc(n ? n * size : 1);
    if (!p || fread(p, size, n, f) != n) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

static double *widen(const float *x, size_t n)
{
    if (!x) return NULL;
    double *d = malloc(n ? n * sizeof(double) : 1);
    for (size_t i = 0; i < n; ++i) d[i] = x[i];
    return d;
}

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    char ta, tb;
    long long M, N, K, lda, ldb, ldc, count, na, nb, nc;
    double alpha, beta;
    int ra, rb, rc;
    if (fscanf(f, " %c %c %lld %lld %lld %lf %lf %lld %lld %lld %lld %d %d %d", &ta, &tb, &M,
               &N, &K, &alpha, &beta, &lda, &ldb, &ldc, &count, &ra, &rb, &rc) != 14)
        return 2;
    if (fgetc(f) != '\n') return 2;
    if (fscanf(f, "%lld %lld %lld", &na, &nb, &nc) != 3 || fgetc(f) != '\n') return 2;
    float *A = ra ? take(f, (size_t)na, sizeof(float)) : NULL;
    float *B = rb ? take(f, (size_t)nb, sizeof(float)) : NULL;
    float *C = rc ? take(f, (size_t)nc, sizeof(float)) : NULL;
    int64_t *rows = take(f, (size_t)count, sizeof(int64_t));
    int64_t *cols = take(f, (size_t)count, sizeof(int64_t));
    fclose(f);

    const long long ldo = M > 1 ? M : 1;
    const size_t nout = (size_t)ldo * (size_t)(N > 0 ? N : 0);
    double *out = malloc(nout ? nout * sizeof(double) : 1);
    double *ent = malloc(count ? (size_t)count * sizeof(double) : 1);
    double *dout = malloc(nout ? nout * sizeof(double) : 1);
    double *Ad = widen(A, (size_t)na), *Bd = widen(B, (size_t)nb), *Cd = widen(C, (size_t)nc);
    int st = oracle_sgemm(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, out, ldo);
    if (st == 0)
        st = oracle_sgemm_entries(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, count,
                                  rows, cols, ent);
    if (st == 0)
        st = oracle_dgemm(ta, tb, M, N, K, alpha, Ad, lda, Bd, ldb, beta, Cd, ldc, dout, ldo);
    if (st != 0) {
        fprintf(stderr, "oracle status %d\n", st);
        return 3;
    }
    FILE *o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(out, sizeof(double), nout, o);
    fwrite(ent, sizeof(double), (size_t)count, o);
    fwrite(dout, sizeof(double), nout, o);
    fclose(o);
    free(A); free(B); free(C); free(Ad); free(Bd); free(Cd);
    free(rows); free(cols); free(out); free(ent); free(dout);
    return 0;
}
