/*
 * CPU driver for the oracle's GEMM (oracle/ref_gemm.c), built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers_cpu.py.  Every operand is its own heap block of
 * exactly rows * ld floats, so a read one element past a matrix (a wrong
 * stride, a transposed index) aborts the run; the special cases that must
 * not read an operand pass NULL for it.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int ref_gemm(int64_t M, int64_t N, int64_t K, double alpha, const float *A, int64_t lda, const float *B,
             int64_t ldb, double beta, const float *C0, int64_t ldc, double *Cref, double *S, double *T);
int ref_gemm_at(int64_t M, int64_t N, int64_t K, double alpha, const float *A, int64_t lda, const float *B,
                int64_t ldb, double beta, const float *C0, int64_t ldc, int64_t nsamp, const int64_t *rows,
                const int64_t *cols, double *Cref, double *S, double *T);

static uint64_t state = 88172645463325252ull;
static uint64_t next(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
}

static float *matrix(int64_t rows, int64_t ld)
{
    size_t n = (size_t)(rows * ld);
    float *p = malloc(n ? n * sizeof(float) : 1);
    for (size_t i = 0; i < n; ++i) p[i] = (float)((int64_t)(next() % 17) - 8);
    return p;
}

static int failures = 0;

int main(void)
{
    for (int trial = 0; trial < 300; ++trial) {
        int64_t M = (int64_t)(next() % 40), N = (int64_t)(next() % 40), K = (int64_t)(next() % 40);
        int64_t lda = K + (int64_t)(next() % 3), ldb = N + (int64_t)(next() % 3), ldc = N + (int64_t)(next() % 3);
        if (lda < 1) lda = 1;
        if (ldb < 1) ldb = 1;
        if (ldc < 1) ldc = 1;
        const double alphas[] = {1.0, 0.0, -1.5}, betas[] = {0.0, 1.0, 0.5};
        double alpha = alphas[next() % 3], beta = betas[next() % 3];
        int use_ab = alpha != 0.0 && K > 0;
        float *A = use_ab ? matrix(M, lda) : NULL;
        float *B = use_ab ? matrix(K, ldb) : NULL;
        float *C0 = beta != 0.0 ? matrix(M, ldc) : NULL;
        size_t mn = (size_t)(M * N);
        double *Cr = malloc(mn ? mn * sizeof(double) : 1), *S = malloc(mn ? mn * sizeof(double) : 1),
               *T = malloc(mn ? mn * sizeof(double) : 1);
        if (ref_gemm(M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc, Cr, S, T) != 0) {
            fprintf(stderr, "ref_gemm refused a valid problem %lldx%lldx%lld\n", (long long)M, (long long)N,
                    (long long)K);
            ++failures;
        }
        /* Integer data: the full and the sampled results agree exactly. */
        if (M > 0 && N > 0) {
            int64_t rows[5], cols[5];
            double c2[5], s2[5], t2[5];
            for (int p = 0; p < 5; ++p) {
                rows[p] = (int64_t)(next() % (uint64_t)M);
                cols[p] = (int64_t)(next() % (uint64_t)N);
            }
            if (ref_gemm_at(M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc, 5, rows, cols, c2, s2, t2) != 0) {
                ++failures;
            } else {
                for (int p = 0; p < 5; ++p)
                    if (c2[p] != Cr[rows[p] * N + cols[p]] || t2[p] != T[rows[p] * N + cols[p]]) ++failures;
            }
            /* An out-of-range sample position is refused, never read. */
            int64_t bad = M;
            if (ref_gemm_at(M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc, 1, &bad, cols, c2, s2, t2) != -1)
                ++failures;
        }
        free(A);
        free(B);
        free(C0);
        free(Cr);
        free(S);
        free(T);
    }
    /* Invalid arguments are refused. */
    double d;
    if (ref_gemm(-1, 1, 1, 1.0, NULL, 1, NULL, 1, 0.0, NULL, 1, &d, &d, &d) != -1) ++failures;
    if (ref_gemm(2, 2, 2, 1.0, NULL, 2, NULL, 2, 0.0, NULL, 2, &d, &d, &d) != -1) ++failures;
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
