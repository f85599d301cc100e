/*
 * Reference oracle for the single-precision GEMM -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file's library.  The product path never links, calls
 * or falls back to it, and it shares no code, header or constant with the
 * HIP kernels or the C-ABI runtime.
 *
 * What it computes is the plain definition of the operation the paper tunes
 * (title and Sec. V-C: SGEMM, results screened against reference kernels):
 *
 *     S[i][j]    = sum_{k<K} A[i][k] * B[k][j]          (FP64)
 *     T[i][j]    = sum_{k<K} |A[i][k]| * |B[k][j]|      (FP64, for error bounds)
 *     Cref[i][j] = alpha * S[i][j] + beta * C0[i][j]    (FP64)
 *
 * with A (M x K, row stride lda), B (K x N, row stride ldb), C0 (M x N, row
 * stride ldc), all row-major FP32.  Outputs are dense row-major M x N FP64.
 *
 * Reference-BLAS special cases are part of the definition:
 *   - alpha == 0 or K == 0: A and B are not read; S = T = 0; Cref = beta*C0.
 *   - beta == 0: C0 is not read (NaN in C0 must not reach Cref).
 *
 * The product of two FP32 numbers is exact in FP64 (24+24 <= 53 significand
 * bits), so every term is exact; only the FP64 summation rounds, with error
 * at most K * 2^-53 * T[i][j].
 *
 * Loop order: for each row i the k loop is outermost and the j loop inner,
 * accumulating into the output row.  Every element's sum is still formed in
 * ascending k order, exactly as in the textbook i-j-k form; only the memory
 * access order differs.  Rows are independent, so they may run on several
 * OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int ref_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Returns 0 on success, -1 on invalid sizes/strides/pointers. */
int ref_gemm(int64_t M, int64_t N, int64_t K, double alpha,
             const float *A, int64_t lda, const float *B, int64_t ldb,
             double beta, const float *C0, int64_t ldc,
             double *Cref, double *S, double *T)
{
    if (M < 0 || N < 0 || K < 0) return -1;
    if (M == 0 || N == 0) return 0;
    if (Cref == NULL || S == NULL || T == NULL) return -1;
    int use_ab = (alpha != 0.0 && K > 0);
    if (use_ab && (A == NULL || B == NULL || lda < K || ldb < N)) return -1;
    if (beta != 0.0 && (C0 == NULL || ldc < N)) return -1;

    int64_t i;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (i = 0; i < M; ++i) {
        double *s = S + i * N;
        double *t = T + i * N;
        double *c = Cref + i * N;
        for (int64_t j = 0; j < N; ++j) { s[j] = 0.0; t[j] = 0.0; }
        if (use_ab) {
            for (int64_t k = 0; k < K; ++k) {
                double a = (double)A[i * lda + k];
                double aa = fabs(a);
                const float *brow = B + k * ldb;
                for (int64_t j = 0; j < N; ++j) {
                    double b = (double)brow[j];
                    s[j] += a * b;
                    t[j] += aa * fabs(b);
                }
            }
        }
        for (int64_t j = 0; j < N; ++j) {
            double v = use_ab ? alpha * s[j] : 0.0;
            if (beta != 0.0) v += beta * (double)C0[i * ldc + j];
            c[j] = v;
        }
    }
    return 0;
}

/*
 * Same definition evaluated only at nsamp given (row, col) positions, for
 * checking sampled outputs of problems too large for the full oracle.
 * Outputs are arrays of length nsamp.
 */
int ref_gemm_at(int64_t M, int64_t N, int64_t K, double alpha,
                const float *A, int64_t lda, const float *B, int64_t ldb,
                double beta, const float *C0, int64_t ldc,
                int64_t nsamp, const int64_t *rows, const int64_t *cols,
                double *Cref, double *S, double *T)
{
    if (M < 0 || N < 0 || K < 0 || nsamp < 0) return -1;
    int use_ab = (alpha != 0.0 && K > 0);
    if (use_ab && (A == NULL || B == NULL || lda < K || ldb < N)) return -1;
    if (beta != 0.0 && (C0 == NULL || ldc < N)) return -1;
    for (int64_t p = 0; p < nsamp; ++p)
        if (rows[p] < 0 || rows[p] >= M || cols[p] < 0 || cols[p] >= N) return -1;

    int64_t p;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (p = 0; p < nsamp; ++p) {
        int64_t i = rows[p], j = cols[p];
        double s = 0.0, t = 0.0;
        if (use_ab) {
            for (int64_t k = 0; k < K; ++k) {
                double a = (double)A[i * lda + k];
                double b = (double)B[k * ldb + j];
                s += a * b;
                t += fabs(a) * fabs(b);
            }
        }
        double v = use_ab ? alpha * s : 0.0;
        if (beta != 0.0) v += beta * (double)C0[i * ldc + j];
        Cref[p] = v;
        S[p] = s;
        T[p] = t;
    }
    return 0;
}
