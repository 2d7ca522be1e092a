/*
 * lu_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU reference for LU factorization with
 * partial pivoting (P*A = L*U), used by the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark.  Nothing in the product path links,
 * loads or calls this file; it shares no code, header or table with the GPU
 * library.
 *
 * What it computes (paper: Sec. 3.4, the description of LAPACK getrf as
 * getf2 -> laswp -> trsm -> gemm; Sec. 3.5, operations RL1-RL3 of LU_blk):
 * the blocked algorithm reaches exactly the result of ordinary Gaussian
 * elimination with partial pivoting, so the oracle is that elimination
 * written out, one column at a time (the unblocked getf2 applied to the whole
 * matrix, with each row interchange applied to every column at once):
 *
 *   for k = 0 .. n-1
 *     p = the smallest row index i >= k maximising |A[i,k]|
 *     ipiv[k] = p
 *     if A[p,k] != 0:  swap rows k and p (all n columns);
 *                      A[i,k] = A[i,k] / A[k,k]            for i > k
 *     else if info == 0: info = k+1      (no swap, no scaling)
 *     A[i,j] = A[i,j] - A[i,k]*A[k,j]    for i > k, j > k
 *
 * Readings where the paper is silent (row-interchange tie-break, zero pivot,
 * division vs reciprocal) follow LAPACK getf2 conventions: first index on
 * ties, info = first zero-pivot column (1-based), true IEEE division.
 *
 * Every floating-point operation is a separately rounded IEEE-754 binary64
 * multiply, subtract or divide: compile with -O2 -ffp-contract=off.  The
 * rank-1 update may be split over threads by column range; each element sees
 * the same sequence of operations whatever the split, so the result is
 * bitwise independent of the thread count.
 *
 * Storage: column-major, element (i,j) at A[i + j*lda]; ipiv is 0-based.
 */
#include <math.h>
#include <pthread.h>
#include <stddef.h>
#include <stdlib.h>

#define AT(A, lda, i, j) ((A)[(size_t)(i) + (size_t)(j) * (size_t)(lda)])

typedef struct {
    double *A;
    int n, lda, nthreads, tid;
    int *ipiv;
    int *info;
    pthread_barrier_t *bar;
} worker_t;

/* Columns [lo, hi) of the range [first, n) owned by thread tid. */
static void split(int first, int n, int nthreads, int tid, int *lo, int *hi)
{
    int len = n - first;
    if (len < 0) len = 0;
    int q = len / nthreads, r = len % nthreads;
    int s = first + tid * q + (tid < r ? tid : r);
    *lo = s;
    *hi = s + q + (tid < r ? 1 : 0);
}

static void *worker(void *arg)
{
    worker_t *w = (worker_t *)arg;
    double *A = w->A;
    const int n = w->n, lda = w->lda;
    for (int k = 0; k < n; ++k) {
        /* pivot search + bookkeeping: thread 0 only */
        if (w->tid == 0) {
            int p = k;
            double best = fabs(AT(A, lda, k, k));
            for (int i = k + 1; i < n; ++i) {
                double v = fabs(AT(A, lda, i, k));
                if (v > best) { best = v; p = i; }   /* strict: first index wins ties */
            }
            w->ipiv[k] = p;
            if (AT(A, lda, p, k) == 0.0 && *w->info == 0) *w->info = k + 1;
        }
        pthread_barrier_wait(w->bar);
        const int p = w->ipiv[k];
        const int nonzero = AT(A, lda, p, k) != 0.0;
        /* row interchange over all columns, split by column */
        if (nonzero && p != k) {
            int lo, hi;
            split(0, n, w->nthreads, w->tid, &lo, &hi);
            for (int j = lo; j < hi; ++j) {
                double t = AT(A, lda, k, j);
                AT(A, lda, k, j) = AT(A, lda, p, j);
                AT(A, lda, p, j) = t;
            }
        }
        pthread_barrier_wait(w->bar);
        /* scale the sub-column by the pivot (thread 0) */
        if (w->tid == 0 && nonzero) {
            const double piv = AT(A, lda, k, k);
            for (int i = k + 1; i < n; ++i) AT(A, lda, i, k) = AT(A, lda, i, k) / piv;
        }
        pthread_barrier_wait(w->bar);
        /* rank-1 update of the trailing matrix, split by column */
        {
            int lo, hi;
            split(k + 1, n, w->nthreads, w->tid, &lo, &hi);
            for (int j = lo; j < hi; ++j) {
                const double ukj = AT(A, lda, k, j);
                double *col = &AT(A, lda, 0, j);
                const double *lk = &AT(A, lda, 0, k);
                for (int i = k + 1; i < n; ++i) {
                    double prod = lk[i] * ukj;
                    col[i] = col[i] - prod;
                }
            }
        }
        pthread_barrier_wait(w->bar);
    }
    return NULL;
}

/*
 * oracle_getrf: factor the n x n column-major matrix A (leading dimension lda)
 * in place.  Returns LAPACK-style info: 0, or k+1 for the first column k whose
 * pivot was exactly zero, or -1 / -3 for an illegal n / lda.
 */
int oracle_getrf(int n, double *A, int lda, int *ipiv, int nthreads)
{
    if (n < 0) return -1;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (n == 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n) nthreads = n;
    int info = 0;
    pthread_barrier_t bar;
    pthread_barrier_init(&bar, NULL, (unsigned)nthreads);
    worker_t *ws = (worker_t *)calloc((size_t)nthreads, sizeof(worker_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; ++t) {
        ws[t].A = A; ws[t].n = n; ws[t].lda = lda; ws[t].nthreads = nthreads;
        ws[t].tid = t; ws[t].ipiv = ipiv; ws[t].info = &info; ws[t].bar = &bar;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, &ws[t]);
    worker(&ws[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_barrier_destroy(&bar);
    free(ws);
    free(th);
    return info;
}

/*
 * oracle_getrs: solve A*X = B given the factors from oracle_getrf
 * (LAPACK getrs semantics, no transpose).  B is n x nrhs column-major with
 * leading dimension ldb and is overwritten by X.
 *   1. apply the interchanges in order: swap B[k,:] and B[ipiv[k],:]
 *   2. forward substitution with the unit lower factor L
 *   3. back substitution with the upper factor U
 */
int oracle_getrs(int n, int nrhs, const double *LU, int lda, const int *ipiv,
                 double *B, int ldb)
{
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (ldb < (n > 1 ? n : 1)) return -7;
    for (int c = 0; c < nrhs; ++c) {
        double *b = &AT(B, ldb, 0, c);
        for (int k = 0; k < n; ++k) {
            int p = ipiv[k];
            if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
        }
        for (int j = 0; j < n; ++j) {              /* L y = Pb, column oriented */
            const double yj = b[j];
            for (int i = j + 1; i < n; ++i) {
                double prod = AT(LU, lda, i, j) * yj;
                b[i] = b[i] - prod;
            }
        }
        for (int j = n - 1; j >= 0; --j) {         /* U x = y, column oriented */
            b[j] = b[j] / AT(LU, lda, j, j);
            const double xj = b[j];
            for (int i = 0; i < j; ++i) {
                double prod = AT(LU, lda, i, j) * xj;
                b[i] = b[i] - prod;
            }
        }
    }
    return 0;
}
