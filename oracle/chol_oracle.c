/*
 * chol_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU reference for the Cholesky factorization
 * A = L * L^T of a symmetric positive definite matrix (lower triangle), used
 * by the test-suite only.  Nothing in the product path links, loads or calls
 * this file; it shares no code, header or table with the GPU library.
 *
 * What it computes: Cholesky is one of the factorizations that fit the
 * paper's general blocked skeleton (Sec. 3.1) -- its blocked form factors a
 * diagonal block, solves for the column block below it and updates the
 * trailing matrix -- and every blocked variant reaches the result of the
 * plain column-by-column elimination, which is what is written out here
 * (the unblocked potf2 form, right-looking, lower triangle):
 *
 *   for k = 0 .. n-1
 *     d = A[k,k]
 *     if not (d > 0):  info = k+1, stop             (not positive definite)
 *     A[k,k] = sqrt(d)
 *     A[i,k] = A[i,k] / A[k,k]                       for i > k
 *     A[i,j] = A[i,j] - A[i,k]*A[j,k]                for j > k, i >= j
 *
 * Only the lower triangle (i >= j) is read or written; the strictly upper
 * triangle is left untouched.  Readings where the paper is silent follow
 * LAPACK potf2: a non-positive (or NaN) pivot stops the factorization with
 * info = its 1-based column; true IEEE division and square root.
 *
 * Every floating-point operation is a separately rounded binary64 multiply,
 * subtract, divide or square root (-O2 -ffp-contract=off).  The trailing
 * update may be split over threads by column range; each element sees the
 * same sequence of operations whatever the split, so the result is bitwise
 * independent of the thread count.
 *
 * Storage: column-major, element (i,j) at A[i + j*lda].
 */
#include <math.h>
#include <pthread.h>
#include <stddef.h>
#include <stdlib.h>

#define AT(A, lda, i, j) ((A)[(size_t)(i) + (size_t)(j) * (size_t)(lda)])

typedef struct {
    double *A;
    int n, lda, nthreads, tid;
    int *stop;
    pthread_barrier_t *bar;
} chol_worker_t;

static void chol_split(int first, int n, int nthreads, int tid, int *lo, int *hi)
{
    int len = n - first;
    if (len < 0) len = 0;
    int q = len / nthreads, r = len % nthreads;
    int s = first + tid * q + (tid < r ? tid : r);
    *lo = s;
    *hi = s + q + (tid < r ? 1 : 0);
}

static void *chol_worker(void *arg)
{
    chol_worker_t *w = (chol_worker_t *)arg;
    double *A = w->A;
    const int n = w->n, lda = w->lda;
    for (int k = 0; k < n; ++k) {
        /* pivot, square root and column scaling: thread 0 only */
        if (w->tid == 0) {
            const double d = AT(A, lda, k, k);
            if (!(d > 0.0)) {
                *w->stop = k + 1;
            } else {
                const double r = sqrt(d);
                AT(A, lda, k, k) = r;
                for (int i = k + 1; i < n; ++i) AT(A, lda, i, k) = AT(A, lda, i, k) / r;
            }
        }
        pthread_barrier_wait(w->bar);
        if (*w->stop) break;
        /* symmetric rank-1 update of the lower trailing triangle, split by column */
        {
            int lo, hi;
            chol_split(k + 1, n, w->nthreads, w->tid, &lo, &hi);
            for (int j = lo; j < hi; ++j) {
                const double ljk = AT(A, lda, j, k);
                double *col = &AT(A, lda, 0, j);
                const double *lk = &AT(A, lda, 0, k);
                for (int i = j; i < n; ++i) {
                    double prod = lk[i] * ljk;
                    col[i] = col[i] - prod;
                }
            }
        }
        pthread_barrier_wait(w->bar);
    }
    return NULL;
}

/*
 * oracle_potrf: factor the lower triangle of the n x n column-major SPD matrix
 * A (leading dimension lda) in place.  Returns 0, or k+1 for the first column
 * k whose pivot was not positive (the factorization stops there), or -1 / -3
 * for an illegal n / lda.
 */
int oracle_potrf(int n, double *A, int lda, int nthreads)
{
    if (n < 0) return -1;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (n == 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n) nthreads = n;
    int stop = 0;
    pthread_barrier_t bar;
    pthread_barrier_init(&bar, NULL, (unsigned)nthreads);
    chol_worker_t *ws = (chol_worker_t *)calloc((size_t)nthreads, sizeof(chol_worker_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; ++t) {
        ws[t].A = A; ws[t].n = n; ws[t].lda = lda; ws[t].nthreads = nthreads; ws[t].tid = t;
        ws[t].stop = &stop; ws[t].bar = &bar;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, chol_worker, &ws[t]);
    chol_worker(&ws[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_barrier_destroy(&bar);
    free(ws);
    free(th);
    return stop;
}
