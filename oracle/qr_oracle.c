/*
 * qr_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU reference for the Householder QR
 * factorization A = Q R of an m x n matrix (m >= n), used by the test-suite
 * only.  Nothing in the product path links, loads or calls this file; it
 * shares no code, header or table with the GPU library.
 *
 * What it computes: QR is one of the factorizations that fit the paper's
 * blocked skeleton (Sec. 3.1); its blocked form factors a panel with
 * Householder reflectors and applies their block form to the trailing
 * matrix, and every blocked variant reaches the result of the plain
 * column-by-column Householder elimination, which is what is written out here
 * (LAPACK geqr2 storage: R on and above the diagonal, the reflector vectors v
 * below it with v_j = 1 implicit, and the scalars tau):
 *
 *   for j = 0 .. n-1
 *     alpha = A[j,j];  s = sum_{i>j} A[i,j]^2   (in row order)
 *     if s == 0:  tau_j = 0                        (H_j = I)
 *     else:
 *       beta  = -sign(alpha) * sqrt(alpha^2 + s)
 *       tau_j = (beta - alpha) / beta
 *       A[i,j] = A[i,j] * (1 / (alpha - beta))   for i > j   (v below the diagonal)
 *       A[j,j] = beta
 *       for c > j:  w = A[j,c] + sum_{i>j} A[i,j] A[i,c]
 *                   A[j,c] = A[j,c] - tau_j w;  A[i,c] = A[i,c] + A[i,j] (-tau_j w)   (i > j)
 *
 * Readings where the paper is silent follow LAPACK geqr2/larfg: the sign of
 * beta is opposite to alpha's (alpha = 0 counts as positive), tau = 0 when the
 * column below the diagonal is zero, v is scaled by a reciprocal.  The norm is
 * the plain square root of the sum of squares (LAPACK rescales to avoid
 * overflow; the test inputs are far from that range).
 *
 * Every floating-point operation is a separately rounded binary64 operation
 * (-O2 -ffp-contract=off); the trailing update may be split over threads by
 * column range with each element's operation order fixed, so the result is
 * bitwise independent of the thread count.
 *
 * Storage: column-major, element (i,j) at A[i + j*lda]; tau has n entries.
 */
#include <math.h>
#include <pthread.h>
#include <stddef.h>
#include <stdlib.h>

#define AT(A, lda, i, j) ((A)[(size_t)(i) + (size_t)(j) * (size_t)(lda)])

typedef struct {
    double *A, *tau;
    int m, n, lda, nthreads, tid;
    pthread_barrier_t *bar;
} qr_worker_t;

static void qr_split(int first, int n, int nthreads, int tid, int *lo, int *hi)
{
    int len = n - first;
    if (len < 0) len = 0;
    int q = len / nthreads, r = len % nthreads;
    int s = first + tid * q + (tid < r ? tid : r);
    *lo = s;
    *hi = s + q + (tid < r ? 1 : 0);
}

static void *qr_worker(void *arg)
{
    qr_worker_t *w = (qr_worker_t *)arg;
    double *A = w->A;
    const int m = w->m, n = w->n, lda = w->lda;
    for (int j = 0; j < n; ++j) {
        /* the reflector of column j: thread 0 only */
        if (w->tid == 0) {
            const double alpha = AT(A, lda, j, j);
            double s = 0.0;
            for (int i = j + 1; i < m; ++i) {
                double x = AT(A, lda, i, j);
                double sq = x * x;
                s = s + sq;
            }
            if (s == 0.0) {
                w->tau[j] = 0.0;
            } else {
                double a2 = alpha * alpha;
                double nrm = sqrt(a2 + s);
                const double beta = alpha >= 0.0 ? -nrm : nrm;
                w->tau[j] = (beta - alpha) / beta;
                const double scal = 1.0 / (alpha - beta);
                for (int i = j + 1; i < m; ++i) AT(A, lda, i, j) = AT(A, lda, i, j) * scal;
                AT(A, lda, j, j) = beta;
            }
        }
        pthread_barrier_wait(w->bar);
        const double tau = w->tau[j];
        if (tau != 0.0) {
            int lo, hi;
            qr_split(j + 1, n, w->nthreads, w->tid, &lo, &hi);
            for (int c = lo; c < hi; ++c) {
                double wc = AT(A, lda, j, c);
                for (int i = j + 1; i < m; ++i) {
                    double p = AT(A, lda, i, j) * AT(A, lda, i, c);
                    wc = wc + p;
                }
                const double t = -tau * wc;
                AT(A, lda, j, c) = AT(A, lda, j, c) + t;
                for (int i = j + 1; i < m; ++i) {
                    double p = AT(A, lda, i, j) * t;
                    AT(A, lda, i, c) = AT(A, lda, i, c) + p;
                }
            }
        }
        pthread_barrier_wait(w->bar);
    }
    return NULL;
}

/*
 * oracle_geqrf: Householder QR of the m x n column-major matrix A (lda >= m,
 * m >= n) in place, tau[0..n) out.  Returns 0, or -1 / -2 / -4 for an illegal
 * m / n / lda.
 */
int oracle_geqrf(int m, int n, double *A, int lda, double *tau, int nthreads)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (n == 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n) nthreads = n;
    pthread_barrier_t bar;
    pthread_barrier_init(&bar, NULL, (unsigned)nthreads);
    qr_worker_t *ws = (qr_worker_t *)calloc((size_t)nthreads, sizeof(qr_worker_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; ++t) {
        ws[t].A = A; ws[t].tau = tau; ws[t].m = m; ws[t].n = n; ws[t].lda = lda;
        ws[t].nthreads = nthreads; ws[t].tid = t; ws[t].bar = &bar;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, qr_worker, &ws[t]);
    qr_worker(&ws[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_barrier_destroy(&bar);
    free(ws);
    free(th);
    return 0;
}
