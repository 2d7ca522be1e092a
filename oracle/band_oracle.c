/*
 * band_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU reference for the two-sided reduction
 * of a square matrix to upper band form, the first stage of a two-stage SVD
 * (the third workload of the paper's evaluation, Sec. 6: per iteration a
 * panel of w columns is factored with Householder reflectors applied from the
 * left, then a panel of w rows with reflectors applied from the right, and
 * the trailing matrix is updated by both).  Used by the test-suite only:
 * nothing in the product path links, loads or calls this file, and it shares
 * no code, header or table with the GPU library.
 *
 * What it computes, one reflector at a time (every blocked variant reaches
 * the same result up to rounding):
 *
 *   for k = 0, w, 2w, ... < n:               kw = min(w, n - k)
 *     for j = k .. k+kw-1:                   (column panel, left reflectors)
 *       H_j from A[j:n, j] (beta on the diagonal, v below it, tauq[j]);
 *       A[j:n, j+1:n] = H_j A[j:n, j+1:n]
 *     for i = 0 .. kw-1 with c = k + w + i < n:   (row panel, right reflectors)
 *       G_r from A[r, c:n], r = k + i (beta at A[r, c], v right of it, taup[r]);
 *       A[r+1:n, c:n] = A[r+1:n, c:n] G_r
 *
 * so that B = U^T A V with U = H_0 H_1 ..., V = G_0 G_1 ... is upper banded:
 * B[i, j] = 0 unless 0 <= j - i <= w.  The band sits on and above the
 * diagonal, the column reflectors below the diagonal (geqrf storage) and the
 * row reflectors of row r from column k + w + i + 1 on (gelqf storage, shifted
 * by the bandwidth); taup[r] = 0 for rows without a reflector.
 *
 * Each reflector follows LAPACK larfg, as in the QR oracle: for x = (alpha,
 * x_2 ..), s = sum x_i^2 over i >= 2 in index order; s == 0 gives tau = 0
 * (G = I); otherwise beta = -sign(alpha) sqrt(alpha^2 + s) (alpha = 0 counts
 * as positive), tau = (beta - alpha) / beta, v_i = x_i * (1 / (alpha - beta)).
 * Applying I - tau v v^T to a vector y: d = y_1 + sum_{i>=2} v_i y_i (index
 * order), t = -tau d, y_1 += t, y_i += v_i t.
 *
 * Every floating-point operation is a separately rounded binary64 operation
 * (-O2 -ffp-contract=off).  Single-threaded.
 *
 * Storage: column-major, element (i,j) at A[i + j*lda].
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>

#define AT(A, lda, i, j) ((A)[(size_t)(i) + (size_t)(j) * (size_t)(lda)])

/* The reflector of x[0], x[inc], ..., x[(len-1)*inc]: x[0] <- beta, the rest
 * <- v (v_0 = 1 implicit).  Returns tau. */
static double band_house(double *x, int len, size_t inc)
{
    const double alpha = x[0];
    double s = 0.0;
    for (int i = 1; i < len; ++i) {
        double y = x[(size_t)i * inc];
        double sq = y * y;
        s = s + sq;
    }
    if (s == 0.0) return 0.0;
    double a2 = alpha * alpha;
    double nrm = sqrt(a2 + s);
    const double beta = alpha >= 0.0 ? -nrm : nrm;
    const double tau = (beta - alpha) / beta;
    const double scal = 1.0 / (alpha - beta);
    for (int i = 1; i < len; ++i) x[(size_t)i * inc] = x[(size_t)i * inc] * scal;
    x[0] = beta;
    return tau;
}

/* Columns j+1 .. n-1, rows j .. n-1: y <- (I - tau v v^T) y with v in column j. */
static void band_left(double *A, int lda, int n, int j, double tau)
{
    for (int c = j + 1; c < n; ++c) {
        double d = AT(A, lda, j, c);
        for (int i = j + 1; i < n; ++i) {
            double p = AT(A, lda, i, j) * AT(A, lda, i, c);
            d = d + p;
        }
        const double t = -tau * d;
        AT(A, lda, j, c) = AT(A, lda, j, c) + t;
        for (int i = j + 1; i < n; ++i) {
            double p = AT(A, lda, i, j) * t;
            AT(A, lda, i, c) = AT(A, lda, i, c) + p;
        }
    }
}

/* Rows r+1 .. n-1, columns c .. n-1: y^T <- y^T (I - tau v v^T) with v in row r
 * from column c on.  The dot products of all rows are formed column by column
 * (each row's sum still runs in column order). */
static void band_right(double *A, int lda, int n, int r, int c, double tau, double *d)
{
    for (int q = r + 1; q < n; ++q) d[q] = AT(A, lda, q, c);
    for (int t = c + 1; t < n; ++t) {
        const double v = AT(A, lda, r, t);
        for (int q = r + 1; q < n; ++q) {
            double p = AT(A, lda, q, t) * v;
            d[q] = d[q] + p;
        }
    }
    for (int q = r + 1; q < n; ++q) d[q] = -tau * d[q];
    for (int q = r + 1; q < n; ++q) AT(A, lda, q, c) = AT(A, lda, q, c) + d[q];
    for (int t = c + 1; t < n; ++t) {
        const double v = AT(A, lda, r, t);
        for (int q = r + 1; q < n; ++q) {
            double p = v * d[q];
            AT(A, lda, q, t) = AT(A, lda, q, t) + p;
        }
    }
}

/*
 * oracle_gebrd_band: reduce the n x n column-major matrix A (lda >= n) to
 * upper band form with bandwidth w in place; tauq[0..n), taup[0..n) out.
 * Returns 0, or -1 / -2 / -4 for an illegal n / w / lda.
 */
int oracle_gebrd_band(int n, int w, double *A, int lda, double *tauq, double *taup)
{
    if (n < 0) return -1;
    if (w < 1) return -2;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (n == 0) return 0;
    double *d = (double *)malloc((size_t)n * sizeof(double));
    if (!d) return -100;
    for (int i = 0; i < n; ++i) taup[i] = 0.0;
    for (int k = 0; k < n; k += w) {
        const int kw = w < n - k ? w : n - k;
        for (int j = k; j < k + kw; ++j) {
            tauq[j] = band_house(&AT(A, lda, j, j), n - j, 1);
            if (tauq[j] != 0.0) band_left(A, lda, n, j, tauq[j]);
        }
        for (int i = 0; i < kw && k + w + i < n; ++i) {
            const int r = k + i, c = k + w + i;
            taup[r] = band_house(&AT(A, lda, r, c), n - c, (size_t)lda);
            if (taup[r] != 0.0) band_right(A, lda, n, r, c, taup[r], d);
        }
    }
    free(d);
    return 0;
}
