/*
 * band.h -- two-sided reduction of a square matrix to upper band form on one
 * MI355X (gfx950): the first stage of a two-stage SVD, the third workload of
 * the paper's evaluation (Sec. 6; its flop count 8n^3/3 is that of the full
 * reduction to bidiagonal form).
 *
 * B = U^T A V with U = H_0 H_1 ... H_{n-1} (column reflectors) and
 * V = G_0 G_1 ... (row reflectors), B upper banded: B[i][j] = 0 unless
 * 0 <= j - i <= w.  Per iteration k = 0, w, 2w, ...: Householder QR of the
 * column panel A[k:n, k:k+w] applied from the left to the columns right of
 * it, then Householder LQ of the row panel A[k:k+w, k+w:n] applied from the
 * right to the rows below it; each trailing update is a block-reflector
 * product on the MFMA GEMM kernel.
 *
 * Storage on return (column major, element (i,j) at A[i + j*lda]):
 *   - the band B on and above the diagonal (entries with 0 <= j - i <= w);
 *   - column reflector j below the diagonal (v_j[j] = 1 implicit), tauq[j];
 *   - row reflector of row r = k + i (k a multiple of w, i < w) in row r from
 *     column k + w + i + 1 on (v[k + w + i] = 1 implicit), taup[r]; rows whose
 *     segment k + w + i .. n-1 is empty have taup[r] = 0.
 * Every reflector follows LAPACK larfg (beta = -sign(alpha) * norm, tau = 0
 * when the part below / right of alpha is zero).
 *
 * Memory and ownership: A, tauq and taup are DEVICE pointers owned by the
 * caller (tauq, taup: n doubles each); lda >= max(1, n).  The library keeps
 * workspace (the transposed row panel, explicit V and V^T, T, the products'
 * buffers: about (7 + ceil(n / 2048)) n w doubles, plus (1 + ceil(w / 128)) n 128
 * doubles for the sub-panels of a panel wider than 128) cached per device;
 * lu_release frees it.
 *
 * Errors: 0 = enqueued; -1 n < 0, -2 A NULL, -3 lda < max(1, n), -4 w < 1 or
 * w > 384, -5 tauq NULL, -6 taup NULL; LU_ERR_UNSUPPORTED for n > 65536 (the
 * panel kernel holds at most 1024 rows per work-group on at most 64 compute units);
 * LU_ERR_* (lu.h) for HIP failures, workspace and panel-barrier time-outs
 * (lu_factor_info reports the latter).
 *
 * Async: ordered on `stream` (the reduction runs on the library's update
 * stream, the column panels factored ahead on its panel stream, both ordered
 * after `stream` on entry and joined back into it on exit) and returns without
 * a host synchronization.  Not thread-safe per device.
 */
#ifndef LU_MI355X_BAND_H
#define LU_MI355X_BAND_H

#include <hip/hip_runtime.h>

#include "lu.h"

#ifdef __cplusplus
extern "C" {
#endif

int band_reduce(int n, double* A, int lda, int w, double* tauq, double* taup, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LU_MI355X_BAND_H */
