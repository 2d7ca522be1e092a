/*
 * chol.h -- Cholesky factorization with look-ahead on one MI355X (gfx950).
 *
 * A = L L^T for a symmetric positive definite A, lower triangle.  Cholesky is
 * one of the factorizations that fit the paper's blocked skeleton (Sec. 3.1:
 * per iteration a panel -- the diagonal block and the column block below it --
 * and a trailing update, here the symmetric rank-b update A22 -= L21 L21^T),
 * and the static look-ahead of Sec. 4 applies to it unchanged; there is no
 * pivoting, so the task list is the LU's without the row interchanges (see
 * lu_plan.h).  FP64 only.
 *
 * Memory and ownership: A is a DEVICE pointer owned by the caller, column
 * major with leading dimension lda >= max(1, n).  Only the lower triangle
 * (i >= j) is read and overwritten with L; the strictly upper triangle is
 * never read or written.
 *
 * Errors: 0 = enqueued; -1 n < 0, -2 A NULL with n > 0, -3 lda < max(1, n),
 * -4 invalid schedule (b not in {32,64,128,256,512}, depth not in {0,1,2},
 * panel_cus > 256); LU_ERR_UNSUPPORTED for n > 65536 (the panel kernel holds
 * at most 1024 rows per compute unit, on at most 64 units); LU_ERR_* (lu.h)
 * for HIP failures, workspace allocation and panel-barrier time-outs.  A matrix that is not positive definite is not
 * an error of the call: as in LAPACK potrf, INFO = j > 0 names the first
 * column whose pivot was not positive (the values from that column on are
 * not a factorization).  INFO goes to d_info (device int, zeroed by the call)
 * when given, else to the library's INFO word, read with lu_factor_info()
 * (lu.h), which synchronizes with the last factorization of either kind.
 *
 * Async: both calls are ordered on `stream` (the factorization runs on the
 * library's update and panel streams, ordered after `stream` on entry and
 * joined back into it on exit) and return without a host synchronization.
 * Not thread-safe per device.
 */
#ifndef LU_MI355X_CHOL_H
#define LU_MI355X_CHOL_H

#include <hip/hip_runtime.h>

#include "lu.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Default schedule: b = 256, look-ahead depth 2, 32 panel CUs. */
int chol_factor(int n, double* A, int lda, hipStream_t stream);

/* sched: fields b, depth, panel_cus as in lu_schedule_t (0 / negative =
 * default); taper is ignored (every panel b wide, the last one ragged). */
int chol_factor_ex(int n, double* A, int lda, const lu_schedule_t* sched, int* d_info, hipStream_t stream);

/* Solve A X = B with the factor of chol_factor (LAPACK potrs, lower):
 * B <- L^-T L^-1 B, nrhs columns, in place.  L and B are DEVICE pointers
 * (column-major, lda, ldb >= max(1, n)); only L's lower triangle is read.
 * Asynchronous on `stream`.  Errors: -1 n < 0, -2 nrhs < 0, -3 L NULL, -4 lda,
 * -5 B NULL, -6 ldb; LU_ERR_* for HIP failures.  A wait between the solve's
 * blocks that times out sets the library's solve error word and leaves B
 * undefined. */
int chol_solve(int n, int nrhs, const double* L, int lda, double* B, int ldb, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LU_MI355X_CHOL_H */
