/*
 * qr.h -- Householder QR factorization with look-ahead on one MI355X (gfx950).
 *
 * A = Q R for an m x n matrix (m >= n), FP64, LAPACK geqrf storage: R on and
 * above the diagonal, the Householder vectors v_j below it (v_j has an
 * implicit 1 at row j), tau[j] the reflector scalars, Q = H_0 H_1 ... H_{n-1},
 * H_j = I - tau_j v_j v_j^T.  QR is one of the factorizations of the paper's
 * blocked skeleton (Sec. 3.1): per iteration a panel is factored with
 * Householder reflectors, and their block form I - V T V^T (T upper
 * triangular, LAPACK larft) is applied to the trailing matrix; the static
 * look-ahead of Sec. 4 overlaps the next panels with that update exactly as
 * for the LU (the task list of lu_plan.h without the interchanges).
 *
 * Memory and ownership: A and tau are DEVICE pointers owned by the caller;
 * A is column major with lda >= max(1, m); tau has n entries.  The library
 * keeps workspace (explicit V and V^T of four panels, the T factors, two
 * update buffers of b x n) cached per device; lu_release frees it.
 *
 * Errors: 0 = enqueued; -1 m < 0, -2 n < 0 or n > m, -3 A NULL, -4 lda,
 * -5 tau NULL, -6 invalid schedule (b not in {32,64,128,256}, depth not in
 * {0,1,2}, panel_cus > 256); LU_ERR_UNSUPPORTED for m > 65536 (the panel
 * kernel holds at most 1024 rows per work-group on at most 64 compute units);
 * LU_ERR_* (lu.h) for HIP failures, workspace and panel-barrier time-outs
 * (lu_factor_info reports the latter).
 *
 * Async: ordered on `stream` (the factorization runs on the library's update
 * and panel streams, ordered after `stream` on entry and joined back into it
 * on exit) and returns without a host synchronization.
 * Not thread-safe per device.
 */
#ifndef LU_MI355X_QR_H
#define LU_MI355X_QR_H

#include <hip/hip_runtime.h>

#include "lu.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Default schedule: b = 128, look-ahead depth 2.  The panel kernel runs
 * ceil(m_k / 1024) work-groups for a panel of m_k rows, so the summation
 * order inside a panel, and with it the result, is the same for every
 * schedule at a given b. */
int qr_factor(int m, int n, double* A, int lda, double* tau, hipStream_t stream);

/* sched: b and depth as in lu_schedule_t (0 / negative = default);
 * panel_cus is range-checked only (the panel's group count follows from its
 * height), taper is ignored. */
int qr_factor_ex(int m, int n, double* A, int lda, double* tau, const lu_schedule_t* sched, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LU_MI355X_QR_H */
