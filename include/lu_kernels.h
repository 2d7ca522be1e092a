/*
 * lu_kernels.h -- the individual steps of one LU iteration as callable
 * entry points, for per-kernel testing and micro-benchmarks.  Same
 * conventions as lu.h: device pointers, column-major, asynchronous on
 * `stream`, 0 on success, -i for an illegal argument i, LU_ERR_* otherwise.
 * `prec` selects the element type: LU_FP64 -> double, otherwise float.
 */
#ifndef LU_MI355X_KERNELS_H
#define LU_MI355X_KERNELS_H

#include <hip/hip_runtime_api.h>
#include "lu.h"

#ifdef __cplusplus
extern "C" {
#endif

/* RL1 (Sec. 3.5) on its own: factor the m x w panel P (m >= w >= 1, w <= 512)
 * in place with partial pivoting; ipiv_rel[t] (device int[w]) receives the
 * 0-based panel row interchanged with row t.  Row interchanges are applied
 * to all w panel columns.  `wgs` work-groups cooperate (0 = automatic);
 * d_info (device, may be NULL) receives the first zero pivot, 1-based, if it
 * is still 0.  Errors: -2 m, -3 w, -4 P, -5 ldp, -6 ipiv_rel. */
int lu_k_panel(lu_precision_t prec, int m, int w, void* P, int ldp, int* ipiv_rel,
               int wgs, int* d_info, hipStream_t stream);

/* The trailing-update step for one panel (Sec. 3.4: laswp, trsm, gemm), on
 * the m x ncols block C whose first w rows are the U12 rows:
 *   apply ipiv_rel[0..w) (panel-relative rows, as from lu_k_panel) to the rows
 *   of C; C[0:w,:] := trilu(L11)^-1 C[0:w,:]; C[w:m,:] -= L21 C[0:w,:]
 * where L = [L11; L21] is the m x w factored panel.  Errors: -2 m, -3 w,
 * -4 ncols, -5 L, -6 ldl, -7 ipiv_rel, -8 C, -9 ldc. */
int lu_k_update(lu_precision_t prec, int m, int w, int ncols, const void* L, int ldl,
                const int* ipiv_rel, void* C, int ldc, hipStream_t stream);

/* RL3 alone: C (m x n) -= A (m x k) * B (k x n).  For the mixed precisions A
 * and B are float and are rounded to FP16/BF16 (with power-of-two row / column
 * scales) before the product, which is accumulated in FP32. */
int lu_k_gemm(lu_precision_t prec, int m, int n, int k, const void* A, int lda,
              const void* B, int ldb, void* C, int ldc, hipStream_t stream);

/* Apply the interchanges ipiv_rel[0..w) (relative to row 0) to the m x ncols
 * block C (laswp; m bounds the rows touched).  Errors: -2 m, -3 w, -4 ncols,
 * -5 ipiv_rel, -6 C, -7 ldc. */
int lu_k_laswp(lu_precision_t prec, int m, int w, int ncols, const int* ipiv_rel,
               void* C, int ldc, hipStream_t stream);

/* Timing of the trailing-update GEMM launches of subsequent factorizations
 * (for roofline reporting).  enable = 1 starts recording a pair of timing
 * events around every trailing-update GEMM launch on the stream it runs on
 * (and discards earlier records); enable = 0 stops.  lu_k_timing_read
 * synchronises and returns, over the recorded launches, the summed kernel
 * time in ms, the summed algorithmic flops (2*M*N*K per launch) and the
 * number of launches (host pointers). */
int lu_k_timing(int enable);
int lu_k_timing_read(double* ms, double* flops, int* launches);

/* As lu_k_timing_read for one kind of launch: kind 0 the FP64/FP32 trailing
 * GEMM, kind 1 the FP16/BF16 trailing GEMM of the mixed precisions; bytes
 * (host) receives the summed algorithmic HBM bytes of those launches (kind 1:
 * the FP32 C block read and written, the half operands and scales read once;
 * kind 0: 0).  Errors: -1 kind, -2 ms, -3 flops, -4 bytes, -5 launches. */
int lu_k_timing_read_ex(int kind, double* ms, double* flops, double* bytes, int* launches);

/* Host only (no device call): the moves a trailing kernel takes from a
 * composed interchange list (host int[2 + 4*512]: [0] top count, [1] extra
 * count, top (dst, src) pairs from [2], extra pairs from [2 + 2*512]; rows
 * relative to the panel's first row) of a panel of width w (1..512) in a
 * block of m >= w rows.  The kernels read the list with the same functions:
 * counts clamped to w, a top move kept only if dst in [0, w) and src in
 * [0, m), an extra move only if dst in [w, m) and src in [0, w).  Writes the
 * kept (dst, src) pairs to out (host int[4*512]), top moves first, and
 * returns (kept top << 16) | kept extra.  Errors: -1 moves, -2 w, -3 m,
 * -4 out. */
int lu_k_moves_check(const int* moves, int w, int m, int* out);

/* Host only (no device call): the status lu_solve_ir returns once its FP64
 * solution is settled -- fp64_info is the INFO of the FP64 factorization
 * (0 or the first zero pivot, 1-based), fell_back is 1 when refinement in the
 * working precision was given up, resid the worst-column HPL residual:
 *   fp64_info != 0 -> LU_ERR_SINGULAR;  resid NaN -> LU_ERR_NONFINITE;
 *   resid > 16 -> LU_IR_RESID_HIGH;  else LU_IR_FELL_BACK or LU_IR_OK. */
int lu_ir_outcome(int fp64_info, int fell_back, double resid);

/* Diagnostic: the XCD (hardware register XCC_ID) that each of work-groups
 * 0..63 of one launch runs on, written to out (host int[64]).  Returns 1 if
 * work-group b runs on XCD (b + c) % 8 for one offset c -- the round-robin
 * deal the library's XCD-island schedule relies on (8 P work-groups put P on
 * each XCD), checked once per device when the library first uses it -- 0 if
 * not, or LU_ERR_HIP. */
int lu_k_xcd_probe(int* out);

/* Diagnostic: run one v_mfma_f64_16x16x4f64 on lane-indexed inputs
 * (a = lane, b = 100 + lane, c = 0) and write the 64x4 outputs to out (device
 * double[256], lane-major). */
int lu_k_probe_mfma_f64(double* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LU_MI355X_KERNELS_H */
